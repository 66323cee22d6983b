// adjoint.hip -- vector-Jacobian products of the ZHS and Endpoint traces.
//
// For a scalar loss with upstream gradient G = dL/dA over the traces
// [M][B][3], the share of one (track, antenna) pair is
//     L_p = sum_c I_c / dt * gbar_c,
//     gbar_c = (Phi_c(u_hi) - Phi_c(u_lo)) / (u_hi - u_lo)   (or G_c at the bin
//                                                         when both ends share it)
// where I = k qw beta_perp (t1 - t0) / R_mid is the box's time integral, u_lo
// and u_hi its edges in bins, and Phi_c the integral of the piecewise-constant
// G_c from bin 0 (zero outside the window). Its exact derivatives with respect
// to the track weight, the two end points (through R_mid and beta_perp at the
// midpoint, and through the arrival times of the box edges) and the
// refractivity n0 - 1 (through the path indices of the edges) are accumulated
// per track over all antennas; beta and the emission times are held fixed.
//
// Kernels: phi_kernel (one workgroup per antenna: prefix sums of G in double),
// vjp_kernel (one thread per track, loop over antennas, per-track gradients
// in registers, per-workgroup partial of the n0 - 1 gradient in fixed order)
// and n0_sum_kernel (fixed-order sum of the partials).
#include <type_traits>

#include "rt_internal.h"

namespace rt {

constexpr int kVjpBlock = 256;

// Phi[a][c][j] = sum_{i < j} G[a][i][c], j = 0..B (double).
template <typename TG>
__global__ void __launch_bounds__(256) phi_kernel(const TG *grad, double *phi, int n_bins) {
  const int64_t a = blockIdx.x;
  const TG *g = grad + (size_t)a * n_bins * 3;
  double *out = phi + (size_t)a * 3 * (n_bins + 1);
  __shared__ double carry[256][3];
  const int per = (n_bins + blockDim.x - 1) / blockDim.x;
  const int b0 = min((int)threadIdx.x * per, n_bins), b1 = min(b0 + per, n_bins);
  double run[3] = {0.0, 0.0, 0.0};
  for (int b = b0; b < b1; ++b)
    for (int c = 0; c < 3; ++c) run[c] += (double)g[3 * b + c];
  for (int c = 0; c < 3; ++c) carry[threadIdx.x][c] = run[c];
  __syncthreads();
  if (threadIdx.x < 3) {
    double acc = 0.0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      double x = carry[t][threadIdx.x];
      carry[t][threadIdx.x] = acc;
      acc += x;
    }
    out[threadIdx.x * (n_bins + 1) + n_bins] = acc;   // Phi[B]: the total
  }
  __syncthreads();
  for (int c = 0; c < 3; ++c) run[c] = carry[threadIdx.x][c];
  for (int b = b0; b < b1; ++b)
    for (int c = 0; c < 3; ++c) {
      out[c * (n_bins + 1) + b] = run[c];
      run[c] += (double)g[3 * b + c];
    }
}

template <typename TG>
struct GradView {
  const TG *g;       // [B][3] of one antenna
  const double *phi; // [3][B + 1] of one antenna
  int n_bins;
  double nb;

  // G_c at u (zero outside [0, B))
  __device__ __forceinline__ double value(int c, double u) const {
    if (!(u >= 0.0 && u < nb)) return 0.0;
    return (double)g[3 * (int)u + c];
  }
  // Phi_c(u) = integral of G_c from 0 to u
  __device__ __forceinline__ double cumulative(int c, double u) const {
    if (!(u > 0.0)) return 0.0;
    if (u >= nb) return phi[c * (n_bins + 1) + n_bins];
    int j = (int)u;
    return phi[c * (n_bins + 1) + j] + (u - (double)j) * (double)g[3 * j + c];
  }
};

struct VjpArgs {
  TrackPtrs tr;
  AntPtrs an;
  Consts c;
  const void *grad;     // [M][B][3], float (mixed) or double
  const double *phi;    // [M][3][B+1]
  double *g_qw, *g_p0, *g_p1;   // [n], [3][n], [3][n]
  double *n0_part;      // [gridDim.x]
};

// d t / d z_P of the path index for an end at height zp with height factor
// ep (and of n_eff itself), and d n_eff / d (n0 - 1); antenna at height za
// with height factor ea.
__device__ __forceinline__ void index_derivatives(double zp, double za, double ep, double ea,
                                                  const Consts &c, double &neff, double &dn_dz,
                                                  double &dn_dn0) {
  if (c.medium == 0) {
    neff = c.n_uniform;
    dn_dz = 0.0;
    dn_dn0 = 1.0;
    return;
  }
  neff = path_index(zp, za, ep, ea, c);
  double dz = zp - za;
  if (fabs(dz) >= 1e-3) {
    double f = (ea - ep) / dz;
    dn_dn0 = c.h * f;
    // d f / d zp = (ep / h) / dz - f / dz
    dn_dz = c.n0h * ((ep / c.h) / dz - f / dz);
  } else {
    double e = exp(-(((zp + za) * 0.5) / c.h));
    dn_dn0 = e;
    dn_dz = -c.n0m1 * e / (2.0 * c.h);
  }
}

template <int P>
__global__ void __launch_bounds__(kVjpBlock) vjp_kernel(VjpArgs v) {
  using In = typename std::conditional<P == 0, double, float>::type;
  const Consts &c = v.c;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double gn_local = 0.0;
  if (i < v.tr.n) {
    const double x0 = v.tr.x0[i], y0 = v.tr.y0[i], z0 = v.tr.z0[i], t0 = v.tr.t0[i];
    const double x1 = v.tr.x1[i], y1 = v.tr.y1[i], z1 = v.tr.z1[i], t1 = v.tr.t1[i];
    const double b[3] = {(double)((const In *)v.tr.bx)[i], (double)((const In *)v.tr.by)[i],
                         (double)((const In *)v.tr.bz)[i]};
    const double qw = (double)((const In *)v.tr.qw)[i];
    bool ok = isfinite(qw) && isfinite(x0) && isfinite(y0) && isfinite(z0) && isfinite(t0) &&
              isfinite(x1) && isfinite(y1) && isfinite(z1) && isfinite(t1) && isfinite(b[0]) &&
              isfinite(b[1]) && isfinite(b[2]);
    double gq = 0.0, gp0[3] = {0.0, 0.0, 0.0}, gp1[3] = {0.0, 0.0, 0.0};
    const double e0 = c.medium == 1 ? height_factor(z0, c) : 0.0;
    const double e1 = c.medium == 1 ? height_factor(z1, c) : 0.0;
    const double mx = (x0 + x1) * 0.5, my = (y0 + y1) * 0.5, mz = (z0 + z1) * 0.5;
    const double kdt = c.k * (t1 - t0);   // I = kdt * qw * beta_perp / R_m
    // path indices and their derivatives depend on the antenna height only:
    // recomputed when it changes (a uniform test: every lane sees the same
    // antenna)
    double z_prev = __builtin_nan(""), ne0 = 0, dnz0 = 0, dnn0 = 0, ne1 = 0, dnz1 = 0, dnn1 = 0;
    for (int64_t a = 0; ok && a < v.an.m; ++a) {
      const double ax = v.an.x[a], ay = v.an.y[a], az = v.an.z[a], tau = v.an.t_start[a];
      if (!(az == z_prev)) {
        const double ea = c.medium == 1 ? height_factor(az, c) : 0.0;
        index_derivatives(z0, az, e0, ea, c, ne0, dnz0, dnn0);
        index_derivatives(z1, az, e1, ea, c, ne1, dnz1, dnn1);
        z_prev = az;
      }
      double d0x, d0y, d0z, r0, r02, d1x, d1y, d1z, r1, r12;
      const double us = arrival_bins(x0, y0, z0, t0, ax, ay, az, tau, ne0, c, d0x, d0y, d0z, r0, r02);
      const double ue = arrival_bins(x1, y1, z1, t1, ax, ay, az, tau, ne1, c, d1x, d1y, d1z, r1, r12);
      const bool start_lo = us < ue;
      const double ulo = start_lo ? us : ue, uhi = start_lo ? ue : us;
      if (!(uhi >= 0.0 && ulo < c.nbins_d)) continue;
      // midpoint geometry
      const double d[3] = {ax - mx, ay - my, az - mz};
      const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
      if (r2 == 0.0) continue;
      const double r = sqrt(r2);
      const double ir = 1.0 / r, ir2 = ir * ir;
      const double bd = (b[0] * d[0] + b[1] * d[1]) + b[2] * d[2];
      double iu[3];   // integral per unit weight
      for (int k = 0; k < 3; ++k) iu[k] = kdt * (b[k] - bd * ir2 * d[k]) * ir;
      GradView<In> gv{(const In *)v.grad + (size_t)a * c.n_bins * 3,
                      v.phi + (size_t)a * 3 * (c.n_bins + 1), c.n_bins, c.nbins_d};
      const bool same_bin = floor(ulo) == floor(uhi);
      const double iw = 1.0 / (uhi - ulo);
      double gbar[3], dl_dlo = 0.0, dl_dhi = 0.0;
      for (int k = 0; k < 3; ++k) {
        if (same_bin) {
          gbar[k] = gv.value(k, ulo);
        } else {
          gbar[k] = (gv.cumulative(k, uhi) - gv.cumulative(k, ulo)) * iw;
          const double ik = qw * iu[k] * c.inv_dt;
          dl_dhi += ik * (gv.value(k, uhi) - gbar[k]) * iw;
          dl_dlo += ik * (gbar[k] - gv.value(k, ulo)) * iw;
        }
      }
      // weight: the pair's loss share is linear in qw
      double gam[3];
      for (int k = 0; k < 3; ++k) {
        gam[k] = gbar[k] * c.inv_dt;
        gq += iu[k] * gam[k];
      }
      // midpoint: I = K (beta / R - (beta.d) d / R^3), K = kdt qw, d = X - M
      const double kk = kdt * qw;
      const double gb = (gam[0] * b[0] + gam[1] * b[1]) + gam[2] * b[2];
      const double gd = (gam[0] * d[0] + gam[1] * d[1]) + gam[2] * d[2];
      const double ir3 = ir2 * ir, ir5 = ir3 * ir2;
      for (int k = 0; k < 3; ++k) {
        const double dl_dd = kk * (-(gb * d[k] + gd * b[k] + bd * gam[k]) * ir3 +
                                   3.0 * bd * gd * d[k] * ir5);
        gp0[k] -= 0.5 * dl_dd;   // d = X - (P0 + P1) / 2
        gp1[k] -= 0.5 * dl_dd;
      }
      // box edges: u = (T + n_eff R / c - tau) / dt
      const double dl_ds = (start_lo ? dl_dlo : dl_dhi) * c.inv_dt * c.inv_c;
      const double dl_de = (start_lo ? dl_dhi : dl_dlo) * c.inv_dt * c.inv_c;
      // d (n_eff R) / d P = -n_eff d / R + R dn_eff/dz e_z
      const double n0r = ne0 / r0, n1r = ne1 / r1;
      gp0[0] += dl_ds * (-n0r * d0x);
      gp0[1] += dl_ds * (-n0r * d0y);
      gp0[2] += dl_ds * (-n0r * d0z + r0 * dnz0);
      gp1[0] += dl_de * (-n1r * d1x);
      gp1[1] += dl_de * (-n1r * d1y);
      gp1[2] += dl_de * (-n1r * d1z + r1 * dnz1);
      gn_local += dl_ds * r0 * dnn0 + dl_de * r1 * dnn1;
    }
    v.g_qw[i] = gq;
    for (int k = 0; k < 3; ++k) {
      v.g_p0[(size_t)k * v.tr.n + i] = gp0[k];
      v.g_p1[(size_t)k * v.tr.n + i] = gp1[k];
    }
  }
  // fixed-order workgroup reduction of the n0 - 1 gradient
  __shared__ double red[kVjpBlock];
  red[threadIdx.x] = gn_local;
  __syncthreads();
  for (int s = kVjpBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) v.n0_part[blockIdx.x] = red[0];
}

// Endpoint: the impulse of a landing end is E = c W / num with d = X - P,
// c = s k qw / dt, q = (beta.d) / R^2, W = d q - beta and
// num = R - n_src (beta.d); the bin it lands in is piecewise constant in the
// parameters and held fixed. For f = g.E (g = G at that bin):
//   df/dd_j = (c / num) (g_j q + (g.d) dq/dd_j) - c (g.W) / num^2 dnum/dd_j,
//   dq/dd_j = beta_j / R^2 - 2 (beta.d) d_j / R^4,  dnum/dd_j = d_j / R - n_src beta_j,
//   df/dn_src = c (g.W) (beta.d) / num^2,
// and dP = -dd; n_src = 1 + (n0 - 1) e(z_P) adds the height derivative of e.
template <int P>
__global__ void __launch_bounds__(kVjpBlock) ep_vjp_kernel(VjpArgs v) {
  using In = typename std::conditional<P == 0, double, float>::type;
  const Consts &c = v.c;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double gn_local = 0.0;
  if (i < v.tr.n) {
    const double pos[2][4] = {{v.tr.x0[i], v.tr.y0[i], v.tr.z0[i], v.tr.t0[i]},
                              {v.tr.x1[i], v.tr.y1[i], v.tr.z1[i], v.tr.t1[i]}};
    const double b[3] = {(double)((const In *)v.tr.bx)[i], (double)((const In *)v.tr.by)[i],
                         (double)((const In *)v.tr.bz)[i]};
    const double qw = (double)((const In *)v.tr.qw)[i];
    bool ok = isfinite(qw) && isfinite(b[0]) && isfinite(b[1]) && isfinite(b[2]);
    for (int e = 0; e < 2; ++e)
      for (int k = 0; k < 4; ++k) ok = ok && isfinite(pos[e][k]);
    double gq = 0.0, gp[2][3] = {{0.0, 0.0, 0.0}, {0.0, 0.0, 0.0}};
    double hf[2] = {0.0, 0.0}, ns[2] = {c.n_uniform, c.n_uniform};
    if (c.medium == 1)
      for (int e = 0; e < 2; ++e) {
        hf[e] = height_factor(pos[e][2], c);
        ns[e] = fma(c.n0m1, hf[e], 1.0);
      }
    const double kdt = c.k * c.inv_dt;
    double z_prev = __builtin_nan(""), nes[2] = {c.n_uniform, c.n_uniform};
    for (int64_t a = 0; ok && a < v.an.m; ++a) {
      const double ax = v.an.x[a], ay = v.an.y[a], az = v.an.z[a], tau = v.an.t_start[a];
      if (c.medium == 1 && !(az == z_prev)) {   // uniform test: one antenna per step
        const double ea = height_factor(az, c);
        for (int e = 0; e < 2; ++e) nes[e] = path_index(pos[e][2], az, hf[e], ea, c);
        z_prev = az;
      }
      const In *ga = (const In *)v.grad + (size_t)a * c.n_bins * 3;
      for (int e = 0; e < 2; ++e) {
        const double ne = nes[e];
        double d[3], r, r2;
        const double u = arrival_bins(pos[e][0], pos[e][1], pos[e][2], pos[e][3], ax, ay, az, tau,
                                      ne, c, d[0], d[1], d[2], r, r2);
        if (!(u >= 0.0 && u < c.nbins_d)) continue;
        const double bd = fma(b[0], d[0], fma(b[1], d[1], b[2] * d[2]));
        const double num = fma(-ns[e], bd, r);
        if (num == 0.0) continue;
        const int j = (int)u;
        const double g[3] = {(double)ga[3 * j], (double)ga[3 * j + 1], (double)ga[3 * j + 2]};
        const double s = e == 0 ? 1.0 : -1.0;
        const double ir2 = 1.0 / r2, ir = r * ir2, inum = 1.0 / num;
        const double q = bd * ir2;
        double w[3];
        for (int k = 0; k < 3; ++k) w[k] = fma(d[k], q, -b[k]);
        const double gw = fma(g[0], w[0], fma(g[1], w[1], g[2] * w[2]));
        const double gd = fma(g[0], d[0], fma(g[1], d[1], g[2] * d[2]));
        const double cc = s * kdt * qw;
        gq += s * kdt * gw * inum;
        const double a1 = cc * inum, a2 = a1 * gw * inum;
        for (int k = 0; k < 3; ++k) {
          const double dq = (b[k] - 2.0 * q * d[k]) * ir2;
          const double dnum = d[k] * ir - ns[e] * b[k];
          gp[e][k] -= a1 * (g[k] * q + gd * dq) - a2 * dnum;
        }
        const double dfn = a2 * bd;   // d f / d n_src
        if (c.medium == 1) {
          gn_local += dfn * hf[e];
          gp[e][2] -= dfn * c.n0m1 * hf[e] / c.h;
        } else {
          gn_local += dfn;
        }
      }
    }
    v.g_qw[i] = gq;
    for (int k = 0; k < 3; ++k) {
      v.g_p0[(size_t)k * v.tr.n + i] = gp[0][k];
      v.g_p1[(size_t)k * v.tr.n + i] = gp[1][k];
    }
  }
  __shared__ double red[kVjpBlock];
  red[threadIdx.x] = gn_local;
  __syncthreads();
  for (int s = kVjpBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) v.n0_part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(256) n0_sum_kernel(const double *part, int64_t n, double *out) {
  __shared__ double red[256];
  double s = 0.0;
  for (int64_t j = threadIdx.x; j < n; j += blockDim.x) s += part[j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int k = 128; k > 0; k >>= 1) {
    if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// ZHS: [Phi tables][per-workgroup n0 partials]; Endpoint: the partials only.
static size_t phi_bytes(const rt_plan &p) {
  if (p.formalism != RT_ZHS) return 0;
  return align256((size_t)p.det.n_antennas * 3 * (p.det.n_bins + 1) * sizeof(double));
}

size_t vjp_workspace_bytes(const rt_plan &p, int64_t n) {
  const int64_t blocks = (n + kVjpBlock - 1) / kVjpBlock;
  return phi_bytes(p) + align256((size_t)std::max<int64_t>(blocks, 1) * sizeof(double));
}

hipError_t launch_vjp(const rt_plan &p, const rt_tracks &t, const void *grad, double *g_qw,
                      double *g_p0, double *g_p1, double *g_n0, void *workspace,
                      hipStream_t stream) {
  char *ws = reinterpret_cast<char *>(workspace);
  double *phi = reinterpret_cast<double *>(ws);
  double *part = reinterpret_cast<double *>(ws + phi_bytes(p));
  const unsigned m = (unsigned)p.det.n_antennas;
  if (p.formalism == RT_ZHS) {
    if (p.precision == RT_FP64)
      phi_kernel<double><<<m, 256, 0, stream>>>((const double *)grad, phi, p.det.n_bins);
    else
      phi_kernel<float><<<m, 256, 0, stream>>>((const float *)grad, phi, p.det.n_bins);
  }
  VjpArgs v;
  v.tr = track_ptrs(t);
  v.an = ant_ptrs(p.det);
  v.c = p.c;
  v.grad = grad;
  v.phi = phi;
  v.g_qw = g_qw;
  v.g_p0 = g_p0;
  v.g_p1 = g_p1;
  v.n0_part = part;
  const int64_t blocks = (t.n + kVjpBlock - 1) / kVjpBlock;
  if (p.formalism == RT_ZHS) {
    if (p.precision == RT_FP64)
      vjp_kernel<0><<<(unsigned)blocks, kVjpBlock, 0, stream>>>(v);
    else
      vjp_kernel<1><<<(unsigned)blocks, kVjpBlock, 0, stream>>>(v);
  } else {
    if (p.precision == RT_FP64)
      ep_vjp_kernel<0><<<(unsigned)blocks, kVjpBlock, 0, stream>>>(v);
    else
      ep_vjp_kernel<1><<<(unsigned)blocks, kVjpBlock, 0, stream>>>(v);
  }
  n0_sum_kernel<<<1, 256, 0, stream>>>(part, blocks, g_n0);
  return hipGetLastError();
}

}  // namespace rt
