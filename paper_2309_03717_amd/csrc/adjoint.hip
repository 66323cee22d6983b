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
// Every medium: in the flat ones the path index depends on the heights only
// (its derivative is cached per antenna height); over the spherical Earth its
// gradient in the emission point has horizontal components and is taken per
// pair from the quadrature.
//
// Kernels: phi_kernel (one workgroup per antenna: prefix sums of G in double,
// written with G itself as one record per bin edge, so that a box edge reads
// its Phi and G from one place),
// vjp_kernel (one thread per track, loop over antennas, per-track gradients
// in registers, per-workgroup partial of the n0 - 1 gradient in fixed order)
// and n0_sum_kernel (fixed-order sum of the partials).
#include <type_traits>

#include "rt_internal.h"

namespace rt {

constexpr int kVjpBlock = 256;

// Edge records of one antenna, j = 0..B, kEdge doubles each (16-byte aligned):
// Phi_c[j] = sum_{i < j} G[i][c] in slots 0-2 and G[j][c] (0 for j = B) in
// slots 3-5, both in double.
constexpr int kEdge = 6;

template <typename TG>
__global__ void __launch_bounds__(256) phi_kernel(const TG *grad, double *phi, int n_bins) {
  const int64_t a = blockIdx.x;
  const TG *g = grad + (size_t)a * n_bins * 3;
  double *out = phi + (size_t)a * kEdge * (n_bins + 1);
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
    out[(size_t)n_bins * kEdge + threadIdx.x] = acc;   // Phi[B]: the total
    out[(size_t)n_bins * kEdge + 3 + threadIdx.x] = 0.0;
  }
  __syncthreads();
  for (int c = 0; c < 3; ++c) run[c] = carry[threadIdx.x][c];
  for (int b = b0; b < b1; ++b)
    for (int c = 0; c < 3; ++c) {
      const double gv = (double)g[3 * b + c];
      out[(size_t)b * kEdge + c] = run[c];
      out[(size_t)b * kEdge + 3 + c] = gv;
      run[c] += gv;
    }
}

// G and its integral at a box edge u (in bins) of one antenna:
// value[c] = G_c at u (zero outside [0, B)), cumulative[c] = Phi_c(u), the
// integral of G_c from 0 to u, all from the edge record of bin floor(u)
// (three 16-byte loads).
struct EdgeValues {
  double value[3], cumulative[3];

  __device__ __forceinline__ EdgeValues(const double *edges, int n_bins, double nb, double u) {
    const bool inside = u >= 0.0 && u < nb;
    const bool above = u >= nb;
    for (int c = 0; c < 3; ++c) value[c] = cumulative[c] = 0.0;
    if (!(inside || above)) return;   // below the window (or NaN)
    const int j = inside ? (int)u : n_bins;
    const double2 *r = reinterpret_cast<const double2 *>(edges + (size_t)j * kEdge);
    const double2 p01 = r[0], p2g0 = r[1], g12 = r[2];
    const double phi[3] = {p01.x, p01.y, p2g0.x}, g[3] = {p2g0.y, g12.x, g12.y};
    const double w = u - (double)j;
    for (int c = 0; c < 3; ++c) {
      if (inside) {
        value[c] = g[c];
        cumulative[c] = u > 0.0 ? phi[c] + w * g[c] : 0.0;
      } else {
        cumulative[c] = phi[c];   // the total
      }
    }
  }
};

struct VjpArgs {
  TrackPtrs tr;
  AntPtrs an;
  Consts c;
  const void *grad;     // [M][B][3], float (mixed) or double
  const double *phi;    // ZHS: [M][B+1][kEdge] edge records
  double *g_qw, *g_p0, *g_p1;   // [n], [3][n], [3][n]
  double *n0_part;      // [gridDim.x]
};

// Tabulated profile: slope of f at z (the cell tab_f interpolates in; zero
// beyond the end nodes, where f is constant).
__device__ __forceinline__ double tab_slope(double z, const Consts &c) {
  const double t = (z - c.tz0) * c.tinv_dz;
  if (!(t > 0.0) || t >= (double)(c.n_tab - 1)) return 0.0;
  const int k = (int)floor(t);
  return (c.tab[k + 1] - c.tab[k]) * c.tinv_dz;
}

// The per-height path factor the flat media's path index takes: exp(-z/h)
// (exponential), the integral F (tabulated); 0 otherwise. MED: the medium
// kind (0 uniform, 1 exponential, 2 tabulated, 3 spherical) at compile time.
template <int MED>
__device__ __forceinline__ double path_factor_flat(double z, const Consts &c) {
  return MED == 1 ? height_factor(z, c) : MED == 2 ? tab_F(z, c) : 0.0;
}

// Path index of an end at height zp towards an antenna at height za in the
// flat media (0 uniform, 1 exponential, 2 tabulated), with its derivative in
// zp (dn_dz) and in n0 - 1 (dn_dn0). pp, pa: the path factors of the two
// heights (exponential: exp(-z/h); tabulated: the integral F). The index is
// the one the forward timing uses, so the bins are the forward's.
template <int MED>
__device__ __forceinline__ void index_derivatives(double zp, double za, double pp, double pa,
                                                  const Consts &c, double &neff, double &dn_dz,
                                                  double &dn_dn0) {
  if (MED == 0) {
    neff = c.n_uniform;
    dn_dz = 0.0;
    dn_dn0 = 1.0;
    return;
  }
  neff = path_index_m<MED>(zp, za, pp, pa, c);
  const double dz = zp - za;
  if (fabs(dz) >= 1e-3) {
    if (MED == 2) {   // n = 1 + n0m1 (F(zp) - F(za)) / dz, F' = f
      const double fbar = (pp - pa) / dz;
      dn_dn0 = fbar;
      dn_dz = c.n0m1 * (tab_f(zp, c) - fbar) / dz;
    } else {               // n = 1 + n0m1 h (ea - ep) / dz
      const double f = (pa - pp) / dz;
      dn_dn0 = c.h * f;
      // d f / d zp = (ep / h) / dz - f / dz
      dn_dz = c.n0h * ((pp / c.h) / dz - f / dz);
    }
  } else {                 // the local index at the mid height
    const double mid = (zp + za) * 0.5;
    if (MED == 2) {
      dn_dn0 = tab_f(mid, c);
      dn_dz = c.n0m1 * tab_slope(mid, c) * 0.5;
    } else {
      const double e = exp(-(mid / c.h));
      dn_dn0 = e;
      dn_dz = -c.n0m1 * e / (2.0 * c.h);
    }
  }
}

// Spherical Earth: the gradient of the path index with respect to the
// emission point P (all three components) and its derivative in n0 - 1, from
// the quadrature: n = 1 + n0m1 S, S = sum_k w_k exp(-H(q_k) / h),
// q_k = P + s_k (X - P), dH/dq = (q - C) / |q - C|, dq_k / dP = 1 - s_k.
template <class Nodes>
__device__ __forceinline__ void sph_index_gradient(double px, double py, double pz, double ax,
                                                   double ay, double az, const Consts &c,
                                                   const Nodes &nd, double grad[3],
                                                   double &dn_dn0) {
  double sum = 0.0, g0 = 0.0, g1 = 0.0, g2 = 0.0;
#pragma unroll 1
  for (int k = 0; k < kGl; ++k) {
    const double sk = nd.s(k);
    const double qx = px + sk * (ax - px), qy = py + sk * (ay - py), qz = pz + sk * (az - pz);
    const double rho2 = (qx * qx + qy * qy) + qz * (qz + c.re_twice);
    const double len = sqrt(rho2 + c.re2);   // |q - C|
    const double we = nd.w(k) * exp(-sph_exponent(rho2, c));
    sum += we;
    const double f = we * (1.0 - sk) / len;
    g0 += f * qx;
    g1 += f * qy;
    g2 += f * (qz + c.re);
  }
  const double sc = -c.n0m1 / c.h;
  grad[0] = sc * g0;
  grad[1] = sc * g1;
  grad[2] = sc * g2;
  dn_dn0 = sum;
}

// The local (source) index of the Endpoint Doppler factor at P, its gradient
// in P and its derivative in n0 - 1 (the same value as the forward's
// 1 + n0m1 * local factor).
template <int MED>
__device__ __forceinline__ double source_index(double px, double py, double pz, const Consts &c,
                                               double grad[3], double &dn_dn0) {
  grad[0] = grad[1] = grad[2] = 0.0;
  if (MED == 0) {
    dn_dn0 = 1.0;
    return c.n_uniform;
  }
  double e;
  if (MED == 3) {
    const double rho2 = (px * px + py * py) + pz * (pz + c.re_twice);
    const double len = sqrt(rho2 + c.re2);
    e = exp(-sph_exponent(rho2, c));
    const double sc = -c.n0m1 * (e / c.h) / len;
    grad[0] = sc * px;
    grad[1] = sc * py;
    grad[2] = sc * (pz + c.re);
  } else if (MED == 2) {
    e = tab_f(pz, c);
    grad[2] = c.n0m1 * tab_slope(pz, c);
  } else {
    e = height_factor(pz, c);
    grad[2] = -c.n0m1 * e / c.h;
  }
  dn_dn0 = e;
  return fma(c.n0m1, e, 1.0);
}

// MED: the medium kind at compile time, so that each kernel keeps only its
// own registers.
template <int P, int MED>
__global__ void __launch_bounds__(kVjpBlock) __attribute__((amdgpu_waves_per_eu(3)))
vjp_kernel(VjpArgs v) {
  using In = typename std::conditional<P == 0, double, float>::type;
  const Consts c = resolve_consts(v.c);
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
    const double e0 = path_factor_flat<MED>(z0, c), e1 = path_factor_flat<MED>(z1, c);
    const double mx = (x0 + x1) * 0.5, my = (y0 + y1) * 0.5, mz = (z0 + z1) * 0.5;
    const double kdt = c.k * (t1 - t0);   // I = kdt * qw * beta_perp / R_m
    // in the flat media the path indices and their derivatives depend on the
    // antenna height only: recomputed when it changes (a uniform test: every
    // lane sees the same antenna); over the spherical Earth, per pair
    double z_prev = __builtin_nan(""), ne0 = 0, dnn0 = 0, ne1 = 0, dnn1 = 0;
    double gn0[3] = {0.0, 0.0, 0.0}, gn1[3] = {0.0, 0.0, 0.0};
    for (int64_t a = 0; ok && a < v.an.m; ++a) {
      const double ax = v.an.x[a], ay = v.an.y[a], az = v.an.z[a], tau = v.an.t_start[a];
      if (MED == 3) {
        ne0 = sph_path_index(x0, y0, z0, ax, ay, az, c, ConstNodes{v.c});
        ne1 = sph_path_index(x1, y1, z1, ax, ay, az, c, ConstNodes{v.c});
        sph_index_gradient(x0, y0, z0, ax, ay, az, c, ConstNodes{v.c}, gn0, dnn0);
        sph_index_gradient(x1, y1, z1, ax, ay, az, c, ConstNodes{v.c}, gn1, dnn1);
      } else if (!(az == z_prev)) {
        const double ea = path_factor_flat<MED>(az, c);
        index_derivatives<MED>(z0, az, e0, ea, c, ne0, gn0[2], dnn0);
        index_derivatives<MED>(z1, az, e1, ea, c, ne1, gn1[2], dnn1);
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
      // mixed precision: refined hardware estimates (about 1e-15 relative)
      const double ir = P == 0 ? 1.0 / sqrt(r2) : fast_rsq(r2), ir2 = ir * ir;
      const double bd = (b[0] * d[0] + b[1] * d[1]) + b[2] * d[2];
      double iu[3];   // integral per unit weight
      for (int k = 0; k < 3; ++k) iu[k] = kdt * (b[k] - bd * ir2 * d[k]) * ir;
      const double *edges = v.phi + (size_t)a * kEdge * (c.n_bins + 1);
      const EdgeValues lo(edges, c.n_bins, c.nbins_d, ulo), hi(edges, c.n_bins, c.nbins_d, uhi);
      const bool same_bin = floor(ulo) == floor(uhi);
      const double iw = P == 0 ? 1.0 / (uhi - ulo) : fast_rcp(uhi - ulo);
      double gbar[3], dl_dlo = 0.0, dl_dhi = 0.0;
      for (int k = 0; k < 3; ++k) {
        if (same_bin) {
          gbar[k] = lo.value[k];
        } else {
          gbar[k] = (hi.cumulative[k] - lo.cumulative[k]) * iw;
          const double ik = qw * iu[k] * c.inv_dt;
          dl_dhi += ik * (hi.value[k] - gbar[k]) * iw;
          dl_dlo += ik * (gbar[k] - lo.value[k]) * iw;
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
      // d (n_eff R) / d P = -n_eff d / R + R grad n_eff
      const double n0r = P == 0 ? ne0 / r0 : ne0 * fast_rcp(r0);
      const double n1r = P == 0 ? ne1 / r1 : ne1 * fast_rcp(r1);
      gp0[0] += dl_ds * (-n0r * d0x + r0 * gn0[0]);
      gp0[1] += dl_ds * (-n0r * d0y + r0 * gn0[1]);
      gp0[2] += dl_ds * (-n0r * d0z + r0 * gn0[2]);
      gp1[0] += dl_de * (-n1r * d1x + r1 * gn1[0]);
      gp1[1] += dl_de * (-n1r * d1y + r1 * gn1[1]);
      gp1[2] += dl_de * (-n1r * d1z + r1 * gn1[2]);
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
template <int P, int MED>
__global__ void __launch_bounds__(kVjpBlock) ep_vjp_kernel(VjpArgs v) {
  using In = typename std::conditional<P == 0, double, float>::type;
  const Consts c = resolve_consts(v.c);
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
    // source index n(P) of each end with its gradient and n0 - 1 derivative;
    // the path factors of the flat media for the (bin-deciding) path index
    double ns[2], gsrc[2][3], dsrc[2], pf[2];
    for (int e = 0; e < 2; ++e) {
      ns[e] = source_index<MED>(pos[e][0], pos[e][1], pos[e][2], c, gsrc[e], dsrc[e]);
      pf[e] = path_factor_flat<MED>(pos[e][2], c);
    }
    const double kdt = c.k * c.inv_dt;
    double z_prev = __builtin_nan(""), nes[2] = {c.n_uniform, c.n_uniform};
    for (int64_t a = 0; ok && a < v.an.m; ++a) {
      const double ax = v.an.x[a], ay = v.an.y[a], az = v.an.z[a], tau = v.an.t_start[a];
      if (MED == 3) {
        for (int e = 0; e < 2; ++e)
          nes[e] = sph_path_index(pos[e][0], pos[e][1], pos[e][2], ax, ay, az, c,
                                  ConstNodes{v.c});
      } else if ((MED == 1 || MED == 2) && !(az == z_prev)) {   // uniform test
        const double pa = path_factor_flat<MED>(az, c);
        for (int e = 0; e < 2; ++e) nes[e] = path_index_m<MED>(pos[e][2], az, pf[e], pa, c);
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
        const double ir2 = P == 0 ? 1.0 / r2 : fast_rcp(r2), ir = r * ir2;
        const double inum = P == 0 ? 1.0 / num : fast_rcp(num);
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
        gn_local += dfn * dsrc[e];
        for (int k = 0; k < 3; ++k) gp[e][k] += dfn * gsrc[e][k];
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

// ZHS: [edge records][per-workgroup n0 partials][F table of a tabulated
// medium]; Endpoint: the partials and the F table.
static size_t phi_bytes(const rt_plan &p) {
  if (p.formalism != RT_ZHS) return 0;
  return align256((size_t)p.det.n_antennas * kEdge * (p.det.n_bins + 1) * sizeof(double));
}

using VjpKernel = void (*)(VjpArgs);

template <int F, int P>
static VjpKernel vjp_kernel_med(int med) {
  if (F == RT_ZHS) {
    switch (med) {
      case 0: return vjp_kernel<P, 0>;
      case 1: return vjp_kernel<P, 1>;
      case 2: return vjp_kernel<P, 2>;
      default: return vjp_kernel<P, 3>;
    }
  }
  switch (med) {
    case 0: return ep_vjp_kernel<P, 0>;
    case 1: return ep_vjp_kernel<P, 1>;
    case 2: return ep_vjp_kernel<P, 2>;
    default: return ep_vjp_kernel<P, 3>;
  }
}

// kind = formalism * 8 + precision * 4 + medium kind
static VjpKernel vjp_kernel_for(int kind) {
  const int med = kind & 3, prec = (kind >> 2) & 1, f = kind >> 3;
  if (f == RT_ZHS) return prec ? vjp_kernel_med<RT_ZHS, 1>(med) : vjp_kernel_med<RT_ZHS, 0>(med);
  return prec ? vjp_kernel_med<RT_ENDPOINT, 1>(med) : vjp_kernel_med<RT_ENDPOINT, 0>(med);
}

static size_t part_bytes(int64_t n) {
  const int64_t blocks = (n + kVjpBlock - 1) / kVjpBlock;
  return align256((size_t)std::max<int64_t>(blocks, 1) * sizeof(double));
}

size_t vjp_workspace_bytes(const rt_plan &p, int64_t n) {
  return phi_bytes(p) + part_bytes(n) + table_bytes(p);
}

hipError_t launch_vjp(const rt_plan &p, const rt_tracks &t, const void *grad, double *g_qw,
                      double *g_p0, double *g_p1, double *g_n0, void *workspace,
                      hipStream_t stream) {
  char *ws = reinterpret_cast<char *>(workspace);
  double *phi = reinterpret_cast<double *>(ws);
  double *part = reinterpret_cast<double *>(ws + phi_bytes(p));
  Consts c = p.c;
  if (p.med.kind == RT_TABULATED) {
    double *cells = reinterpret_cast<double *>(ws + phi_bytes(p) + part_bytes(t.n));
    launch_tab_cells(p, cells, stream);
    c.tabF = cells;
  }
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
  v.c = c;
  v.grad = grad;
  v.phi = phi;
  v.g_qw = g_qw;
  v.g_p0 = g_p0;
  v.g_p1 = g_p1;
  v.n0_part = part;
  const int64_t blocks = (t.n + kVjpBlock - 1) / kVjpBlock;
  const int kind = p.formalism * 8 + p.precision * 4 + p.med.kind;
  // no tracks: no per-track launch (a grid of zero workgroups is not a
  // valid launch); the n0 - 1 gradient is then the empty sum, 0
  if (blocks > 0) vjp_kernel_for(kind)<<<(unsigned)blocks, kVjpBlock, 0, stream>>>(v);
  n0_sum_kernel<<<1, 256, 0, stream>>>(part, blocks, g_n0);
  return hipGetLastError();
}

}  // namespace rt
