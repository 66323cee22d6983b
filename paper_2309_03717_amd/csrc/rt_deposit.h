// rt_deposit.h -- device building blocks of the deposit path shared by the
// single-plan kernels (forward.hip) and the batched persistent kernel
// (batch.hip): precision traits, the per-track record, the Endpoint impulse,
// the ZHS box and the per-record deposit loop over a tile of antennas.
#pragma once

#include "rt_device.h"

namespace rt {

using acc_t = double;

template <int P>
struct Prec;
template <>
struct Prec<0> {  // RT_FP64
  using in = double;   // beta, qw
  using out = double;  // traces
};
template <>
struct Prec<1> {  // RT_MIXED
  using in = float;
  using out = float;
};

// ------------------------------------------------------------------ track record

// Per-track record, kRec doubles per track, blocked by waves of 64 tracks:
// field f of track 64 b + l is rec[(b * kRec + f) * 64 + l], so a wave reads
// each field as one contiguous 512-byte run from a single base address.
constexpr int kRec = 16;
enum : int {
  R_X0, R_Y0, R_Z0, R_T0,  // start point and time
  R_X1, R_Y1, R_Z1, R_T1,  // end point and time
  R_NE0, R_NE1,            // path index of each end to the height of antenna 0
  R_E0, R_E1,              // height factors exp(-(z / h)) of the two ends
  R_AMP,                   // Endpoint: k qw / dt;  ZHS: k qw (t1 - t0) / dt
  R_BX, R_BY, R_BZ         // velocity (units of c)
};

// Builds the record of one track (fields as above). A track with any
// non-finite field gets NaN times so that no antenna window accepts it.
// z_ref, e_ref: height of antenna 0 and its height factor.
template <int F, int P>
__device__ __forceinline__ void make_record(const TrackPtrs &tr, int64_t i, bool present,
                                            const Consts &c, double z_ref, double e_ref,
                                            double *v) {
  using In = typename Prec<P>::in;
  bool ok = present;
  if (ok) {
    v[R_X0] = tr.x0[i];
    v[R_Y0] = tr.y0[i];
    v[R_Z0] = tr.z0[i];
    v[R_T0] = tr.t0[i];
    v[R_X1] = tr.x1[i];
    v[R_Y1] = tr.y1[i];
    v[R_Z1] = tr.z1[i];
    v[R_T1] = tr.t1[i];
    v[R_BX] = (double)((const In *)tr.bx)[i];
    v[R_BY] = (double)((const In *)tr.by)[i];
    v[R_BZ] = (double)((const In *)tr.bz)[i];
    double qw = (double)((const In *)tr.qw)[i];
    v[R_AMP] = F == 0 ? c.k * qw * c.inv_dt : c.k * qw * (v[R_T1] - v[R_T0]) * c.inv_dt;
    ok = isfinite(qw);
    for (int f = R_X0; f <= R_T1; ++f) ok = ok && isfinite(v[f]);
    for (int f = R_BX; f <= R_BZ; ++f) ok = ok && isfinite(v[f]);
  }
  if (!ok) {
    for (int f = 0; f < kRec; ++f) v[f] = 0.0;
    v[R_T0] = v[R_T1] = __builtin_nan("");
  }
  v[R_E0] = v[R_E1] = 0.0;
  v[R_NE0] = v[R_NE1] = c.n_uniform;
  if (c.medium == 1) {
    v[R_E0] = height_factor(v[R_Z0], c);
    v[R_E1] = height_factor(v[R_Z1], c);
    v[R_NE0] = path_index(v[R_Z0], z_ref, v[R_E0], e_ref, c);
    v[R_NE1] = path_index(v[R_Z1], z_ref, v[R_E1], e_ref, c);
  }
}

__device__ __forceinline__ void put3(acc_t *row, int j, double vx, double vy, double vz) {
  acc_t *p = row + 3 * j;
  lds_add(p, vx);
  lds_add(p + 1, vy);
  lds_add(p + 2, vz);
}

// ZHS difference deposit at absolute bin j of a segment [lo, hi): bins before
// the segment fold into its first bin (the segment's prefix scan starts
// there), bins at or after its end are dropped.
__device__ __forceinline__ void put3_clamped(acc_t *row, int j, int lo, int hi, double vx,
                                             double vy, double vz) {
  if (j < lo) j = lo;
  if (j < hi) put3(row, j - lo, vx, vy, vz);
}

// 1/x and 1/sqrt(x) from the hardware estimate plus one Newton step.
__device__ __forceinline__ double fast_rcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double fast_rsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = fma(-0.5 * x * y, y, 1.5);
  return y * h;
}

// Endpoint impulse of one track end at one antenna: s k qw [r x (r x beta)] /
// ((1 - n_src beta.r) R dt), evaluated as sc (d (beta.d) / R^2 - beta) / num
// with num = R - n_src (beta.d) = (1 - n_src beta.r) R and sc = s k qw / dt.
template <int P>
__device__ __forceinline__ void endpoint_end(acc_t *row, int lo, double lo_d, double hi_d,
                                             double sc, double px, double py, double pz,
                                             double tp, double ax, double ay, double az,
                                             double tau, double neff, double nsrc, double bx,
                                             double by, double bz, const Consts &c) {
  double dx, dy, dz, r, r2;
  double u = arrival_bins(px, py, pz, tp, ax, ay, az, tau, neff, c, dx, dy, dz, r, r2);
  if (!(u >= lo_d && u < hi_d)) return;   // outside this segment of the window (or NaN)
  const int j = (int)u - lo;
  double bd = fma(bx, dx, fma(by, dy, bz * dz));
  double num = fma(-nsrc, bd, r);
  if (num == 0.0) return;   // on the Cherenkov cone, or R = 0
  double q, a;
  if (P == 0) {
    q = bd / r2;
    a = sc / num;
  } else {
    q = bd * fast_rcp(r2);
    a = sc * fast_rcp(num);
  }
  put3(row, j, fma(dx, q, -bx) * a, fma(dy, q, -by) * a, fma(dz, q, -bz) * a);
}

// ZHS box of one segment at one antenna. us, ue: arrival of start and end in
// bins. The box [u_lo, u_hi] of time integral I = k qw beta_perp (t1-t0) /
// R_mid has bin averages Ibar * overlap / (u_hi - u_lo), Ibar = I / dt; it is
// deposited as at most four differences whose prefix sum is that average,
// each bounded by |Ibar|.
template <int P>
__device__ __forceinline__ void zhs_box(acc_t *row, int lo, int hi, double lo_d, double hi_d,
                                        double us, double ue, double mx, double my, double mz,
                                        double ax, double ay, double az, double cz, double bx,
                                        double by, double bz) {
  double ulo = us < ue ? us : ue;
  double uhi = us < ue ? ue : us;
  if (!(uhi >= lo_d && ulo < hi_d)) return;   // outside this segment (or NaN)
  // midpoint geometry: Ibar = cz * beta_perp / R_m, cz = k qw (t1 - t0) / dt
  double dx = ax - mx, dy = ay - my, dz = az - mz;
  double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
  if (r2 == 0.0) return;
  double rinv = P == 0 ? 1.0 / sqrt(r2) : fast_rsq(r2);
  double q = fma(bx, dx, fma(by, dy, bz * dz)) * (rinv * rinv);
  double s = cz * rinv;
  double ix = fma(-dx, q, bx) * s, iy = fma(-dy, q, by) * s, iz = fma(-dz, q, bz) * s;
  double kl = floor(ulo), kh = floor(uhi);
  if (kl == kh) {   // whole box inside one bin of this segment
    int j = (int)kl;
    put3(row, j - lo, ix, iy, iz);
    if (j + 1 < hi) put3(row, j + 1 - lo, -ix, -iy, -iz);
    return;
  }
  double w = uhi - ulo;
  double wi = P == 0 ? 1.0 / w : fast_rcp(w);
  double flo = (kl + 1.0) - ulo;   // share of bin kl, in (0, 1]
  double fhi = uhi - kh;           // share of bin kh, in [0, 1)
  // clamp far-out indices before the int conversion (all fold or drop alike)
  int jl = (int)fmax(kl, lo_d - 2.0);
  int jh = (int)fmin(kh, hi_d);
  if (kh == kl + 1.0) {
    double fa = flo * wi, fb = fhi * wi;
    double ax_ = ix * fa, ay_ = iy * fa, az_ = iz * fa;
    double bx_ = ix * fb, by_ = iy * fb, bz_ = iz * fb;
    put3_clamped(row, jl, lo, hi, ax_, ay_, az_);
    put3_clamped(row, jl + 1, lo, hi, bx_ - ax_, by_ - ay_, bz_ - az_);
    put3_clamped(row, jl + 2, lo, hi, -bx_, -by_, -bz_);
  } else {
    double hx = ix * wi, hy = iy * wi, hz = iz * wi;
    double gl = 1.0 - flo, gh = 1.0 - fhi;
    put3_clamped(row, jl, lo, hi, hx * flo, hy * flo, hz * flo);
    put3_clamped(row, jl + 1, lo, hi, hx * gl, hy * gl, hz * gl);
    put3_clamped(row, jh, lo, hi, -hx * gh, -hy * gh, -hz * gh);
    put3_clamped(row, jh + 1, lo, hi, -hx * fhi, -hy * fhi, -hz * fhi);
  }
}

// The tile antennas of one workgroup (uniform values).
template <int AT>
struct Tile {
  double ax[AT], ay[AT], az[AT], tau[AT], ea[AT];
  bool at_ref[AT];   // at the height of antenna 0: the record's path index applies
};

// All deposits of one track record (this lane's track) into the tile
// antennas selected by mask.
template <int F, int P, int MED, int AT>
__device__ __forceinline__ void deposit_record(const double *v, uint64_t mask, const Tile<AT> &t,
                                               acc_t *tile, int row_len, int lo, int hi,
                                               double lo_d, double hi_d, const Consts &c) {
  const double x0 = v[R_X0], y0 = v[R_Y0], z0 = v[R_Z0], t0 = v[R_T0];
  const double x1 = v[R_X1], y1 = v[R_Y1], z1 = v[R_Z1], t1 = v[R_T1];
  const double amp = v[R_AMP], bx = v[R_BX], by = v[R_BY], bz = v[R_BZ];
  const double e0 = MED == 1 ? v[R_E0] : 0.0, e1 = MED == 1 ? v[R_E1] : 0.0;
  if (F == 0) {
    const double ns0 = MED == 1 ? fma(c.n0m1, e0, 1.0) : c.n_uniform;
    const double ns1 = MED == 1 ? fma(c.n0m1, e1, 1.0) : c.n_uniform;
#pragma unroll
    for (int a = 0; a < AT; ++a) {
      if ((mask >> a) & 1) {
        double ne0 = v[R_NE0], ne1 = v[R_NE1];
        if (MED == 1 && !t.at_ref[a]) {
          ne0 = path_index(z0, t.az[a], e0, t.ea[a], c);
          ne1 = path_index(z1, t.az[a], e1, t.ea[a], c);
        }
        acc_t *row = tile + a * row_len;
        endpoint_end<P>(row, lo, lo_d, hi_d, amp, x0, y0, z0, t0, t.ax[a], t.ay[a], t.az[a],
                        t.tau[a], ne0, ns0, bx, by, bz, c);
        endpoint_end<P>(row, lo, lo_d, hi_d, -amp, x1, y1, z1, t1, t.ax[a], t.ay[a], t.az[a],
                        t.tau[a], ne1, ns1, bx, by, bz, c);
      }
    }
  } else {
    const double mx = (x0 + x1) * 0.5, my = (y0 + y1) * 0.5, mz = (z0 + z1) * 0.5;
#pragma unroll
    for (int a = 0; a < AT; ++a) {
      if ((mask >> a) & 1) {
        double ne0 = v[R_NE0], ne1 = v[R_NE1];
        if (MED == 1 && !t.at_ref[a]) {
          ne0 = path_index(z0, t.az[a], e0, t.ea[a], c);
          ne1 = path_index(z1, t.az[a], e1, t.ea[a], c);
        }
        double dx, dy, dz, rr, r2;
        double us = arrival_bins(x0, y0, z0, t0, t.ax[a], t.ay[a], t.az[a], t.tau[a], ne0, c, dx,
                                 dy, dz, rr, r2);
        double ue = arrival_bins(x1, y1, z1, t1, t.ax[a], t.ay[a], t.az[a], t.tau[a], ne1, c, dx,
                                 dy, dz, rr, r2);
        zhs_box<P>(tile + a * row_len, lo, hi, lo_d, hi_d, us, ue, mx, my, mz, t.ax[a], t.ay[a],
                   t.az[a], amp, bx, by, bz);
      }
    }
  }
}

// Deposits of the wave blocks [b_first, b_end) (stride `waves`, one block per
// wave per step) of a record array into the LDS tile, with the next record
// loaded before the current one is processed.
template <int F, int P, int MED, int AT>
__device__ __forceinline__ void deposit_blocks(const double *rec, int64_t b_first, int64_t b_end,
                                               int64_t waves, uint64_t mask, const Tile<AT> &t,
                                               acc_t *tile, int row_len, int lo, int hi,
                                               double lo_d, double hi_d, const Consts &c) {
  const int lane = threadIdx.x & 63;
  double nx[kRec];
  if (b_first < b_end) {
    const double *r = rec + b_first * (kRec * 64) + lane;
#pragma unroll
    for (int f = 0; f < kRec; ++f) nx[f] = r[f * 64];
  }
  for (int64_t blk = b_first; blk < b_end; blk += waves) {
    double rv[kRec];
#pragma unroll
    for (int f = 0; f < kRec; ++f) rv[f] = nx[f];
    if (blk + waves < b_end) {
      const double *r = rec + (blk + waves) * (kRec * 64) + lane;
#pragma unroll
      for (int f = 0; f < kRec; ++f) nx[f] = r[f * 64];
    }
    deposit_record<F, P, MED, AT>(rv, mask, t, tile, row_len, lo, hi, lo_d, hi_d, c);
  }
}

// Loads the tile antennas [a_begin, a_begin + n_ant) (uniform per workgroup).
template <int AT, int MED>
__device__ __forceinline__ void load_tile(const AntPtrs &an, int64_t a_begin, int n_ant,
                                          const Consts &c, Tile<AT> &t) {
  const double z_ref = an.z[0];
#pragma unroll
  for (int a = 0; a < AT; ++a) {
    int64_t ai = a_begin + (a < n_ant ? a : 0);
    t.ax[a] = an.x[ai];
    t.ay[a] = an.y[ai];
    t.az[a] = an.z[ai];
    t.tau[a] = an.t_start[ai];
    t.ea[a] = MED == 1 ? height_factor(t.az[a], c) : 0.0;
    t.at_ref[a] = t.az[a] == z_ref;
  }
}

}  // namespace rt
