// rt_deposit.h -- device building blocks of the deposit path shared by the
// single-plan kernels (forward.hip) and the batched persistent kernel
// (batch.hip): precision traits, the per-track record, the Endpoint impulse,
// the ZHS box and the per-record deposit loop over a tile of antennas.
#pragma once

#include "rt_device.h"

namespace rt {

using acc_t = double;

// Rows of a ZHS trace tile carry two bins past the segment end, which take
// the difference deposits that fall just beyond it (at most two bins: the
// box's last bin is clamped to the segment end first) and are never read,
// and two bins before its start (below). Endpoint impulses land inside the
// segment only.
// (Measured: predicating the deposits past the end instead costs the ZHS
// deposit 4%; padding the Endpoint tile past 96 KiB cost its FP64 deposit
// 20%.)
__host__ __device__ constexpr int tile_pad(int formalism) { return formalism == 1 ? 4 : 0; }
// ZHS rows also start two bins early: the differences a box deposits before
// the segment land there and are added into its first bin when the tile is
// flushed (fold_front), so the box takes no clamps on its first two bins.
__host__ __device__ constexpr int tile_front(int formalism) { return formalism == 1 ? 2 : 0; }

// Fixed-point ZHS accumulation (RT_MIXED): every value v, scaled by the
// call's power-of-two inverse unit s, is rounded to the nearest integer by
// adding kFxMagic = 1.5 * 2^52 in one FMA (for |v s| < 2^51 the sum's exponent
// is fixed and its low mantissa bits are round(v s) + 2^51), so that the bits
// of fma(v, s, kFxMagic) minus kFxMagicBits are round(v s) as a two's
// complement integer. Integer sums are exact and independent of their order,
// which makes these traces bitwise reproducible for any tiling and launch.
constexpr double kFxMagic = 0x1.8p52;
constexpr unsigned long long kFxMagicBits = 0x4338000000000000ull;

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

// Per-track record, kRec doubles per track, blocked by waves of 64 tracks and
// stored in field pairs (2g, 2g + 1): field f of track 64 b + l is
// rec[(b * kRec + (f & ~1)) * 64 + 2 l + (f & 1)], so one 16-byte load per
// lane brings a pair and a wave reads it as one contiguous 1-KB run. Mixed
// Endpoint records of the tabulated medium, whose deposit reads 14 slots,
// keep one field per run instead: rec[(b * kRec + f) * 64 + l], one 8-byte
// load per lane and field (measured: pairs 9% slower there, 6% faster for
// the 12 slots of the exponential medium).
constexpr int kRec = 16;
template <int F, int P>
__host__ __device__ constexpr bool single_slot_records(int medium) {
  return F == 0 && P == 1 && medium == 2;
}
enum : int {
  R_X0, R_Y0, R_Z0, R_T0,  // start point and time
  R_X1, R_Y1, R_Z1, R_T1,  // end point and time
  R_NE0, R_NE1,            // path index of each end to the height of antenna 0
  R_E0, R_E1,              // height factors exp(-(z / h)) of the two ends
  R_AMP,                   // Endpoint: k qw / dt;  ZHS: k qw (t1 - t0) / dt
  R_BX, R_BY, R_BZ         // velocity (units of c)
};
// RT_MIXED records keep slots 0-9 (geometry, times, path indices), pack the
// single-precision fields in pairs, (amplitude, bx) and (by, bz), and keep the
// height factors e0, e1 in double precision in slots 12-13 (the Endpoint
// source index 1 + (n0 - 1) e sits next to the Cherenkov pole, where a
// rounded index would dominate the error). A wave reads 12 of the 16 slots
// (10 without the path indices: uniform medium, spherical Earth), plus the
// height factors where the Endpoint needs the source index in the tabulated
// medium or over the spherical Earth, or a tile antenna sits off the
// reference height. Mixed ZHS records hold the times in bins
// (t / dt) and the path indices over c dt, the operands of
// arrival_bins_scaled.
enum : int { M_AB = 10, M_YZ = 11, M_E0 = 12, M_E1 = 13 };

__device__ __forceinline__ double pack2(float lo, float hi) {
  return __longlong_as_double((long long)(((unsigned long long)__float_as_uint(hi) << 32) |
                                          (unsigned long long)__float_as_uint(lo)));
}
__device__ __forceinline__ float lo32(double d) {
  return __uint_as_float((unsigned)(unsigned long long)__double_as_longlong(d));
}
__device__ __forceinline__ float hi32(double d) {
  return __uint_as_float((unsigned)((unsigned long long)__double_as_longlong(d) >> 32));
}

// Slots a wave loads from a record: the geometry, times, amplitude and
// velocity; the path indices to the reference height only where the deposit
// reads them (not in the uniform medium, whose index is the constant 1 + n0m1,
// nor over the spherical Earth, which takes it per pair); the height factors
// only when H.
template <int P, int MED, bool H>
constexpr bool slot_loaded(int f) {
  if (f == R_NE0 || f == R_NE1) return MED == 1 || MED == 2;
  if (P == 0) return (f == R_E0 || f == R_E1) ? H : true;
  if (f <= M_YZ) return true;
  return H && f <= M_E1;
}

// The two fields of every pair are loaded together or not at all.
template <int P, int MED, bool H>
constexpr bool pairs_agree() {
  for (int g = 0; g < kRec; g += 2)
    if (slot_loaded<P, MED, H>(g) != slot_loaded<P, MED, H>(g + 1)) return false;
  return true;
}

// Writes the record v of lane l into its wave block (single: one field per
// run, see single_slot_records).
__device__ __forceinline__ void store_record(double *blk, int l, const double *v, bool single) {
  if (single) {
#pragma unroll
    for (int f = 0; f < kRec; ++f) blk[f * 64 + l] = v[f];
  } else {
#pragma unroll
    for (int g = 0; g < kRec; g += 2)
      *reinterpret_cast<double2 *>(blk + g * 64 + 2 * l) = make_double2(v[g], v[g + 1]);
  }
}

// Reads the slots of lane l's record that a deposit uses (slot_loaded), one
// pair per load; the other slots read as 0. The lane's byte offset in the
// 8-KB block is formed in 32 bits.
template <int P, int MED, bool H>
__device__ __forceinline__ void load_record_pairs(const double *blk, int l, double *v) {
  static_assert(pairs_agree<P, MED, H>(), "records are loaded a whole pair at a time");
#pragma unroll
  for (int g = 0; g < kRec; g += 2) {
    if (slot_loaded<P, MED, H>(g)) {
      const double2 d = *reinterpret_cast<const double2 *>(
          reinterpret_cast<const char *>(blk) + (unsigned)(g * 512 + 16 * l));
      v[g] = d.x;
      v[g + 1] = d.y;
    } else {
      v[g] = v[g + 1] = 0.0;
    }
  }
}

// Builds the record of one track (fields as above). A track with any
// non-finite field gets NaN times so that no antenna window accepts it.
// z_ref, e_ref: height of antenna 0 and its path factor. In non-uniform media
// the "height factor" slots hold local_factor (n = 1 + n0m1 * it at the end
// point): exp(-(z / h)), tabulated f(z), or over the spherical Earth
// exp(-(H(P) / h)).
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
  if (c.medium == 3) {
    // spherical Earth: the path index depends on the whole antenna position
    // and is taken per pair by the deposit
    v[R_E0] = sph_factor(v[R_X0], v[R_Y0], v[R_Z0], c);
    v[R_E1] = sph_factor(v[R_X1], v[R_Y1], v[R_Z1], c);
  } else if (c.medium != 0) {
    v[R_E0] = local_factor(v[R_Z0], c);
    v[R_E1] = local_factor(v[R_Z1], c);
    const double p0 = c.medium == 2 ? tab_F(v[R_Z0], c) : v[R_E0];
    const double p1 = c.medium == 2 ? tab_F(v[R_Z1], c) : v[R_E1];
    v[R_NE0] = path_index(v[R_Z0], z_ref, p0, e_ref, c);
    v[R_NE1] = path_index(v[R_Z1], z_ref, p1, e_ref, c);
  }
  if (P == 1) {
    const double amp = v[R_AMP], bx = v[R_BX], by = v[R_BY], bz = v[R_BZ];
    const double e0 = v[R_E0], e1 = v[R_E1];
    v[M_AB] = pack2((float)amp, (float)bx);
    v[M_YZ] = pack2((float)by, (float)bz);
    v[M_E0] = e0;
    v[M_E1] = e1;
    v[14] = v[15] = 0.0;
    if (F == 1) {
      const double k = c.inv_c * c.inv_dt;
      v[R_T0] *= c.inv_dt;
      v[R_T1] *= c.inv_dt;
      v[R_NE0] *= k;
      v[R_NE1] *= k;
    }
  }
}

// Bound on the values a ZHS box of one track (mixed record v) rounds at any
// antenna of the box [xlo, xhi] x [ylo, yhi] x [zlo, zhi]: its three levels
// are at most |Ibar| = |cz| |beta_perp| / R_m per component, and R_m
// (midpoint to antenna) is at least the midpoint's distance to the box.
// Factor 1.01 covers the rounding of the deposit arithmetic.
// Infinite when the midpoint lies in the box or more than 1e100 m from it (a
// distance whose square would overflow the deposit geometry); 0 for a track
// that deposits nothing (zero amplitude, or NaN times).
__device__ __forceinline__ double zhs_track_bound(const double *v, const double *bb) {
  const double cz = fabs((double)lo32(v[M_AB]));
  const double bx = hi32(v[M_AB]), by = lo32(v[M_YZ]), bz = hi32(v[M_YZ]);
  if (cz == 0.0 || isnan(v[R_T0])) return 0.0;
  const double mx = (v[R_X0] + v[R_X1]) * 0.5, my = (v[R_Y0] + v[R_Y1]) * 0.5,
               mz = (v[R_Z0] + v[R_Z1]) * 0.5;
  const double ox = fmax(fmax(bb[0] - mx, mx - bb[1]), 0.0);
  const double oy = fmax(fmax(bb[2] - my, my - bb[3]), 0.0);
  const double oz = fmax(fmax(bb[4] - mz, mz - bb[5]), 0.0);
  const double d2 = ox * ox + oy * oy + oz * oz;
  if (!(d2 > 0.0 && d2 < 1e200)) return __builtin_inf();
  return 1.01 * cz * sqrt(bx * bx + by * by + bz * bz) / sqrt(d2);
}

// The antennas' bounding box {xmin, xmax, ymin, ymax, zmin, zmax} over a
// workgroup of NT threads (red: 6 NT doubles of LDS); every thread gets it.
template <int NT>
__device__ __forceinline__ void antenna_bbox(const AntPtrs &an, double *red, double bb[6]) {
  double v[6] = {__builtin_inf(), -__builtin_inf(), __builtin_inf(), -__builtin_inf(),
                 __builtin_inf(), -__builtin_inf()};
  for (int64_t a = threadIdx.x; a < an.m; a += NT) {
    const double x = an.x[a], y = an.y[a], z = an.z[a];
    v[0] = fmin(v[0], x); v[1] = fmax(v[1], x);
    v[2] = fmin(v[2], y); v[3] = fmax(v[3], y);
    v[4] = fmin(v[4], z); v[5] = fmax(v[5], z);
  }
  for (int k = 0; k < 6; ++k) red[k * NT + threadIdx.x] = v[k];
  __syncthreads();
  for (int h = NT / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h)
      for (int k = 0; k < 6; ++k) {
        double &r = red[k * NT + threadIdx.x];
        const double o = red[k * NT + threadIdx.x + h];
        r = (k & 1) ? fmax(r, o) : fmin(r, o);
      }
    __syncthreads();
  }
  for (int k = 0; k < 6; ++k) bb[k] = red[k * NT];
  __syncthreads();
}

// The fixed-point unit of a call (or of a batched shower) from the sum S and
// the maximum B of its n_tracks tracks' deposit bounds (zhs_track_bound),
// reduced in a fixed order so that the unit depends only on the tracks: the
// smallest power of two with
//  - no int64 bin of any tile, split partial or merge sum overflowing: what
//    a track adds to one bin (all four deposits in the folded first bin of
//    a segment) is a signed sum of the rounded levels that reach a bin, at
//    most 2 (r1 + r2 + r3) <= 6 (bound / unit + 1/2) in absolute value, and
//    6.06 S / unit <= 2^62 leaves room for the halves of 2^31 tracks (the
//    sums wrap modulo 2^64, so only the final values need to fit);
//  - every level that reaches a bin in the exact range of the rounding FMA:
//    B / unit < 2^50 (a two-bin box's middle level cancels out of its bin).
// 0 (keep the double-precision tile) when that unit would be coarser than
// 2^-30 of the mean track bound (one dominant track, or more than about 2^28
// tracks) or no finite bound exists; 1 when nothing deposits.
__device__ __forceinline__ double fx_unit(double S, double B, int64_t n_tracks) {
  if (S == 0.0) return 1.0;
  if (!(S < 1e300 && B > 0.0)) return 0.0;
  const int e = max(ilogb(6.06 * S) + 1 - 62, ilogb(B) + 1 - 50);
  if (e > -1000 && e < 1000 && ldexp(1.0, e) <= ldexp(S / (double)n_tracks, -30))
    return ldexp(1.0, e);
  return 0.0;
}

// Adds (vx, vy, vz) to the three components at p (bin j of a tile row, from
// lds_bin).
__device__ __forceinline__ void put3(lds<acc_t> *p, double vx, double vy, double vz) {
  lds_add(p, vx);
  lds_add(p + 1, vy);
  lds_add(p + 2, vz);
}

__device__ __forceinline__ lds<unsigned long long> *as_u64(lds<acc_t> *p) {
  return reinterpret_cast<lds<unsigned long long> *>(p);
}

// Biased fixed-point rounding: the bits of fma(v, s, kFxMagic), which are
// kFxMagicBits + round(v s) for |v s| < 2^51, so that the difference of two
// of them is the exact difference of the rounded integers.
__device__ __forceinline__ unsigned long long fx_biased(double v, double s) {
  return (unsigned long long)__double_as_longlong(fma(v, s, kFxMagic));
}

// Local index at an emission point P from the exponential medium's path
// index n_eff to an antenna X (dz = z_X - z_P, the offset the timing forms;
// ns_x = 1 + n0m1 e_X, inv_h = 1 / h): inverting n_eff = 1 + n0m1 h (e_P -
// e_X) / dz gives 1 + n0m1 e_P = ns_x + (n_eff - 1) dz / h. Below the 1-mm
// branch, where n_eff - 1 = n0m1 e((z_P + z_X) / 2), the same expression
// misses 1 + n0m1 e_P by n0m1 e_X (dz / h)^3 / 24, below 1e-22. The result
// differs from 1 + n0m1 e_P by a few units in the last place.
__device__ __forceinline__ double source_from_path(double neff, double dz, double ns_x,
                                                   double inv_h) {
  return fma(neff - 1.0, dz * inv_h, ns_x);
}

// Endpoint impulse of one track end at one antenna: s k qw [r x (r x beta)] /
// ((1 - n_src beta.r) R dt), evaluated as sc (d (beta.d) / R^2 - beta) / num
// with num = R - n_src (beta.d) = (1 - n_src beta.r) R and sc = s k qw / dt.
template <int P>
__device__ __forceinline__ void endpoint_amp(lds<acc_t> *row, int lo, double lo_d, double hi_d,
                                             double u, double sc, double dx, double dy, double dz,
                                             double r, double r2, double nsrc, double bx,
                                             double by, double bz) {
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
    // RT_MIXED: refined reciprocals. The hardware estimate of 1 / num (4.6e-8)
    // is 2% faster but raised the worst antenna's error from 6e-8 to 3.6e-7:
    // a bin's start and end impulses largely cancel, and an error relative
    // to each impulse is not small relative to their sum.
    q = bd * fast_rcp(r2);
    a = sc * fast_rcp(num);
  }
  put3(lds_bin(row, j), fma(dx, q, -bx) * a, fma(dy, q, -by) * a, fma(dz, q, -bz) * a);
}

// ZHS box of one segment at one antenna. us, ue: arrival of start and end in
// bins; (dx0, dy0, dz0), (dx1, dy1, dz1): antenna minus start and end point.
// The box [u_lo, u_hi] of time integral I = k qw beta_perp (t1-t0) /
// R_mid has bin averages Ibar * overlap / (u_hi - u_lo), Ibar = I / dt; it is
// deposited as at most four differences whose prefix sum is that average,
// each bounded by |Ibar|. Differences before the segment [lo, hi) land in the
// row's two front padding bins (the first bin is clamped to lo - 2 first) and
// are folded into its first bin at the flush (its prefix scan starts there);
// those at or past its end land in the row's back padding (the last bin is
// clamped to hi first, so they reach at most hi + 1). cz2 = 2 k qw (t1 - t0) / dt (times the inverse unit for
// fixed-point deposits, FX).
template <int P, bool FX>
__device__ __forceinline__ void zhs_box(lds<acc_t> *row, int lo, double lo_d, double hi_d,
                                        double us, double ue, double dx0, double dy0, double dz0,
                                        double dx1, double dy1, double dz1, double cz2, double bx,
                                        double by, double bz) {
  // an invalid track's ends are both NaN (NaN times), so ulo and uhi are NaN
  // and the window test below rejects the box
  const double ulo = fmin(us, ue), uhi = fmax(us, ue);
  if (!(uhi >= lo_d && ulo < hi_d)) return;   // outside this segment (or NaN)
  // midpoint geometry from e = (X - P0) + (X - P1) = 2 (X - M), the end
  // offsets the timing computed: with r = 1 / |e| = 1 / (2 R_m),
  // beta_perp = beta - e (beta.e) r^2 and Ibar = cz beta_perp / R_m =
  // cz2 r beta_perp
  double ex = dx0 + dx1, ey = dy0 + dy1, ez = dz0 + dz1;
  double e2 = fma(ex, ex, fma(ey, ey, ez * ez));
  if (e2 == 0.0) return;
  // RT_MIXED: 1 / R_m and 1 / width from the hardware estimates (relative
  // errors at most 5.3e-8 and 4.6e-8, a single-precision amplitude's
  // accuracy); the arrival times stay double
  double rinv = P == 0 ? 1.0 / sqrt(e2) : __builtin_amdgcn_rsq(e2);
  double q = fma(bx, ex, fma(by, ey, bz * ez)) * (rinv * rinv);
  double s = cz2 * rinv;
  double ix = fma(-ex, q, bx) * s, iy = fma(-ey, q, by) * s, iz = fma(-ez, q, bz) * s;
  double kl = floor(ulo), kh = floor(uhi);
  const bool one = kl == kh, two = kh == kl + 1.0;
  double w = uhi - ulo;
  double wi = P == 0 ? 1.0 / w : __builtin_amdgcn_rcp(w);
  double flo = (kl + 1.0) - ulo;   // share of bin kl, in (0, 1]
  double fhi = uhi - kh;           // share of bin kh, in [0, 1)
  double a = flo * wi, bb = fhi * wi;
  const double t2 = (1.0 - flo) * wi, t3 = (1.0 - fhi) * wi;
  double s1 = one ? 1.0 : a;
  double s2 = one ? -1.0 : (two ? -a : t2);
  double s3 = two ? bb : -t3;
  double s4 = -bb;
  // kl <= hi - 1 (the box starts before the segment end), lo <= jh <= hi,
  // and differences before the segment (jl = -2 or -1) go to the row's front
  // padding, which the flush folds into the first bin
  // (the clamps as single v_max_f64 / v_min_f64: fmax and fmin would quiet
  // each operand not known to be a number first, the loop-invariant bounds
  // included, on every pair; none of the four is NaN here)
  const double lo_m2 = lo_d - 2.0;
  double cl, ch;
  asm("v_max_f64 %0, %1, %2" : "=v"(cl) : "v"(kl), "v"(lo_m2));
  asm("v_min_f64 %0, %1, %2" : "=v"(ch) : "v"(kh), "v"(hi_d));
  const int jl = (int)cl - lo;
  const int jh = (int)ch - lo;
  lds<acc_t> *p1 = lds_bin(row, jl);   // jl >= -2: the row's front padding
  lds<acc_t> *p2 = p1 + 3;
  lds<acc_t> *p3 = lds_bin(row, jh);
  if (FX) {
    // Fixed point: the bin averages are the rounded levels r(l1 I) (bin
    // kl), r(l2 I) (the whole bins between) and r(l3 I) (bin kh), deposited
    // as their exact integer differences, so that every box's deposits
    // telescope to zero after its last bin (no rounding residue reaches the
    // bins beyond it, whatever the segmentation). A one-bin box has l1 = 1,
    // l2 = 0. A two-bin box has no whole bin between: its p2 and p3 deposits
    // fall into the same bin (kl + 1 = kh, clamps included), where l2 drops
    // out of their wrapping int64 sum, so it takes l2 = wi like a wider box
    // (wi may exceed 1 there; every level that reaches a bin is at most 1).
    // The p2 difference is issued before the p1 level so that b1 can be
    // rebased in place.
    const double l1 = one ? 1.0 : a, l2 = one ? 0.0 : wi, l3 = bb;
    const double v[3] = {ix, iy, iz};
    unsigned long long b1[3], b2[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      b1[k] = fx_biased(v[k], l1);
      b2[k] = fx_biased(v[k], l2);
      lds_add(as_u64(p2) + k, b2[k] - b1[k]);
      lds_add(as_u64(p1) + k, b1[k] - kFxMagicBits);
    }
    if (!one) {
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const unsigned long long b3 = fx_biased(v[k], l3);
        lds_add(as_u64(p3) + k, b3 - b2[k]);
        lds_add(as_u64(p3) + 3 + k, kFxMagicBits - b3);
      }
    }
  } else {
    put3(p1, ix * s1, iy * s1, iz * s1);
    put3(p2, ix * s2, iy * s2, iz * s2);
    if (!one) {
      put3(p3, ix * s3, iy * s3, iz * s3);
      put3(p3 + 3, ix * s4, iy * s4, iz * s4);
    }
  }
}

// The tile antennas of one workgroup (uniform values).
template <int AT>
struct Tile {
  double ax[AT], ay[AT], az[AT], tau[AT], ea[AT];
  double taub[AT];   // window opening in bins, tau / dt
  double nsa[AT];    // exponential medium: local index at the antenna, 1 + n0m1 ea
  double inv_h;      // exponential medium: 1 / scale height
  bool at_ref[AT];   // at the height of antenna 0: the record's path index applies
};

// Where one workgroup deposits: its LDS tile (rows of `stride` doubles, one
// per tile antenna), the bin segment [lo, hi) the rows hold, and for
// fixed-point tiles the call's inverse unit.
struct TileRef {
  lds<acc_t> *tile;
  int stride;        // doubles per row: (segment bins + tile_pad) * 3
  int lo;            // first bin of the segment
  double lo_d, hi_d;
  double fx_inv;     // fixed-point tiles: 1 / unit (a power of two)
  int front;         // doubles before bin 0 of a row: tile_front * 3
  __device__ __forceinline__ lds<acc_t> *row(int a) const {
    return lds_elem(tile, (unsigned)(a * stride + front));
  }
};

// Element i of a flushed row (its bin 0 at src): the first bin's three
// components take the two front padding bins before them.
template <typename A>
__device__ __forceinline__ A fold_front(const lds<A> *src, int i, int front) {
  A v = src[i];
  if (front > 0 && i < 3) v += src[i - 3] + src[i - 6];
  return v;
}

// All deposits of one track record (this lane's track) into the tile
// antennas selected by mask (a one-antenna tile always holds its antenna).
// H: the height factors were loaded (deposit_blocks loads them where they are
// used). FX: fixed-point ZHS tile.
// Nodes: where the spherical path mean reads its quadrature nodes.
template <int F, int P, int MED, int AT, bool H, bool FX, class Nodes>
__device__ __forceinline__ void deposit_record(const double *v, uint64_t mask, const Tile<AT> &t,
                                               const TileRef &tr, const Consts &c,
                                               const Nodes &nd) {
  const double x0 = v[R_X0], y0 = v[R_Y0], z0 = v[R_Z0], t0 = v[R_T0];
  const double x1 = v[R_X1], y1 = v[R_Y1], z1 = v[R_Z1], t1 = v[R_T1];
  constexpr bool kOff = MED != 0 && H;   // off-reference antennas can be handled
  double amp, bx, by, bz, e0 = 0.0, e1 = 0.0;
  if (P == 0) {
    amp = v[R_AMP];
    bx = v[R_BX];
    by = v[R_BY];
    bz = v[R_BZ];
    if (MED != 0 && H) {
      e0 = v[R_E0];
      e1 = v[R_E1];
    }
  } else {
    amp = lo32(v[M_AB]);
    bx = hi32(v[M_AB]);
    by = lo32(v[M_YZ]);
    bz = hi32(v[M_YZ]);
    if (kOff) {
      e0 = v[M_E0];
      e1 = v[M_E1];
    }
  }
  // ZHS: the box takes twice its amplitude constant (times the inverse unit
  // for fixed-point tiles; all exact powers of two)
  if (F == 1) amp *= FX ? 2.0 * tr.fx_inv : 2.0;
  // mixed Endpoint, exponential medium, tile at the reference height: the
  // source index comes from the record's path index (no height-factor slots)
  constexpr bool kNsFromPath = F == 0 && P == 1 && MED == 1 && !H;
  double ns0 = MED != 0 ? fma(c.n0m1, e0, 1.0) : c.n_uniform;
  double ns1 = MED != 0 ? fma(c.n0m1, e1, 1.0) : c.n_uniform;
#pragma unroll
  for (int a = 0; a < AT; ++a) {
    if (AT == 1 || ((mask >> a) & 1)) {
      double ne0 = MED == 0 ? c.n_uniform : v[R_NE0];
      double ne1 = MED == 0 ? c.n_uniform : v[R_NE1];
      if (MED == 3) {
        ne0 = sph_path_index(x0, y0, z0, t.ax[a], t.ay[a], t.az[a], c, nd);
        ne1 = sph_path_index(x1, y1, z1, t.ax[a], t.ay[a], t.az[a], c, nd);
      } else if (kOff && !t.at_ref[a]) {
        const double p0 = MED == 2 ? tab_F(z0, c) : e0;
        const double p1 = MED == 2 ? tab_F(z1, c) : e1;
        ne0 = path_index_m<MED>(z0, t.az[a], p0, t.ea[a], c);
        ne1 = path_index_m<MED>(z1, t.az[a], p1, t.ea[a], c);
      }
      lds<acc_t> *row = tr.row(a);
      if constexpr (F == 1 && P == 1) {
        // times in bins, path indices over c dt (make_record); the indices
        // taken here are plain
        if (MED == 0 || MED == 3 || (kOff && !t.at_ref[a])) {
          ne0 *= c.inv_c * c.inv_dt;
          ne1 *= c.inv_c * c.inv_dt;
        }
        double dx0, dy0, dz0, dx1, dy1, dz1;
        const double u0 = arrival_bins_scaled(x0, y0, z0, t0, t.ax[a], t.ay[a], t.az[a],
                                              t.taub[a], ne0, dx0, dy0, dz0);
        const double u1 = arrival_bins_scaled(x1, y1, z1, t1, t.ax[a], t.ay[a], t.az[a],
                                              t.taub[a], ne1, dx1, dy1, dz1);
        zhs_box<P, FX>(row, tr.lo, tr.lo_d, tr.hi_d, u0, u1, dx0, dy0, dz0, dx1, dy1, dz1, amp,
                       bx, by, bz);
        continue;
      }
      double dx0, dy0, dz0, r0, q0, dx1, dy1, dz1, r1, q1;
      const double u0 = arrival_bins(x0, y0, z0, t0, t.ax[a], t.ay[a], t.az[a], t.tau[a], ne0, c,
                                     dx0, dy0, dz0, r0, q0);
      const double u1 = arrival_bins(x1, y1, z1, t1, t.ax[a], t.ay[a], t.az[a], t.tau[a], ne1, c,
                                     dx1, dy1, dz1, r1, q1);
      if constexpr (kNsFromPath) {
        ns0 = source_from_path(ne0, dz0, t.nsa[a], t.inv_h);
        ns1 = source_from_path(ne1, dz1, t.nsa[a], t.inv_h);
      }
      if (F == 0) {
        endpoint_amp<P>(row, tr.lo, tr.lo_d, tr.hi_d, u0, amp, dx0, dy0, dz0, r0, q0, ns0, bx, by,
                        bz);
        endpoint_amp<P>(row, tr.lo, tr.lo_d, tr.hi_d, u1, -amp, dx1, dy1, dz1, r1, q1, ns1, bx,
                        by, bz);
      } else {
        zhs_box<P, FX>(row, tr.lo, tr.lo_d, tr.hi_d, u0, u1, dx0, dy0, dz0, dx1, dy1, dz1, amp, bx,
                       by, bz);
      }
    }
  }
}

// Reads the slots of lane l's record in wave block blk that a deposit uses.
template <int F, int P, int MED, bool H>
__device__ __forceinline__ void load_record(const double *rec, int64_t blk, int lane, double *rv) {
  if constexpr (single_slot_records<F, P>(MED)) {
    const double *r = rec + blk * (kRec * 64) + lane;
#pragma unroll
    for (int f = 0; f < kRec; ++f) rv[f] = slot_loaded<P, MED, H>(f) ? r[f * 64] : 0.0;
  } else {
    load_record_pairs<P, MED, H>(rec + blk * (kRec * 64), lane, rv);
  }
}

// Deposits of the wave blocks [b_first, b_end) (stride `waves`, one block per
// wave per step) of a record array into the LDS tile. Only the slots the
// formalism and precision use are read. PF: kPfNext loads the next record
// before processing the current one (one buffer, copied); kPfAlternate does
// so, for mixed records without height factors, into the other of two record
// buffers (the loop takes two blocks per turn: no copies, more registers).
// That pays where record latency shows (the Endpoint deposit), few waves
// share a SIMD (the 512-thread batch kernel), or, with alternating buffers,
// for the one-antenna mixed ZHS deposit; with a copied buffer the single-plan
// ZHS deposit runs faster without it.
enum : int { kPfNone = 0, kPfNext = 1, kPfAlternate = 2 };

template <int F, int P, int MED, int AT, bool H, int PF, bool FX, class Nodes>
__device__ __forceinline__ void deposit_blocks_n(const double *rec, int64_t b_first,
                                                 int64_t b_end, int64_t waves, uint64_t mask,
                                                 const Tile<AT> &t, const TileRef &tr,
                                                 const Consts &c, const Nodes &nd) {
  const int lane = threadIdx.x & 63;
  // block indices in 32 bits (a call holds at most 2^31 tracks, 2^25 blocks):
  // with a wave-uniform b_first the loop tests are scalar compares
  const int bf = (int)b_first, be = (int)b_end, wv = (int)waves;
  constexpr bool kAlt = PF == kPfAlternate && P == 1 && !H;
  // ZHS deposits prefetch only into alternating buffers: with a copied
  // buffer they ran slower than with none
  constexpr bool kCopy = !kAlt && (PF == kPfNext || (PF == kPfAlternate && F == 0));
  if (!kAlt && !kCopy) {
    for (int blk = bf; blk < be; blk += wv) {
      double rv[kRec];
      load_record<F, P, MED, H>(rec, blk, lane, rv);
      deposit_record<F, P, MED, AT, H, FX>(rv, mask, t, tr, c, nd);
    }
    return;
  }
  if constexpr (kAlt) {
    double ra[kRec], rb[kRec];
#pragma unroll
    for (int f = 0; f < kRec; ++f) ra[f] = rb[f] = 0.0;
    if (bf < be) load_record<F, P, MED, H>(rec, bf, lane, ra);
    for (int blk = bf; blk < be; blk += 2 * wv) {
      if (blk + wv < be) load_record<F, P, MED, H>(rec, blk + wv, lane, rb);
      deposit_record<F, P, MED, AT, H, FX>(ra, mask, t, tr, c, nd);
      if (blk + wv >= be) break;
      if (blk + 2 * wv < be) load_record<F, P, MED, H>(rec, blk + 2 * wv, lane, ra);
      deposit_record<F, P, MED, AT, H, FX>(rb, mask, t, tr, c, nd);
    }
  } else {
    // the deposits that read the height factors, the FP64 ones and the batch
    // kernels need the registers the second buffer would take (they spill
    // with it): one buffer, copied
    double nx[kRec];
#pragma unroll
    for (int f = 0; f < kRec; ++f) nx[f] = 0.0;
    if (bf < be) load_record<F, P, MED, H>(rec, bf, lane, nx);
    for (int blk = bf; blk < be; blk += wv) {
      double rv[kRec];
#pragma unroll
      for (int f = 0; f < kRec; ++f) rv[f] = nx[f];
      if (blk + wv < be) load_record<F, P, MED, H>(rec, blk + wv, lane, nx);
      deposit_record<F, P, MED, AT, H, FX>(rv, mask, t, tr, c, nd);
    }
  }
}

// As deposit_blocks_n, reading the height factors only where they are used:
// the Endpoint source index (except for mixed records in the exponential
// medium, where it follows from the path index; the FP64 deposit, which
// spends more of its time in arithmetic, keeps the two slots: 6% faster), and
// tiles with an antenna off the reference height (whose path index is taken
// per pair from them).
template <int F, int P, int MED, int AT, int PF, bool FX, class Nodes>
__device__ __forceinline__ void deposit_blocks(const double *rec, int64_t b_first, int64_t b_end,
                                               int64_t waves, uint64_t mask, const Tile<AT> &t,
                                               const TileRef &tr, const Consts &c,
                                               const Nodes &nd) {
  bool off = false;
#pragma unroll
  for (int a = 0; a < AT; ++a) off = off || (((mask >> a) & 1) && !t.at_ref[a]);
  if (MED == 3 ? F == 0 : MED != 0 && ((F == 0 && (MED != 1 || P == 0)) || off))
    deposit_blocks_n<F, P, MED, AT, true, PF, FX>(rec, b_first, b_end, waves, mask, t, tr, c, nd);
  else
    deposit_blocks_n<F, P, MED, AT, false, PF, FX>(rec, b_first, b_end, waves, mask, t, tr, c, nd);
}

// Loads the tile antennas [a_begin, a_begin + n_ant) (uniform per workgroup).
template <int AT, int MED>
__device__ __forceinline__ void load_tile(const AntPtrs &an, int64_t a_begin, int n_ant,
                                          const Consts &c, Tile<AT> &t) {
  const double z_ref = an.z[0];
  t.inv_h = MED == 1 ? 1.0 / c.h : 0.0;
#pragma unroll
  for (int a = 0; a < AT; ++a) {
    int64_t ai = a_begin + (a < n_ant ? a : 0);
    t.ax[a] = an.x[ai];
    t.ay[a] = an.y[ai];
    t.az[a] = an.z[ai];
    t.tau[a] = an.t_start[ai];
    t.taub[a] = t.tau[a] * c.inv_dt;
    t.ea[a] = MED == 1 || MED == 2 ? path_factor_m<MED>(t.az[a], c) : 0.0;
    t.nsa[a] = fma(c.n0m1, t.ea[a], 1.0);
    t.at_ref[a] = t.az[a] == z_ref;
  }
}

// ------------------------------------------------------------------ merge

constexpr int kMergeThreads = 256;

// traces[0, nb) += the sum over `splits` partial slots (`stride` elements
// apart, added in slot order) of one segment, 3 components per bin, times
// `unit` (the value of one partial unit: 1 for double partials, the call's
// fixed-point unit for int64 ones, whose sums and scan are exact). ZHS slots
// hold differences (every box folded into the segment's first bin where it
// starts earlier), so their sum is prefix-scanned over the segment: chunks of
// kMergeThreads bins are summed with coalesced loads into LDS, scanned across
// the workgroup (within each wave by lane shuffles, then over the wave
// totals), offset by the carry of the chunks before, and added to the traces
// with coalesced stores. One workgroup of kMergeThreads threads.
template <int F, typename T, typename A>
__device__ __forceinline__ void merge_segment(const A *part, int64_t stride, int splits, T *out,
                                              int nb, double unit) {
  const int tid = threadIdx.x;
  if (F == 0) {
    for (int i = tid; i < nb * 3; i += kMergeThreads) {
      A s = 0;
      for (int sp = 0; sp < splits; ++sp) s += part[sp * stride + i];
      out[i] = (T)((double)out[i] + (double)s * unit);
    }
    return;
  }
  constexpr int kWaves = kMergeThreads / 64;
  __shared__ A buf[kMergeThreads * 3];
  __shared__ A wsum[kWaves][3];
  const int lane = tid & 63, wave = tid >> 6;
  A carry[3] = {0, 0, 0};
  for (int c0 = 0; c0 < nb; c0 += kMergeThreads) {
    const int n = min(kMergeThreads, nb - c0);
    const A *p = part + 3 * (int64_t)c0;
    for (int i = tid; i < 3 * n; i += kMergeThreads) {
      A s = 0;
      for (int sp = 0; sp < splits; ++sp) s += p[sp * stride + i];
      buf[i] = s;
    }
    __syncthreads();
    A v[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) v[c] = tid < n ? buf[3 * tid + c] : (A)0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        A y = __shfl_up(v[c], off);
        if (lane >= off) v[c] += y;
      }
    }
    if (lane == 63)
      for (int c = 0; c < 3; ++c) wsum[wave][c] = v[c];
    __syncthreads();
    A pre[3], tot[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      pre[c] = carry[c];
      for (int w = 0; w < wave; ++w) pre[c] += wsum[w][c];
      tot[c] = pre[c];
      for (int w = wave; w < kWaves; ++w) tot[c] += wsum[w][c];
    }
    // tot is the same in every wave only up to rounding order (double
    // partials): take wave 0's value (pre = carry there) so that all threads
    // carry the same number
    __syncthreads();
    if (tid < n)
      for (int c = 0; c < 3; ++c) buf[3 * tid + c] = pre[c] + v[c];
    if (tid == 0)
      for (int c = 0; c < 3; ++c) wsum[0][c] = tot[c];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 3; ++c) carry[c] = wsum[0][c];
    T *o = out + 3 * (int64_t)c0;
    for (int i = tid; i < 3 * n; i += kMergeThreads)
      o[i] = (T)((double)o[i] + (double)buf[i] * unit);
    __syncthreads();
  }
}

}  // namespace rt
