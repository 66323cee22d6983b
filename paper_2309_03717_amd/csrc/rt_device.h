// rt_device.h -- device-side building blocks shared by the radtrace kernels:
// launch arguments, the straight-line propagator and the media.
//
// The propagator's timing chain is evaluated in double precision in one fixed
// operation order (the whole library is compiled with -ffp-contract=off), so
// that the arrival bin of every (end, track, antenna) is reproducible
// bit-for-bit by any implementation of the same definition:
//     d = X - P;  R = sqrt((dx*dx + dy*dy) + dz*dz)
//     n_eff = 1 + n0m1                                   (uniform medium)
//     n_eff = 1 + (n0m1*h) * ((eX - eP) / (zP - zX))     (exponential,
//             e = exp(-(z / h)), |zP - zX| >= 1e-3 m)
//     n_eff = 1 + n0m1 * exp(-(((zP + zX) * 0.5) / h))   (|zP - zX| < 1e-3 m)
//     n_eff = 1 + n0m1 * ((F(zP) - F(zX)) / (zP - zX))   (tabulated, F below;
//             1 + n0m1 * f((zP + zX) * 0.5) when |zP - zX| < 1e-3 m)
//     n_eff = 1 + n0m1 * S                               (spherical Earth,
//             S = S + w_k * exp(-(r_k / ((sqrt(r_k + re*re) + re) * h)))
//             summed over the nodes k ascending, r_k = A + s_k * (B + s_k * D),
//             A = (px*px + py*py) + pz * (pz + 2 re),
//             B = 2 * ((px*dx + py*dy) + (pz + re) * dz),
//             D = (dx*dx + dy*dy) + dz*dz)
//     t = T + (n_eff * R) * (1 / c);   u = (t - t_start) * (1 / dt)
//     in the window iff 0 <= u < n_bins; bin = floor(u)
// The exponential form is the mean of n(z) = 1 + n0m1 exp(-z/h) along the
// straight path (§2: the propagator gives the emission path of each pair);
// over a spherical Earth the same mean is taken by Gauss-Legendre quadrature.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rt {

constexpr int kMaxTile = 8;     // antennas per workgroup tile (template bound)
constexpr int64_t kDefaultPass = 1 << 20;   // tracks per deposit pass by default
constexpr int kXcds = 8;        // MI355X: 8 XCDs, workgroups dealt round-robin
constexpr int64_t kZhsSplitBlocks = 2048;   // ZHS track split cap: 128K tracks
constexpr int64_t kEpSplitBlocks = 4096;    // Endpoint track split cap: 256K tracks
constexpr int kGl = 8;          // Gauss-Legendre nodes of the spherical path mean

struct Consts {
  double inv_c;       // 1 / c
  double inv_dt;      // 1 / dt
  double k;           // field prefactor
  double n_uniform;   // 1 + n0m1
  double n0m1, h, n0h;  // n0h = n0m1 * h
  double nbins_d;     // (double) n_bins
  int32_t n_bins;
  int32_t medium;     // 0 uniform, 1 exponential, 2 tabulated, 3 spherical
  // tabulated profile: f at tz0 + i tdz (i < n_tab), and its cumulative
  // integral at the nodes (tabF, or null: summed on the fly)
  const double *tab, *tabF;
  int32_t n_tab;
  double tz0, tdz, tinv_dz;   // tinv_dz = 1 / tdz
  // spherical Earth: radius, its square and twice it; quadrature nodes on
  // [0, 1] (ascending) and weights
  double re, re2, re_twice;
  double gl_s[kGl], gl_w[kGl];
  // non-null: n0 - 1 is read from this device address by every kernel (the
  // n0m1, n0h and n_uniform fields above are then recomputed from it)
  const double *n0m1_dev;
};

// The constants a kernel works with: n0 - 1 and the values derived from it
// (n0h = n0m1 * h, n_uniform = 1 + n0m1, the host's operations) taken from
// device memory when the plan points at it.
__device__ __forceinline__ Consts resolve_consts(const Consts &c0) {
  Consts c = c0;
  if (c.n0m1_dev) {
    const double n = *c.n0m1_dev;
    c.n0m1 = n;
    c.n0h = n * c.h;
    c.n_uniform = 1.0 + n;
  }
  return c;
}

struct TrackPtrs {
  const double *x0, *y0, *z0, *t0, *x1, *y1, *z1, *t1;
  const void *bx, *by, *bz, *qw;
  int64_t n;
};

struct AntPtrs {
  const double *x, *y, *z, *t_start;
  int64_t m;
};

// exp(-(z / h)): the height factor of the exponential profile.
__device__ __forceinline__ double height_factor(double z, const Consts &c) {
  return exp(-(z / c.h));
}

// Tabulated profile: f(z), linear between nodes, constant beyond the ends.
__device__ __forceinline__ double tab_f(double z, const Consts &c) {
  const double t = (z - c.tz0) * c.tinv_dz;
  const int last = c.n_tab - 1;
  if (!(t > 0.0)) return c.tab[0];
  if (t >= (double)last) return c.tab[last];
  const int i = (int)floor(t);
  const double w = t - (double)i;
  return c.tab[i] + w * (c.tab[i + 1] - c.tab[i]);
}

// Trapezoids of the first i cells, summed from the first node up.
__device__ __forceinline__ double tab_cells(int i, const Consts &c) {
  if (c.tabF) return c.tabF[i];
  double acc = 0.0;
  for (int j = 1; j <= i; ++j) acc += (0.5 * c.tdz) * (c.tab[j - 1] + c.tab[j]);
  return acc;
}

// The same sums at every node, written to cells[0 .. n_tab), by one thread.
__device__ __forceinline__ void fill_tab_cells(const Consts &c, double *cells) {
  double acc = 0.0;
  cells[0] = 0.0;
  for (int j = 1; j < c.n_tab; ++j) {
    acc += (0.5 * c.tdz) * (c.tab[j - 1] + c.tab[j]);
    cells[j] = acc;
  }
}

// Tabulated profile: F(z) = integral of f from tz0 to z (exact for the
// piecewise-linear f; slope f at the ends beyond the nodes).
__device__ __forceinline__ double tab_F(double z, const Consts &c) {
  const double t = (z - c.tz0) * c.tinv_dz;
  const int last = c.n_tab - 1;
  if (!(t > 0.0)) return c.tab[0] * (z - c.tz0);
  const int i = t >= (double)last ? last : (int)floor(t);
  const double acc = tab_cells(i, c);
  if (i == last) return acc + c.tab[last] * (z - (c.tz0 + (double)last * c.tdz));
  const double w = t - (double)i;
  return acc + c.tdz * (w * c.tab[i] + (0.5 * w * w) * (c.tab[i + 1] - c.tab[i]));
}

// n(z) - 1 = n0m1 * local_factor(z) (non-uniform media).
__device__ __forceinline__ double local_factor(double z, const Consts &c) {
  return c.medium == 2 ? tab_f(z, c) : height_factor(z, c);
}

// The per-height value path_index takes: the height factor (exponential) or
// the integral F (tabulated).
__device__ __forceinline__ double path_factor(double z, const Consts &c) {
  return c.medium == 2 ? tab_F(z, c) : height_factor(z, c);
}

// Compile-time forms for the deposit kernels (MED: 1 exponential, 2
// tabulated), so that each kernel carries the code of its own medium only.
template <int MED>
__device__ __forceinline__ double path_factor_m(double z, const Consts &c) {
  return MED == 2 ? tab_F(z, c) : height_factor(z, c);
}

template <int MED>
__device__ __forceinline__ double path_index_m(double zp, double za, double pp, double pa,
                                               const Consts &c) {
  double dz = zp - za;
  if (MED == 2) {
    if (fabs(dz) >= 1e-3) return 1.0 + c.n0m1 * ((pp - pa) / dz);
    return 1.0 + c.n0m1 * tab_f((zp + za) * 0.5, c);
  }
  if (fabs(dz) >= 1e-3) return 1.0 + c.n0h * ((pa - pp) / dz);
  return 1.0 + c.n0m1 * exp(-(((zp + za) * 0.5) / c.h));
}

// Path-mean refractive index from emission height zp to an antenna at height
// za, given their path factors pp and pa (non-uniform media).
__device__ __forceinline__ double path_index(double zp, double za, double pp, double pa,
                                             const Consts &c) {
  double dz = zp - za;
  if (c.medium == 2) {
    if (fabs(dz) >= 1e-3) return 1.0 + c.n0m1 * ((pp - pa) / dz);
    return 1.0 + c.n0m1 * tab_f((zp + za) * 0.5, c);
  }
  if (fabs(dz) >= 1e-3) return 1.0 + c.n0h * ((pa - pp) / dz);
  return 1.0 + c.n0m1 * exp(-(((zp + za) * 0.5) / c.h));
}

// 1/x and 1/sqrt(x) from the hardware estimate plus one Newton step, which
// squares the estimate's relative error: measured on gfx950 over 1.3e8
// log-uniform inputs in [1e-6, 1e12], at most 2.2e-15 (fast_rcp) and 4.3e-15
// (fast_rsq), from estimates good to 4.6e-8 and 5.3e-8. The mixed-precision
// Endpoint amplitude and the adjoints use them.
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

// sqrt(x) from the hardware reciprocal square root and one Newton step on
// the root: relative error at most about 1.5 e^2 plus rounding, 4.5e-15 for
// the estimate's e = 5.3e-8; inputs outside (2^-767, inf) take the library
// sqrt, as in sqrt_rn. Not correctly rounded: for arrival times that enter a
// continuous function of the time only (the ZHS box).
__device__ __forceinline__ double sqrt_fast(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  g = fma(g, fma(-0.5 * y, g, 0.5), g);
  if (__builtin_expect(!(x > 0x1p-767 && x < __builtin_inf()), 0)) g = sqrt(x);
  return g;
}

// Correctly rounded sqrt: the hardware reciprocal square root refined by
// Newton steps (the same operations as the compiler's own expansion, without
// its range scaling); inputs outside (2^-767, inf) take the library sqrt.
__device__ __forceinline__ double sqrt_rn(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double g = x * y;
  double h = y * 0.5;
  double r = fma(-h, g, 0.5);
  g = fma(g, r, g);
  double d = fma(-g, g, x);
  h = fma(h, r, h);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  g = fma(d, h, g);
  if (__builtin_expect(!(x > 0x1p-767 && x < __builtin_inf()), 0)) g = sqrt(x);
  return g;
}

// Spherical Earth of radius re centred at (0, 0, -re). For a point q, rho2 =
// |q - C|^2 - re^2 = (x*x + y*y) + z * (z + 2 re), and its height above the
// sphere is H = |q - C| - re = rho2 / (sqrt(rho2 + re^2) + re) (no
// cancellation of two radii); sph_exponent is H / h with one division.
__device__ __forceinline__ double sph_exponent(double rho2, const Consts &c) {
  return rho2 / ((sqrt_rn(rho2 + c.re2) + c.re) * c.h);
}

// exp(-(H(q) / h)): n(q) = 1 + n0m1 * sph_factor(q).
__device__ __forceinline__ double sph_factor(double x, double y, double z, const Consts &c) {
  return exp(-sph_exponent((x * x + y * y) + z * (z + c.re_twice), c));
}

// The quadrature nodes and weights of the spherical path mean as the
// constants hold them (a single plan's kernel arguments).
// Nodes read from a Consts in constant memory: a kernel argument, never a
// kernel's local copy (indexing a local copy by the loop counter puts the whole
// copy in per-lane scratch memory).
struct ConstNodes {
  const Consts &c;
  __device__ __forceinline__ double s(int k) const { return c.gl_s[k]; }
  __device__ __forceinline__ double w(int k) const { return c.gl_w[k]; }
};

// Path mean of n over the straight path from P to the antenna X (spherical
// Earth): 1 + n0m1 * (sum over the nodes of w_k * exp(-(H(q_k) / h))), the
// nodes taken in ascending order. Along q = P + s d (d = X - P), rho2 is the
// quadratic A + s (B + s D) with A = rho2(P), B = 2 (P - C).d, D = d.d.
// Nodes: where the nodes and weights are read from (s(k), w(k)).
template <class Nodes>
__device__ __forceinline__ double sph_path_index(double px, double py, double pz, double ax,
                                                 double ay, double az, const Consts &c,
                                                 const Nodes &nd) {
  const double dx = ax - px, dy = ay - py, dz = az - pz;
  const double qa = (px * px + py * py) + pz * (pz + c.re_twice);
  const double qb = 2.0 * ((px * dx + py * dy) + (pz + c.re) * dz);
  const double qd = (dx * dx + dy * dy) + dz * dz;
  double s = 0.0;
#pragma unroll 1
  for (int k = 0; k < kGl; ++k) {
    const double sk = nd.s(k);
    s = s + nd.w(k) * exp(-sph_exponent(qa + sk * (qb + sk * qd), c));
  }
  return 1.0 + c.n0m1 * s;
}


// Straight-line propagation of an emission at (px,py,pz), time tp, to an
// antenna at (ax,ay,az) whose bin 0 starts at tau. Returns u, the arrival in
// bins; d = X - P, R and R^2 are returned for the amplitude.
__device__ __forceinline__ double arrival_bins(double px, double py, double pz, double tp,
                                               double ax, double ay, double az, double tau,
                                               double neff, const Consts &c, double &dx,
                                               double &dy, double &dz, double &r, double &r2) {
  dx = ax - px;
  dy = ay - py;
  dz = az - pz;
  r2 = (dx * dx + dy * dy) + dz * dz;
  r = sqrt_rn(r2);
  double t = tp + (neff * r) * c.inv_c;
  return (t - tau) * c.inv_dt;
}

// Arrival in bins from an end whose emission time is given in bins (tb = t /
// dt) and whose path index over c dt (nb = n_eff / (c dt)), at an antenna
// whose window opens at taub = t_start / dt: u = nb R + (tb - taub), R^2
// by fused multiply-adds and R from sqrt_fast. Differs from arrival_bins by
// rounding only (a few 1e-15 of u); the deposits that use it are continuous
// in u.
__device__ __forceinline__ double arrival_bins_scaled(double px, double py, double pz, double tb,
                                                      double ax, double ay, double az, double taub,
                                                      double nb, double &dx, double &dy,
                                                      double &dz) {
  dx = ax - px;
  dy = ay - py;
  dz = az - pz;
  return fma(nb, sqrt_fast(fma(dx, dx, fma(dy, dy, dz * dz))), tb - taub);
}

// Arrival time (seconds) by the canonical chain of arrival_bins; used by the
// propagate entry point.
__device__ __forceinline__ double arrival_time(double px, double py, double pz, double tp,
                                               double ax, double ay, double az, double neff,
                                               const Consts &c) {
  double dx = ax - px, dy = ay - py, dz = az - pz;
  double r = sqrt_rn((dx * dx + dy * dy) + dz * dz);
  return tp + (neff * r) * c.inv_c;
}

// Bijection of [0, grid) that gives each XCD a contiguous range of virtual
// block ids (hardware deals workgroup b to XCD b % 8), so workgroups that
// share a track range run on the same XCD and share its L2.
__device__ __forceinline__ int xcd_major(int b, int grid) {
  int per = grid / kXcds, rem = grid % kXcds;
  int x = b % kXcds, j = b / kXcds;
  return x < rem ? x * (per + 1) + j : rem * (per + 1) + (x - rem) * per + j;
}

// LDS (address space 3) objects: pointers to them are 32-bit, so offsets
// into a tile stay in 32-bit arithmetic.
template <class T>
using lds = __attribute__((address_space(3))) T;

// Element i of an LDS array by a 24-bit multiply (i * sizeof(T) < 2^24).
template <class T>
__device__ __forceinline__ lds<T> *lds_elem(lds<T> *base, unsigned i) {
  return (lds<T> *)((lds<char> *)base + __umul24(i, (unsigned)sizeof(T)));
}

// The first of the three components of bin j of a trace row (|24 j
// sizeof(T) / 8| < 2^23; j may be negative where the row has front padding):
// one signed 24-bit multiply.
template <class T>
__device__ __forceinline__ lds<T> *lds_bin(lds<T> *row, int j) {
  return (lds<T> *)((lds<char> *)row + __mul24(j, 3 * (int)sizeof(T)));
}

template <typename T>
__device__ __forceinline__ void lds_add(lds<T> *p, T v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

}  // namespace rt
