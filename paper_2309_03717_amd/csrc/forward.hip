// forward.hip -- the track x antenna loop on gfx950: per-track media values,
// LDS-resident antenna trace tiles fed by streamed tracks, fixed-order merge
// of track-split partials (with the ZHS prefix scan), and the propagator
// alone.
//
// Work decomposition (the analogue of §4's "bunch of antennas" per task): a
// workgroup owns a tile of up to kMaxTile antennas x one segment of bins in
// LDS and streams one range ("split") of the tracks past it; each lane takes
// one track and loops over the tile's antennas, so the track loads are
// coalesced structure-of-arrays reads and each deposit is an LDS atomic add.
// The tile is then written once to a partial buffer [split][M][B][3] and a
// second kernel sums the splits in index order into the caller's traces, so
// no float atomic ever touches global memory and a fixed tiling gives the
// same merge order on every call.
#include "rt_internal.h"

namespace rt {

// Accumulation in LDS and in the split partials is double precision in both
// modes: gfx950 executes LDS double-precision atomic adds (ds_add_f64) at
// close to the rate of plain LDS stores, while single-precision ones
// (ds_add_f32) are several times slower on this workload.
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

struct DepositArgs {
  TrackPtrs tr;
  AntPtrs an;
  Consts c;
  const double *e0, *e1;   // per-track height factors (exponential medium)
  void *partial;           // [splits][M][n_bins][3]
  int64_t per_split;       // tracks per split
  int n_atiles, n_segs, seg_len;
};

// ------------------------------------------------------------------ prepare

// Height factors exp(-(z / h)) of both track ends, once per call instead of
// once per workgroup.
__global__ void __launch_bounds__(256) prepare_kernel(TrackPtrs tr, Consts c, double *e0,
                                                      double *e1) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < tr.n;
       i += (int64_t)gridDim.x * blockDim.x) {
    e0[i] = height_factor(tr.z0[i], c);
    e1[i] = height_factor(tr.z1[i], c);
  }
}

// ------------------------------------------------------------------ deposits

template <typename T>
__device__ __forceinline__ void put3(T *row, int j, T vx, T vy, T vz) {
  T *p = row + 3 * j;
  lds_add(p, vx);
  lds_add(p + 1, vy);
  lds_add(p + 2, vz);
}

// ZHS difference deposit at absolute bin j of a segment [lo, hi): bins before
// the segment fold into its first bin (the segment's prefix scan starts
// there), bins at or after its end are dropped.
template <typename T>
__device__ __forceinline__ void put3_clamped(T *row, int j, int lo, int hi, T vx, T vy, T vz) {
  if (j < lo) j = lo;
  if (j < hi) put3(row, j - lo, vx, vy, vz);
}

// Endpoint impulse of one track end at one antenna: s k qw [r x (r x beta)] /
// ((1 - n_src beta.r) R dt), written as sc * (d (beta.d) / R^2 - beta) / num
// with num = R - n_src (beta.d) = (1 - n_src beta.r) R and sc = s k qw / dt.
template <int P>
__device__ __forceinline__ void endpoint_end(acc_t *row, int lo, int hi, double sc,
                                             double px, double py, double pz, double tp,
                                             double ax, double ay, double az, double tau,
                                             double neff, double nsrc, double bx, double by,
                                             double bz, const Consts &c) {
  using T = acc_t;
  double dx, dy, dz, r;
  double u = arrival_bins(px, py, pz, tp, ax, ay, az, tau, neff, c, dx, dy, dz, r);
  if (!(u >= 0.0 && u < c.nbins_d)) return;
  int kb = (int)u;
  if (kb < lo || kb >= hi) return;
  double bd = (bx * dx + by * dy) + bz * dz;
  double num = r - nsrc * bd;
  if (num == 0.0) return;   // on the Cherenkov cone, or R = 0
  if (P == 0) {
    double q = bd / (r * r);
    double a = sc / num;
    put3<T>(row, kb - lo, (T)((dx * q - bx) * a), (T)((dy * q - by) * a), (T)((dz * q - bz) * a));
  } else {
    float fr = (float)r;
    float q = (float)bd * __builtin_amdgcn_rcpf(fr * fr);
    float a = (float)sc * __builtin_amdgcn_rcpf((float)num);
    float vx = fmaf((float)dx, q, -(float)bx);
    float vy = fmaf((float)dy, q, -(float)by);
    float vz = fmaf((float)dz, q, -(float)bz);
    put3<T>(row, kb - lo, (T)(vx * a), (T)(vy * a), (T)(vz * a));
  }
}

// ZHS box of one segment at one antenna. us, ue: arrival of start and end in
// bins. The box [u_lo, u_hi] of time integral I = k qw beta_perp (t1-t0) /
// R_mid has bin averages Ibar * overlap / (u_hi - u_lo), Ibar = I / dt; it is
// deposited as at most four differences whose prefix sum is that average,
// each bounded by |Ibar|.
template <int P>
__device__ __forceinline__ void zhs_box(acc_t *row, int lo, int hi, double us, double ue,
                                        double mx, double my, double mz, double ax, double ay,
                                        double az, double cz, double bx, double by, double bz) {
  // T: arithmetic type of the amplitudes (deposits are widened to acc_t)
  using T = typename Prec<P>::out;
  double ulo = us < ue ? us : ue;
  double uhi = us < ue ? ue : us;
  if (!(uhi >= (double)lo && ulo < (double)hi)) return;   // outside this segment (or NaN)
  // midpoint geometry: Ibar = cz * beta_perp / R_m, cz = k qw (t1 - t0) / dt
  T ix, iy, iz;
  if (P == 0) {
    double dx = ax - mx, dy = ay - my, dz = az - mz;
    double r2 = (dx * dx + dy * dy) + dz * dz;
    if (r2 == 0.0) return;
    double rm = sqrt(r2);
    double q = ((bx * dx + by * dy) + bz * dz) / r2;
    double s = cz / rm;
    ix = (bx - dx * q) * s;
    iy = (by - dy * q) * s;
    iz = (bz - dz * q) * s;
  } else {
    float dx = (float)(ax - mx), dy = (float)(ay - my), dz = (float)(az - mz);
    float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
    if (r2 == 0.0f) return;
    float rinv = __builtin_amdgcn_rsqf(r2);
    float fbx = (float)bx, fby = (float)by, fbz = (float)bz;
    float q = fmaf(fbx, dx, fmaf(fby, dy, fbz * dz)) * (rinv * rinv);
    float s = (float)cz * rinv;
    ix = fmaf(-dx, q, fbx) * s;
    iy = fmaf(-dy, q, fby) * s;
    iz = fmaf(-dz, q, fbz) * s;
  }
  double kl = floor(ulo), kh = floor(uhi);
  if (kl == kh) {   // whole box inside one bin of this segment
    int j = (int)kl;
    put3<acc_t>(row, j - lo, ix, iy, iz);
    if (j + 1 < hi) put3<acc_t>(row, j + 1 - lo, -ix, -iy, -iz);
    return;
  }
  double w = uhi - ulo;
  double flo = (kl + 1.0) - ulo;   // share of bin kl, in (0, 1]
  double fhi = uhi - kh;           // share of bin kh, in [0, 1)
  // clamp far-out indices before the int conversion (all fold or drop alike)
  int jl = (int)fmax(kl, (double)lo - 2.0);
  int jh = (int)fmin(kh, (double)hi);
  if (kh == kl + 1.0) {
    T fa, fb;
    if (P == 0) {
      fa = (T)(flo / w);
      fb = (T)(fhi / w);
    } else {
      float wi = __builtin_amdgcn_rcpf((float)w);
      fa = (T)((float)flo * wi);
      fb = (T)((float)fhi * wi);
    }
    T axv = ix * fa, ayv = iy * fa, azv = iz * fa;
    T bxv = ix * fb, byv = iy * fb, bzv = iz * fb;
    put3_clamped<acc_t>(row, jl, lo, hi, axv, ayv, azv);
    put3_clamped<acc_t>(row, jl + 1, lo, hi, bxv - axv, byv - ayv, bzv - azv);
    put3_clamped<acc_t>(row, jl + 2, lo, hi, -bxv, -byv, -bzv);
  } else {
    T wi;
    if (P == 0) wi = (T)(1.0 / w);
    else wi = (T)__builtin_amdgcn_rcpf((float)w);
    T hx = ix * wi, hy = iy * wi, hz = iz * wi;
    T fl = (T)flo, fh = (T)fhi;
    T gl = (T)1 - fl, gh = (T)1 - fh;
    put3_clamped<acc_t>(row, jl, lo, hi, hx * fl, hy * fl, hz * fl);
    put3_clamped<acc_t>(row, jl + 1, lo, hi, hx * gl, hy * gl, hz * gl);
    put3_clamped<acc_t>(row, jh, lo, hi, -hx * gh, -hy * gh, -hz * gh);
    put3_clamped<acc_t>(row, jh + 1, lo, hi, -hx * fh, -hy * fh, -hz * fh);
  }
}

// F: 0 Endpoint, 1 ZHS.  P: 0 FP64, 1 mixed.  MED: 0 uniform, 1 exponential.
// AT: antennas per tile.
template <int F, int P, int MED, int AT>
__global__ void __launch_bounds__(1024) deposit_kernel(DepositArgs g) {
  using T = acc_t;
  using In = typename Prec<P>::in;
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  T *tile = reinterpret_cast<T *>(smem);

  const int v = xcd_major(blockIdx.x, gridDim.x);
  const int n_tiles = g.n_atiles * g.n_segs;
  const int tl = v % n_tiles;
  const int split = v / n_tiles;
  const int atile = tl / g.n_segs;
  const int seg = tl % g.n_segs;
  const int64_t a_begin = (int64_t)atile * AT;
  const int n_ant = (int)min((int64_t)AT, g.an.m - a_begin);
  const int lo = seg * g.seg_len;
  const int hi = min(lo + g.seg_len, g.c.n_bins);
  const int row_len = (hi - lo) * 3;

  for (int i = threadIdx.x; i < AT * row_len; i += blockDim.x) tile[i] = T(0);

  double ax[AT], ay[AT], az[AT], tau[AT], ea[AT];
#pragma unroll
  for (int a = 0; a < AT; ++a) {
    int64_t ai = a_begin + (a < n_ant ? a : 0);
    ax[a] = g.an.x[ai];
    ay[a] = g.an.y[ai];
    az[a] = g.an.z[ai];
    tau[a] = g.an.t_start[ai];
    ea[a] = MED == 1 ? height_factor(az[a], g.c) : 0.0;
  }
  // all tile antennas at one height: one path index per track end
  bool flat = true;
#pragma unroll
  for (int a = 1; a < AT; ++a) flat = flat && (a >= n_ant || az[a] == az[0]);
  __syncthreads();

  const int64_t i0 = (int64_t)split * g.per_split;
  const int64_t i1 = min(g.tr.n, i0 + g.per_split);
  const In *pbx = (const In *)g.tr.bx, *pby = (const In *)g.tr.by, *pbz = (const In *)g.tr.bz,
           *pqw = (const In *)g.tr.qw;

  for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) {
    const double x0 = g.tr.x0[i], y0 = g.tr.y0[i], z0 = g.tr.z0[i], t0 = g.tr.t0[i];
    const double x1 = g.tr.x1[i], y1 = g.tr.y1[i], z1 = g.tr.z1[i], t1 = g.tr.t1[i];
    const double bx = (double)pbx[i], by = (double)pby[i], bz = (double)pbz[i];
    const double qw = (double)pqw[i];
    // a track with any non-finite field contributes nothing (the sum is
    // non-finite iff some field is, barring overflow of finite fields)
    if (!isfinite(((((x0 + y0) + (z0 + t0)) + ((x1 + y1) + (z1 + t1))) + ((bx + by) + (bz + qw)))))
      continue;
    double e0 = 0.0, e1 = 0.0;
    if (MED == 1) {
      e0 = g.e0[i];
      e1 = g.e1[i];
    }
    double nf0 = g.c.n_uniform, nf1 = g.c.n_uniform;
    if (MED == 1 && flat) {
      nf0 = path_index(z0, az[0], e0, ea[0], g.c);
      nf1 = path_index(z1, az[0], e1, ea[0], g.c);
    }
    if (F == 0) {
      double ns0 = g.c.n_uniform, ns1 = g.c.n_uniform;
      if (MED == 1) {
        ns0 = 1.0 + g.c.n0m1 * e0;
        ns1 = 1.0 + g.c.n0m1 * e1;
      }
      const double sc = g.c.k * qw * g.c.inv_dt;
#pragma unroll
      for (int a = 0; a < AT; ++a) {
        if (a < n_ant) {
          double ne0 = nf0, ne1 = nf1;
          if (MED == 1 && !flat) {
            ne0 = path_index(z0, az[a], e0, ea[a], g.c);
            ne1 = path_index(z1, az[a], e1, ea[a], g.c);
          }
          T *row = tile + a * row_len;
          endpoint_end<P>(row, lo, hi, sc, x0, y0, z0, t0, ax[a], ay[a], az[a], tau[a], ne0, ns0,
                          bx, by, bz, g.c);
          endpoint_end<P>(row, lo, hi, -sc, x1, y1, z1, t1, ax[a], ay[a], az[a], tau[a], ne1, ns1,
                          bx, by, bz, g.c);
        }
      }
    } else {
      const double mx = (x0 + x1) * 0.5, my = (y0 + y1) * 0.5, mz = (z0 + z1) * 0.5;
      const double cz = g.c.k * qw * (t1 - t0) * g.c.inv_dt;
#pragma unroll
      for (int a = 0; a < AT; ++a) {
        if (a < n_ant) {
          double ne0 = nf0, ne1 = nf1;
          if (MED == 1 && !flat) {
            ne0 = path_index(z0, az[a], e0, ea[a], g.c);
            ne1 = path_index(z1, az[a], e1, ea[a], g.c);
          }
          double dx, dy, dz, r;
          double us = arrival_bins(x0, y0, z0, t0, ax[a], ay[a], az[a], tau[a], ne0, g.c, dx, dy,
                                   dz, r);
          double ue = arrival_bins(x1, y1, z1, t1, ax[a], ay[a], az[a], tau[a], ne1, g.c, dx, dy,
                                   dz, r);
          zhs_box<P>(tile + a * row_len, lo, hi, us, ue, mx, my, mz, ax[a], ay[a], az[a], cz, bx,
                     by, bz);
        }
      }
    }
  }
  __syncthreads();

  T *dst = reinterpret_cast<T *>(g.partial);
  for (int a = 0; a < n_ant; ++a) {
    T *out = dst + (((size_t)split * g.an.m + (size_t)(a_begin + a)) * g.c.n_bins + lo) * 3;
    const T *src = tile + a * row_len;
    for (int i = threadIdx.x; i < row_len; i += blockDim.x) out[i] = src[i];
  }
}

// ------------------------------------------------------------------ merge

// One workgroup per (antenna, segment): traces += sum over splits (index
// order) of the partials; for ZHS the summed differences are prefix-scanned
// over the segment's bins first. Accumulation is in double precision.
template <int F, int P>
__global__ void __launch_bounds__(256) merge_kernel(const void *partial, void *traces, int64_t m,
                                                    int n_bins, int splits, int seg_len,
                                                    int n_segs) {
  using T = typename Prec<P>::out;
  const acc_t *part = reinterpret_cast<const acc_t *>(partial);
  T *out = reinterpret_cast<T *>(traces);
  const int64_t a = blockIdx.x / n_segs;
  const int seg = blockIdx.x % n_segs;
  const int lo = seg * seg_len;
  const int nb = min(lo + seg_len, n_bins) - lo;
  const size_t plane = (size_t)m * n_bins * 3;
  const size_t base = ((size_t)a * n_bins + lo) * 3;
  if (F == 0) {
    for (int i = threadIdx.x; i < nb * 3; i += blockDim.x) {
      double s = 0.0;
      for (int sp = 0; sp < splits; ++sp) s += (double)part[sp * plane + base + i];
      out[base + i] = (T)((double)out[base + i] + s);
    }
    return;
  }
  __shared__ double carry[256][3];
  const int per = (nb + blockDim.x - 1) / blockDim.x;
  const int b0 = min((int)threadIdx.x * per, nb), b1 = min(b0 + per, nb);
  double run[3] = {0.0, 0.0, 0.0};
  for (int b = b0; b < b1; ++b)
    for (int c = 0; c < 3; ++c)
      for (int sp = 0; sp < splits; ++sp) run[c] += (double)part[sp * plane + base + 3 * b + c];
  for (int c = 0; c < 3; ++c) carry[threadIdx.x][c] = run[c];
  __syncthreads();
  if (threadIdx.x < 3) {
    double acc = 0.0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      double x = carry[t][threadIdx.x];
      carry[t][threadIdx.x] = acc;
      acc += x;
    }
  }
  __syncthreads();
  for (int c = 0; c < 3; ++c) run[c] = carry[threadIdx.x][c];
  for (int b = b0; b < b1; ++b)
    for (int c = 0; c < 3; ++c) {
      double d = 0.0;
      for (int sp = 0; sp < splits; ++sp) d += (double)part[sp * plane + base + 3 * b + c];
      run[c] += d;
      size_t o = base + 3 * b + c;
      out[o] = (T)((double)out[o] + run[c]);
    }
}

// ------------------------------------------------------------------ propagator

__global__ void __launch_bounds__(256) propagate_kernel(TrackPtrs tr, AntPtrs an, Consts c,
                                                        double *t_out, int32_t *bin_out) {
  const int64_t total = tr.n * an.m;
  for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx / an.m, a = idx % an.m;
    const double ax = an.x[a], ay = an.y[a], az = an.z[a], tau = an.t_start[a];
    for (int e = 0; e < 2; ++e) {
      double px = e ? tr.x1[i] : tr.x0[i];
      double py = e ? tr.y1[i] : tr.y0[i];
      double pz = e ? tr.z1[i] : tr.z0[i];
      double tp = e ? tr.t1[i] : tr.t0[i];
      double neff = c.n_uniform;
      if (c.medium == 1) neff = path_index(pz, az, height_factor(pz, c), height_factor(az, c), c);
      double t = arrival_time(px, py, pz, tp, ax, ay, az, neff, c);
      double u = (t - tau) * c.inv_dt;
      size_t o = ((size_t)e * tr.n + i) * an.m + a;
      if (t_out) t_out[o] = t;
      if (bin_out) bin_out[o] = (u >= 0.0 && u < c.nbins_d) ? (int32_t)u : -1;
    }
  }
}

// ------------------------------------------------------------------ host side

size_t acc_bytes(int) { return sizeof(acc_t); }

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t prep_bytes(const rt_plan &p, int64_t n) {
  return p.med.kind == RT_EXPONENTIAL ? align256((size_t)n * 2 * sizeof(double)) : 0;
}

Tiling choose_tiling(const rt_plan &p, int64_t n) {
  Tiling t;
  const size_t acc = acc_bytes(p.precision);
  const int B = p.det.n_bins;
  const int64_t M = p.det.n_antennas;
  const size_t budget = p.lds_per_block;
  int seg = p.seg_user > 0 ? p.seg_user : B;
  if ((size_t)seg * 3 * acc > budget) seg = (int)(budget / (3 * acc)) / 64 * 64;
  if (seg > B) seg = B;
  if (seg < 1) seg = 1;
  t.seg_len = seg;
  t.n_segs = (B + seg - 1) / seg;
  int at = p.at_user > 0 ? p.at_user : (int)(budget / ((size_t)seg * 3 * acc));
  if (at > kMaxTile) at = kMaxTile;
  if (at < 1) at = 1;
  if (at > M) at = (int)M;
  t.at = at;
  t.n_atiles = (int)((M + at - 1) / at);
  t.lds_bytes = (size_t)at * seg * 3 * acc;
  t.block = p.block_user > 0 ? p.block_user : 1024;
  const int64_t n_tiles = (int64_t)t.n_atiles * t.n_segs;
  int64_t splits;
  if (p.splits_user > 0) {
    splits = p.splits_user;
  } else {
    // aim for two rounds of workgroups over the chip, each split >= 2 blocks of tracks
    int64_t resident = (int64_t)p.num_cus * (int64_t)std::max<size_t>(1, p.lds_per_cu / t.lds_bytes);
    splits = (2 * resident + n_tiles - 1) / n_tiles;
    int64_t cap = std::max<int64_t>(1, n / (2 * t.block));
    if (splits > cap) splits = cap;
    if (splits < 1) splits = 1;
  }
  if (n > 0 && splits > n) splits = n;
  t.per_split = n > 0 ? (n + splits - 1) / splits : 1;
  t.splits = n > 0 ? (int)((n + t.per_split - 1) / t.per_split) : 1;
  return t;
}

size_t workspace_bytes(const rt_plan &p, int64_t n) {
  Tiling t = choose_tiling(p, n);
  return prep_bytes(p, n) +
         align256((size_t)t.splits * p.det.n_antennas * p.det.n_bins * 3 * acc_bytes(p.precision));
}

TrackPtrs track_ptrs(const rt_tracks &t) {
  return TrackPtrs{t.x0, t.y0, t.z0, t.t0, t.x1, t.y1, t.z1, t.t1, t.bx, t.by, t.bz, t.qw, t.n};
}

AntPtrs ant_ptrs(const rt_detector &d) { return AntPtrs{d.x, d.y, d.z, d.t_start, d.n_antennas}; }

using DepositFn = void (*)(DepositArgs);

template <int F, int P, int MED>
static DepositFn pick_at(int at) {
  switch (at) {
    case 1: return deposit_kernel<F, P, MED, 1>;
    case 2: return deposit_kernel<F, P, MED, 2>;
    case 3: return deposit_kernel<F, P, MED, 3>;
    default: return deposit_kernel<F, P, MED, 4>;
  }
}

static DepositFn pick_deposit(int f, int prec, int med, int at) {
  if (f == RT_ENDPOINT) {
    if (prec == RT_FP64) return med ? pick_at<0, 0, 1>(at) : pick_at<0, 0, 0>(at);
    return med ? pick_at<0, 1, 1>(at) : pick_at<0, 1, 0>(at);
  }
  if (prec == RT_FP64) return med ? pick_at<1, 0, 1>(at) : pick_at<1, 0, 0>(at);
  return med ? pick_at<1, 1, 1>(at) : pick_at<1, 1, 0>(at);
}

using MergeFn = void (*)(const void *, void *, int64_t, int, int, int, int);

static MergeFn pick_merge(int f, int prec) {
  if (f == RT_ENDPOINT) return prec == RT_FP64 ? merge_kernel<0, 0> : merge_kernel<0, 1>;
  return prec == RT_FP64 ? merge_kernel<1, 0> : merge_kernel<1, 1>;
}

hipError_t launch_forward(const rt_plan &p, const rt_tracks &t, void *traces, void *workspace,
                          hipStream_t stream) {
  const Tiling tl = choose_tiling(p, t.n);
  char *ws = reinterpret_cast<char *>(workspace);
  DepositArgs g;
  g.tr = track_ptrs(t);
  g.an = ant_ptrs(p.det);
  g.c = p.c;
  g.e0 = g.e1 = nullptr;
  const int med = p.med.kind == RT_EXPONENTIAL ? 1 : 0;
  if (med) {
    double *e = reinterpret_cast<double *>(ws);
    g.e0 = e;
    g.e1 = e + t.n;
    int blocks = (int)std::min<int64_t>((t.n + 255) / 256, 65536);
    prepare_kernel<<<blocks, 256, 0, stream>>>(g.tr, p.c, e, e + t.n);
  }
  g.partial = ws + prep_bytes(p, t.n);
  g.per_split = tl.per_split;
  g.n_atiles = tl.n_atiles;
  g.n_segs = tl.n_segs;
  g.seg_len = tl.seg_len;
  DepositFn fn = pick_deposit(p.formalism, p.precision, med, tl.at);
  if (tl.lds_bytes > 65536)
    (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)tl.lds_bytes);
  const int64_t grid = (int64_t)tl.n_atiles * tl.n_segs * tl.splits;
  if (p.ev_start) (void)hipEventRecord(p.ev_start, stream);
  fn<<<dim3((unsigned)grid), dim3(tl.block), tl.lds_bytes, stream>>>(g);
  if (p.ev_stop) (void)hipEventRecord(p.ev_stop, stream);
  MergeFn mf = pick_merge(p.formalism, p.precision);
  mf<<<dim3((unsigned)(p.det.n_antennas * tl.n_segs)), dim3(256), 0, stream>>>(
      g.partial, traces, p.det.n_antennas, p.det.n_bins, tl.splits, tl.seg_len, tl.n_segs);
  return hipGetLastError();
}

hipError_t launch_propagate(const rt_plan &p, const rt_tracks &t, double *t_arrival,
                            int32_t *bin, hipStream_t stream) {
  const int64_t total = t.n * p.det.n_antennas;
  int blocks = (int)std::min<int64_t>((total + 255) / 256, 1 << 20);
  propagate_kernel<<<blocks, 256, 0, stream>>>(track_ptrs(t), ant_ptrs(p.det), p.c, t_arrival,
                                               bin);
  return hipGetLastError();
}

}  // namespace rt
