// forward.hip -- the track x antenna loop on gfx950: a per-track record
// written once per call, LDS-resident antenna trace tiles fed by streamed
// track records, a fixed-order merge of track-split partials (with the ZHS
// prefix scan), and the propagator alone.
//
// Work decomposition (the analogue of the antenna bunch a thread takes in §4): a
// workgroup owns a tile of up to kMaxTile antennas x one segment of bins in
// LDS and streams one range ("split") of the tracks past it; each lane takes
// one track and loops over the tile's antennas, so track loads are coalesced
// and each deposit is an LDS atomic add. The tile is then written once to a
// partial buffer [split][M][B][3] and a second kernel sums the splits in index
// order into the caller's traces, so no float atomic ever touches global
// memory and a fixed tiling gives the same merge order on every call.
//
// With one 4096-bin FP64 trace per workgroup every record is read once per
// antenna, which makes this loop sensitive to load latency. Workgroups of 1024
// threads (four waves per SIMD, one workgroup per CU) cover most of it; the
// Endpoint deposit, bound by record delivery, also loads each record one wave
// block ahead (register double-buffering).
//
// Precision. The LDS tiles accumulate in double (ds_add_f64), or for RT_MIXED
// ZHS calls in 64-bit fixed point (ds_add_u64, exact and order-independent):
// on gfx950 a single-precision LDS atomic add (ds_add_f32) executes about 13x
// slower than ds_add_f64 at any address pattern, and ds_add_u64 about twice as
// fast. In RT_MIXED the Endpoint arrival time and bin are computed exactly as
// in RT_FP64 (an impulse's bin is a step function of its time) and its
// amplitude uses the hardware reciprocals refined by one Newton step
// (relative error a few 1e-15); the ZHS box, continuous in the arrival times,
// takes them from a square root good to 5e-15 and from times and path
// indices stored in bins, and its amplitude and weights from the unrefined
// hardware estimates (5e-8, single-precision accuracy). All of it runs in
// double precision: unpacked single-precision arithmetic issues at the same
// rate on this chip and would only add conversions. Tracks carry beta and qw
// as float and the traces are float in RT_MIXED.
#include "rt_deposit.h"
#include "rt_internal.h"

namespace rt {

struct PrepArgs {
  TrackPtrs tr;
  AntPtrs an;
  Consts c;
  double *rec;
  int64_t n_blocks;   // wave blocks (tracks rounded up to 64)
  // fixed-point ZHS calls: the antennas' bounding box (written by
  // bbox_kernel) and, per prepare workgroup, the sum and the maximum of the
  // per-track deposit bounds; null otherwise
  const double *bbox;
  double *fx_part;
};

constexpr int kPrepThreads = 256;
constexpr int kPrepMaxBlocks = 65536;

// One thread per (padded) track. A track with any non-finite field, and the
// padding past the last track, get NaN times so that no antenna window
// accepts them. Fixed-point ZHS calls also reduce the per-track deposit
// bounds of each workgroup (fixed order: a tree over its threads) into
// fx_part.
template <int F, int P>
__global__ void __launch_bounds__(kPrepThreads) prepare_kernel(PrepArgs g) {
  const Consts c = resolve_consts(g.c);
  const double z_ref = g.an.z[0];
  const double e_ref = c.medium == 1 || c.medium == 2 ? path_factor(z_ref, c) : 0.0;
  const int64_t n_pad = g.n_blocks * 64;
  constexpr bool kFx = F == 1 && P == 1;
  double bsum = 0.0, bmax = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_pad;
       i += (int64_t)gridDim.x * blockDim.x) {
    double v[kRec];
    make_record<F, P>(g.tr, i, i < g.tr.n, c, z_ref, e_ref, v);
    store_record(g.rec + ((i >> 6) * kRec) * 64, (int)(i & 63), v,
                 single_slot_records<F, P>(c.medium));
    if (kFx && g.fx_part) {
      const double b = zhs_track_bound(v, g.bbox);
      bsum += b;
      bmax = fmax(bmax, b);
    }
  }
  if (kFx && g.fx_part) {
    __shared__ double ssum[kPrepThreads], smax[kPrepThreads];
    ssum[threadIdx.x] = bsum;
    smax[threadIdx.x] = bmax;
    __syncthreads();
    for (int h = kPrepThreads / 2; h > 0; h >>= 1) {
      if ((int)threadIdx.x < h) {
        ssum[threadIdx.x] += ssum[threadIdx.x + h];
        smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + h]);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      g.fx_part[2 * blockIdx.x] = ssum[0];
      g.fx_part[2 * blockIdx.x + 1] = smax[0];
    }
  }
}

// The antennas' bounding box: bbox = {xmin, xmax, ymin, ymax, zmin, zmax}.
// One workgroup of kPrepThreads threads.
__global__ void __launch_bounds__(kPrepThreads) bbox_kernel(AntPtrs an, double *bbox) {
  __shared__ double red[6 * kPrepThreads];
  double bb[6];
  antenna_bbox<kPrepThreads>(an, red, bb);
  if (threadIdx.x < 6) bbox[threadIdx.x] = bb[threadIdx.x];
}

// The call's fixed-point unit (fx_unit) from the prepare workgroups' bound
// sums and maxima, summed in a fixed order, written as fx = {unit, 1 / unit},
// both powers of two, or {0, 0} when the call keeps the double-precision tile.
__global__ void fx_reduce_kernel(const double *fx_part, int n_parts, int64_t n_tracks,
                                 double *fx) {
  __shared__ double ssum[kPrepThreads], smax[kPrepThreads];
  double sum = 0.0, mx = 0.0;
  for (int i = threadIdx.x; i < n_parts; i += kPrepThreads) {
    sum += fx_part[2 * i];
    mx = fmax(mx, fx_part[2 * i + 1]);
  }
  ssum[threadIdx.x] = sum;
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int h = kPrepThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      ssum[threadIdx.x] += ssum[threadIdx.x + h];
      smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double unit = fx_unit(ssum[0], smax[0], n_tracks);
  fx[0] = unit;
  fx[1] = unit > 0.0 ? 1.0 / unit : 0.0;
}

// ------------------------------------------------------------------ deposits

struct DepositArgs {
  AntPtrs an;
  Consts c;
  const double *rec;       // per-track records of this pass (first wave block)
  void *partial;           // [splits][M][n_bins][3] doubles (int64 for fixed-point tiles)
  const double *fx;        // fixed-point ZHS calls: {unit, 1 / unit}, unit 0 = off; else null
  int64_t n_blocks;        // wave blocks of tracks in this pass
  int64_t blocks_per_split;
  int n_atiles, n_segs, seg_len;
  int accumulate;          // 0: first pass writes the partials; 1: later passes add
};

// Adds (or, on a call's first pass, writes) the tile rows of the workgroup's
// antennas into their partial slots.
template <typename A>
__device__ __forceinline__ void flush_tile(const DepositArgs &g, lds<acc_t> *tile, int stride,
                                           int front, int split, int64_t a_begin, int n_ant,
                                           int lo, int row_len) {
  A *dst = reinterpret_cast<A *>(g.partial);
  for (int a = 0; a < n_ant; ++a) {
    A *out = dst + (((size_t)split * g.an.m + (size_t)(a_begin + a)) * g.c.n_bins + lo) * 3;
    const lds<A> *src = reinterpret_cast<lds<A> *>(tile) + a * stride + front;
    if (g.accumulate)
      for (int i = threadIdx.x; i < row_len; i += blockDim.x) out[i] += fold_front(src, i, front);
    else
      for (int i = threadIdx.x; i < row_len; i += blockDim.x) out[i] = fold_front(src, i, front);
  }
}

// F: 0 Endpoint, 1 ZHS.  P: 0 FP64, 1 mixed.  MED: 0 uniform, 1 exponential,
// 2 tabulated, 3 spherical Earth.  AT: antennas per tile. Mixed ZHS calls
// accumulate in int64 fixed point when the call's unit allows it (g.fx[0] >
// 0) and in double otherwise.
template <int F, int P, int MED, int AT>
__global__ void __launch_bounds__(1024) deposit_kernel(DepositArgs g) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  lds<acc_t> *tile = (lds<acc_t> *)smem;

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
  const int stride = (g.seg_len + tile_pad(F)) * 3;

  for (int i = threadIdx.x; i < AT * stride; i += blockDim.x) tile[i] = 0.0;

  const Consts c = resolve_consts(g.c);
  Tile<AT> t;
  load_tile<AT, MED>(g.an, a_begin, n_ant, c, t);
  constexpr bool kFxCap = F == 1 && P == 1;
  const double fx_unit = kFxCap ? g.fx[0] : 0.0;
  const TileRef tr{tile, stride, lo, (double)lo, (double)hi, kFxCap ? g.fx[1] : 0.0,
                   tile_front(F) * 3};
  __syncthreads();

  const uint64_t mask = (1ull << n_ant) - 1;
  const int64_t waves = blockDim.x >> 6;
  // the wave index as a wave-uniform value: block counters and loop tests
  // then live in scalar registers
  const int64_t b_first =
      (int64_t)split * g.blocks_per_split + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t b_end = min(g.n_blocks, (int64_t)(split + 1) * g.blocks_per_split);
  // record prefetch: the Endpoint deposit and the one-antenna ZHS deposit
  // (alternating buffers for mixed records; the wider ZHS tiles would spill
  // the second buffer), except over the spherical Earth, whose per-pair
  // quadrature dominates
  constexpr int kPf = MED != 3 && (F == 0 || AT == 1) ? kPfAlternate : kPfNone;
  if (kFxCap && fx_unit > 0.0)
    deposit_blocks<F, P, MED, AT, kPf, true>(g.rec, b_first, b_end, waves, mask, t, tr, c,
                                             ConstNodes{g.c});
  else
    deposit_blocks<F, P, MED, AT, kPf, false>(g.rec, b_first, b_end, waves, mask, t, tr, c,
                                              ConstNodes{g.c});
  __syncthreads();

  if (kFxCap && fx_unit > 0.0)
    flush_tile<long long>(g, tile, stride, tile_front(F) * 3, split, a_begin, n_ant, lo, row_len);
  else
    flush_tile<acc_t>(g, tile, stride, tile_front(F) * 3, split, a_begin, n_ant, lo, row_len);
}

// ------------------------------------------------------------------ merge

// One workgroup per (antenna, segment): traces += sum over splits (index
// order) of the partials, prefix-scanned over the segment for ZHS.
template <int F, int P>
__global__ void __launch_bounds__(kMergeThreads) merge_kernel(const void *partial, void *traces,
                                                              int64_t m, int n_bins, int splits,
                                                              int seg_len, int n_segs,
                                                              const double *fx) {
  using T = typename Prec<P>::out;
  const int64_t a = blockIdx.x / n_segs;
  const int seg = blockIdx.x % n_segs;
  const int lo = seg * seg_len;
  const int nb = min(lo + seg_len, n_bins) - lo;
  const size_t base = ((size_t)a * n_bins + lo) * 3;
  const int64_t stride = (int64_t)m * n_bins * 3;
  T *out = reinterpret_cast<T *>(traces) + base;
  if (F == 1 && P == 1 && fx[0] > 0.0)
    merge_segment<F, T>(reinterpret_cast<const long long *>(partial) + base, stride, splits, out,
                        nb, fx[0]);
  else
    merge_segment<F, T>(reinterpret_cast<const acc_t *>(partial) + base, stride, splits, out, nb,
                        1.0);
}

// ------------------------------------------------------------------ propagator

__global__ void __launch_bounds__(256) propagate_kernel(TrackPtrs tr, AntPtrs an, Consts c0,
                                                        double *t_out, int32_t *bin_out) {
  const Consts c = resolve_consts(c0);
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
      if (c.medium == 3)
        neff = sph_path_index(px, py, pz, ax, ay, az, c, ConstNodes{c0});
      else if (c.medium != 0)
        neff = path_index(pz, az, path_factor(pz, c), path_factor(az, c), c);
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

static int64_t wave_blocks(int64_t n) { return (n + 63) / 64; }

// Workspace: [records][fixed-point region][partials][tabulated profile's
// cumulative integral]. The fixed-point region (mixed ZHS plans) holds the
// antennas' bounding box (6 doubles), the unit pair fx (2 doubles), then the
// sum and maximum of the track bounds of every prepare workgroup.
size_t prep_bytes(const rt_plan &, int64_t n) {
  return align256((size_t)wave_blocks(n) * kRec * 64 * sizeof(double));
}

static int prep_blocks(int64_t n) {
  return (int)std::min<int64_t>((wave_blocks(n) * 64 + kPrepThreads - 1) / kPrepThreads,
                                kPrepMaxBlocks);
}

static bool uses_fx(const rt_plan &p) { return p.formalism == RT_ZHS && p.precision == RT_MIXED; }

static size_t fx_bytes(const rt_plan &p, int64_t n) {
  return uses_fx(p) ? align256((8 + 2 * (size_t)prep_blocks(n)) * sizeof(double)) : 0;
}

size_t table_bytes(const rt_plan &p) {
  return p.med.kind == RT_TABULATED ? align256((size_t)p.med.n_table * sizeof(double)) : 0;
}

// F at the nodes of a tabulated profile: trapezoids summed from the first
// node up, one thread (the order every lookup relies on).
__global__ void tab_cells_kernel(Consts c, double *cells) {
  if (threadIdx.x == 0 && blockIdx.x == 0) fill_tab_cells(c, cells);
}

void launch_tab_cells(const rt_plan &p, double *cells, hipStream_t stream) {
  tab_cells_kernel<<<1, 64, 0, stream>>>(p.c, cells);
}

Tiling choose_tiling(const rt_plan &p, int64_t n) {
  Tiling t;
  const size_t acc = acc_bytes(p.precision);
  const int B = p.det.n_bins;
  const int64_t M = p.det.n_antennas;
  const size_t budget = p.lds_per_block;
  // a tile row holds the segment's bins plus the formalism's padding bins
  const int pad = tile_pad(p.formalism);
  int seg = p.seg_user > 0 ? p.seg_user : B;
  if ((size_t)(seg + pad) * 3 * acc > budget) seg = (int)(budget / (3 * acc) - pad) / 64 * 64;
  if (seg > B) seg = B;
  if (seg < 1) seg = 1;
  t.seg_len = seg;
  t.n_segs = (B + seg - 1) / seg;
  const size_t row_bytes = (size_t)(seg + pad) * 3 * acc;
  int at = p.at_user > 0 ? p.at_user : (int)(budget / row_bytes);
  if (at > kMaxTile) at = kMaxTile;
  if (at < 1) at = 1;
  if (at > M) at = (int)M;
  t.at = at;
  t.n_atiles = (int)((M + at - 1) / at);
  t.lds_bytes = (size_t)at * row_bytes;
  // 1024 threads: with one workgroup per CU (the trace tile fills most of
  // the LDS) this keeps four waves per SIMD to hide the LDS atomics and the
  // record loads; the deposit kernels are built for at most 128 VGPRs
  t.block = p.block_user > 0 ? p.block_user : 1024;
  t.pass_tracks = p.pass_user > 0 ? p.pass_user : kDefaultPass;
  const int64_t n_tiles = (int64_t)t.n_atiles * t.n_segs;
  const int64_t nb = std::max<int64_t>(1, wave_blocks(std::min(n, t.pass_tracks)));
  int64_t splits;
  if (p.splits_user > 0) {
    splits = p.splits_user;
  } else {
    // aim for two rounds of workgroups over the chip, each split >= 4 passes
    // of the workgroup over its tracks
    int64_t resident = (int64_t)p.num_cus * (int64_t)std::max<size_t>(1, p.lds_per_cu / t.lds_bytes);
    splits = (2 * resident + n_tiles - 1) / n_tiles;
    // workgroups drift apart where deposits cost unequally across antennas
    // (a ZHS box costs more than a missed window; shower-like tracks land far
    // more often near the axis), so the workgroups resident together stop
    // sharing records in L2 over long track ranges: cap a split at
    // kZhsSplitBlocks (ZHS) or kEpSplitBlocks (Endpoint) wave blocks
    const int64_t cap_blocks = p.formalism == RT_ZHS ? kZhsSplitBlocks : kEpSplitBlocks;
    splits = std::max(splits, (nb + cap_blocks - 1) / cap_blocks);
    int64_t cap = std::max<int64_t>(1, nb / (4 * (t.block / 64)));
    if (splits > cap) splits = cap;
    if (splits < 1) splits = 1;
  }
  if (splits > nb) splits = nb;
  t.blocks_per_split = (nb + splits - 1) / splits;
  t.splits = (int)((nb + t.blocks_per_split - 1) / t.blocks_per_split);
  t.per_split = t.blocks_per_split * 64;
  return t;
}

size_t workspace_bytes(const rt_plan &p, int64_t n) {
  Tiling t = choose_tiling(p, n);
  return prep_bytes(p, n) + fx_bytes(p, n) +
         align256((size_t)t.splits * p.det.n_antennas * p.det.n_bins * 3 * acc_bytes(p.precision)) +
         table_bytes(p);
}

TrackPtrs track_ptrs(const rt_tracks &t) {
  return TrackPtrs{t.x0, t.y0, t.z0, t.t0, t.x1, t.y1, t.z1, t.t1, t.bx, t.by, t.bz, t.qw, t.n};
}

AntPtrs ant_ptrs(const rt_detector &d) { return AntPtrs{d.x, d.y, d.z, d.t_start, d.n_antennas}; }

using DepositFn = void (*)(DepositArgs);
using PrepFn = void (*)(PrepArgs);

template <int F, int P, int MED>
static DepositFn pick_at(int at) {
  switch (at) {
    case 1: return deposit_kernel<F, P, MED, 1>;
    case 2: return deposit_kernel<F, P, MED, 2>;
    case 3: return deposit_kernel<F, P, MED, 3>;
    case 4: return deposit_kernel<F, P, MED, 4>;
    case 5: return deposit_kernel<F, P, MED, 5>;
    case 6: return deposit_kernel<F, P, MED, 6>;
    case 7: return deposit_kernel<F, P, MED, 7>;
    default: return deposit_kernel<F, P, MED, 8>;
  }
}

template <int F, int P>
static DepositFn pick_med(int med, int at) {
  if (med == 3) return pick_at<F, P, 3>(at);
  if (med == 2) return pick_at<F, P, 2>(at);
  return med ? pick_at<F, P, 1>(at) : pick_at<F, P, 0>(at);
}

static DepositFn pick_deposit(int f, int prec, int med, int at) {
  if (f == RT_ENDPOINT) return prec == RT_FP64 ? pick_med<0, 0>(med, at) : pick_med<0, 1>(med, at);
  return prec == RT_FP64 ? pick_med<1, 0>(med, at) : pick_med<1, 1>(med, at);
}

static PrepFn pick_prep(int f, int prec) {
  if (f == RT_ENDPOINT) return prec == RT_FP64 ? prepare_kernel<0, 0> : prepare_kernel<0, 1>;
  return prec == RT_FP64 ? prepare_kernel<1, 0> : prepare_kernel<1, 1>;
}

using MergeFn = void (*)(const void *, void *, int64_t, int, int, int, int, const double *);

static MergeFn pick_merge(int f, int prec) {
  if (f == RT_ENDPOINT) return prec == RT_FP64 ? merge_kernel<0, 0> : merge_kernel<0, 1>;
  return prec == RT_FP64 ? merge_kernel<1, 0> : merge_kernel<1, 1>;
}

hipError_t launch_forward(const rt_plan &p, const rt_tracks &t, void *traces, void *workspace,
                          hipStream_t stream) {
  const Tiling tl = choose_tiling(p, t.n);
  char *ws = reinterpret_cast<char *>(workspace);
  Consts c = p.c;
  if (p.med.kind == RT_TABULATED) {
    double *cells = reinterpret_cast<double *>(ws + workspace_bytes(p, t.n) - table_bytes(p));
    launch_tab_cells(p, cells, stream);
    c.tabF = cells;
  }
  PrepArgs pa;
  pa.tr = track_ptrs(t);
  pa.an = ant_ptrs(p.det);
  pa.c = c;
  pa.rec = reinterpret_cast<double *>(ws);
  pa.n_blocks = wave_blocks(t.n);
  pa.bbox = nullptr;
  pa.fx_part = nullptr;
  double *fx = nullptr;
  const int blocks = prep_blocks(t.n);
  if (uses_fx(p)) {
    // bounding box -> records and per-workgroup bounds -> the call's unit
    double *region = reinterpret_cast<double *>(ws + prep_bytes(p, t.n));
    pa.bbox = region;
    fx = region + 6;
    pa.fx_part = region + 8;
    bbox_kernel<<<1, kPrepThreads, 0, stream>>>(pa.an, region);
  }
  pick_prep(p.formalism, p.precision)<<<blocks, kPrepThreads, 0, stream>>>(pa);
  if (uses_fx(p)) fx_reduce_kernel<<<1, kPrepThreads, 0, stream>>>(pa.fx_part, blocks, t.n, fx);
  DepositArgs g;
  g.an = pa.an;
  g.c = c;
  g.fx = fx;
  g.partial = ws + prep_bytes(p, t.n) + fx_bytes(p, t.n);
  g.blocks_per_split = tl.blocks_per_split;
  g.n_atiles = tl.n_atiles;
  g.n_segs = tl.n_segs;
  g.seg_len = tl.seg_len;
  const int med = p.med.kind;   // 0 uniform, 1 exponential, 2 tabulated, 3 spherical
  DepositFn fn = pick_deposit(p.formalism, p.precision, med, tl.at);
  MergeFn mf = pick_merge(p.formalism, p.precision);
  if (tl.lds_bytes > 65536)
    (void)hipFuncSetAttribute((const void *)fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)tl.lds_bytes);
  // Passes run back to back; each workgroup adds its tile into the partial
  // slot of its (split, tile), which only it touches within a pass, so the
  // partials hold the sum over passes and one merge follows the last pass.
  // The first pass has the most blocks, hence every split, and writes all
  // slots.
  const int64_t pass_blocks = tl.pass_tracks / 64;
  if (p.ev_start) (void)hipEventRecord(p.ev_start, stream);
  for (int64_t b0 = 0; b0 < pa.n_blocks; b0 += pass_blocks) {
    g.rec = pa.rec + b0 * (kRec * 64);
    g.n_blocks = std::min(pass_blocks, pa.n_blocks - b0);
    g.accumulate = b0 > 0;
    const int64_t splits = (g.n_blocks + tl.blocks_per_split - 1) / tl.blocks_per_split;
    const int64_t grid = (int64_t)tl.n_atiles * tl.n_segs * splits;
    fn<<<dim3((unsigned)grid), dim3(tl.block), tl.lds_bytes, stream>>>(g);
  }
  if (p.ev_stop) (void)hipEventRecord(p.ev_stop, stream);
  mf<<<dim3((unsigned)(p.det.n_antennas * tl.n_segs)), dim3(kMergeThreads), 0, stream>>>(
      g.partial, traces, p.det.n_antennas, p.det.n_bins, tl.splits, tl.seg_len, tl.n_segs, fx);
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
