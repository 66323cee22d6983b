// batch.hip -- many independent showers (each with its own antenna array,
// time binning, medium, formalism and tracks) in one persistent launch.
//
// The host cuts every shower into work items (antenna tile x bin segment x
// track split) of similar cost and sorts them longest first. A persistent
// grid (one or more workgroups per compute unit) takes items in that order
// from an integer atomic counter; each item deposits into an LDS tile exactly
// as the single-plan kernel does and writes the tile to its own partial slot,
// so the result does not depend on which workgroup took which item. A merge
// kernel then adds, per (shower, antenna, segment), the slots of the splits in
// index order into the shower's traces (with the ZHS prefix scan). Mixed
// ZHS showers accumulate in 64-bit fixed point, with a unit per shower from
// its tracks' deposit bounds (as a single plan's call does), so their traces
// do not depend on the launch shape. On a non-null stream the whole sequence
// is captured once into a HIP graph and replayed by later launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "rt_deposit.h"
#include "rt_internal.h"

namespace rt {

struct ShowerDesc {
  TrackPtrs tr;
  AntPtrs an;
  Consts c;
  void *traces;
  int32_t formalism, at, seg_len, n_segs, n_atiles, splits;
  int64_t rec_block0;        // first wave block of this shower in the record array
  int64_t n_blocks;          // wave blocks of 64 tracks of this shower
  int64_t blocks_per_split;
  int64_t part0;             // first double of this shower's partial slots
  int64_t slot_len;          // doubles per slot: at * seg_len * 3
  int64_t tab_off;           // tabulated medium: first double of its F table in the
                             // workspace's table region (-1 otherwise)
  int32_t fx_chunk0, fx_chunks;   // mixed ZHS: its chunks of the fixed-point bound
                                  // reduction (none otherwise)
};

// A range of one mixed ZHS shower's record blocks whose deposit bounds one
// workgroup reduces (the fixed-point unit's sum and maximum).
struct FxChunk {
  int32_t shower, pad;
  int64_t block0, n_blocks;   // first wave block (within the shower) and count
};
constexpr int64_t kFxChunkBlocks = 1024;   // 65536 tracks per chunk
constexpr int kFxThreads = 256;

struct WorkItem {
  int32_t shower, atile, seg, split;
};

struct MergeTask {
  int32_t shower, antenna, seg, pad;
};

// Work-item groups, each taken by its own persistent kernel from its own
// counter: the uniform and exponential media (all of them, or with
// one-antenna tiles their Endpoint items, group 0, and their ZHS items,
// group 1), then the tabulated and spherical media (group 2).
enum : int { kGroupLight = 0, kGroupLightZhs = 1, kGroupHeavy = 2, kGroups = 3 };

struct BatchArgs {
  const ShowerDesc *sh;
  const WorkItem *items;       // grouped: [group_begin[g], group_begin[g + 1])
  const MergeTask *merges;
  const int64_t *cum_blocks;   // [n_showers + 1] first wave block of each shower
  const FxChunk *fx_chunks;    // [n_fx_chunks]
  int32_t n_showers, n_items, n_fx_chunks;
  int32_t group_begin[kGroups + 1];
  int *counter;                // [kGroups]: next item of each group
  double *rec;
  double *partial;
  double *tables;              // F tables of the tabulated showers
  double *fx;                  // [n_showers][2]: fixed-point unit and its inverse
                               // (0: the shower keeps the double tile)
  double *fx_part;             // [n_fx_chunks][2]: bound sum and maximum
  int64_t total_blocks;
};

__global__ void batch_reset_kernel(int *counter) {
  if (threadIdx.x < kGroups && blockIdx.x == 0) counter[threadIdx.x] = 0;
}

// A wave-uniform copy of a 4- or 8-byte value: values a workgroup reads from
// a shower descriptor in global memory are the same in every lane, and
// saying so lets them live in scalar registers.
template <class T>
__device__ __forceinline__ T uniform(T x) {
  static_assert(sizeof(T) == 4 || sizeof(T) == 8, "4- or 8-byte values");
  if constexpr (sizeof(T) == 4) {
    int v;
    __builtin_memcpy(&v, &x, 4);
    v = __builtin_amdgcn_readfirstlane(v);
    __builtin_memcpy(&x, &v, 4);
  } else {
    long long v;
    __builtin_memcpy(&v, &x, 8);
    const int lo = __builtin_amdgcn_readfirstlane((int)v);
    const int hi = __builtin_amdgcn_readfirstlane((int)(v >> 32));
    v = (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
    __builtin_memcpy(&x, &v, 8);
  }
  return x;
}

// The constants of a shower as the kernels use them (wave-uniform): a
// tabulated medium reads its F table from the workspace. The quadrature
// nodes are not used from here: the deposits read the LDS copy (LdsNodes).
__device__ __forceinline__ Consts shower_consts(const ShowerDesc &s, const BatchArgs &b) {
  Consts c = s.c;
  if (c.medium == 2) c.tabF = b.tables + s.tab_off;
  c.inv_c = uniform(c.inv_c);
  c.inv_dt = uniform(c.inv_dt);
  c.k = uniform(c.k);
  c.n_uniform = uniform(c.n_uniform);
  c.n0m1 = uniform(c.n0m1);
  c.h = uniform(c.h);
  c.n0h = uniform(c.n0h);
  c.nbins_d = uniform(c.nbins_d);
  c.n_bins = uniform(c.n_bins);
  c.medium = uniform(c.medium);
  c.tab = uniform(c.tab);
  c.tabF = uniform(c.tabF);
  c.n_tab = uniform(c.n_tab);
  c.tz0 = uniform(c.tz0);
  c.tdz = uniform(c.tdz);
  c.tinv_dz = uniform(c.tinv_dz);
  c.re = uniform(c.re);
  c.re2 = uniform(c.re2);
  c.re_twice = uniform(c.re_twice);
  return c;
}

// F at the nodes of every tabulated shower's profile, one workgroup per
// shower, the sums of a single plan's table.
__global__ void batch_tables_kernel(BatchArgs b) {
  const ShowerDesc &s = b.sh[blockIdx.x];
  if (threadIdx.x == 0 && s.c.medium == 2) fill_tab_cells(s.c, b.tables + s.tab_off);
}

// Records of every shower, one thread per padded track.
template <int P>
__global__ void __launch_bounds__(256) batch_prepare_kernel(BatchArgs b) {
  const int64_t n_pad = b.total_blocks * 64;
  for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_pad;
       g += (int64_t)gridDim.x * blockDim.x) {
    const int64_t blk = g >> 6;
    int lo = 0, hi = b.n_showers;   // cum[lo] <= blk < cum[hi]
    while (hi - lo > 1) {
      int mid = (lo + hi) >> 1;
      if (b.cum_blocks[mid] <= blk) lo = mid; else hi = mid;
    }
    const ShowerDesc &s = b.sh[lo];
    const int64_t i = g - s.rec_block0 * 64;
    const Consts c = shower_consts(s, b);
    const double z_ref = s.an.z[0];
    const double e_ref = c.medium == 1 || c.medium == 2 ? path_factor(z_ref, c) : 0.0;
    double v[kRec];
    if (s.formalism == RT_ENDPOINT)
      make_record<0, P>(s.tr, i, i < s.tr.n, c, z_ref, e_ref, v);
    else
      make_record<1, P>(s.tr, i, i < s.tr.n, c, z_ref, e_ref, v);
    const bool single = s.formalism == RT_ENDPOINT ? single_slot_records<0, P>(c.medium)
                                                   : single_slot_records<1, P>(c.medium);
    store_record(b.rec + (blk * kRec) * 64, (int)(g & 63), v, single);
  }
}

// Deposit bounds of one chunk of a mixed ZHS shower's records (its antennas'
// bounding box first): their sum and maximum, reduced over the workgroup in
// a fixed order.
__global__ void __launch_bounds__(kFxThreads) batch_fx_part_kernel(BatchArgs b) {
  __shared__ double red[6 * kFxThreads];
  const FxChunk ch = b.fx_chunks[blockIdx.x];
  const ShowerDesc &s = b.sh[ch.shower];
  double bb[6];
  antenna_bbox<kFxThreads>(s.an, red, bb);
  const double *rec = b.rec + (s.rec_block0 + ch.block0) * (kRec * 64);
  double sum = 0.0, mx = 0.0;
  for (int64_t i = threadIdx.x; i < ch.n_blocks * 64; i += kFxThreads) {
    double v[kRec];
    const double *blk = rec + (i >> 6) * (kRec * 64);
    const int l = (int)(i & 63);
    // the slots the bound reads: points, times, amplitude and velocity
#pragma unroll
    for (int f = 0; f < kRec; ++f)
      v[f] = (f <= R_T1 || f == M_AB || f == M_YZ) ? blk[(f & ~1) * 64 + 2 * l + (f & 1)] : 0.0;
    const double bnd = zhs_track_bound(v, bb);
    sum += bnd;
    mx = fmax(mx, bnd);
  }
  red[threadIdx.x] = sum;
  red[kFxThreads + threadIdx.x] = mx;
  __syncthreads();
  for (int h = kFxThreads / 2; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      red[threadIdx.x] += red[threadIdx.x + h];
      red[kFxThreads + threadIdx.x] = fmax(red[kFxThreads + threadIdx.x],
                                           red[kFxThreads + threadIdx.x + h]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    b.fx_part[2 * blockIdx.x] = red[0];
    b.fx_part[2 * blockIdx.x + 1] = red[kFxThreads];
  }
}

// The fixed-point unit of every shower (chunk partials added in chunk
// order); 0 for the showers that keep the double tile. One thread per shower.
__global__ void batch_fx_unit_kernel(BatchArgs b) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= b.n_showers) return;
  const ShowerDesc &d = b.sh[s];
  double unit = 0.0;
  if (d.fx_chunks > 0) {
    double S = 0.0, B = 0.0;
    for (int c = 0; c < d.fx_chunks; ++c) {
      S += b.fx_part[2 * (d.fx_chunk0 + c)];
      B = fmax(B, b.fx_part[2 * (d.fx_chunk0 + c) + 1]);
    }
    unit = fx_unit(S, B, d.tr.n);
  }
  b.fx[2 * s] = unit;
  b.fx[2 * s + 1] = unit > 0.0 ? 1.0 / unit : 0.0;
}

// The quadrature nodes and weights of a spherical shower, copied to LDS for
// the item (kGl nodes, then kGl weights): every lane reads the same node, so
// the reads are broadcasts, and the constants copied per item need no
// dynamically indexed array.
struct LdsNodes {
  const double *p;
  __device__ __forceinline__ double s(int k) const { return p[k]; }
  __device__ __forceinline__ double w(int k) const { return p[kGl + k]; }
};

// The deposits of one work item into the LDS tile (FX: the fixed-point ZHS
// tile, for mixed ZHS showers whose unit is not 0).
template <int F, int P, int MED, int AT>
__device__ __forceinline__ void run_item(const double *rec, int64_t b_first, int64_t b_end,
                                         const AntPtrs &an, const Consts &c, const TileRef &tr,
                                         int64_t a_begin, int n_ant, const double *nodes,
                                         bool fx) {
  Tile<AT> t;
  load_tile<AT, MED>(an, a_begin, n_ant, c, t);
  const uint64_t mask = (1ull << n_ant) - 1;
  const int64_t waves = blockDim.x >> 6;
  constexpr int kPf = MED != 3 ? kPfNext : kPfNone;
  if (F == 1 && P == 1 && fx)
    deposit_blocks<F, P, MED, AT, kPf, true>(rec, b_first, b_end, waves, mask, t, tr, c,
                                             LdsNodes{nodes});
  else
    deposit_blocks<F, P, MED, AT, kPf, false>(rec, b_first, b_end, waves, mask, t, tr, c,
                                              LdsNodes{nodes});
}

// Tile width switch; ATMAX = 1 compiles the one-antenna path only.
template <int ATMAX, int F, int P, int MED>
__device__ __forceinline__ void run_item_at(int at, const double *rec, int64_t b_first,
                                            int64_t b_end, const AntPtrs &an, const Consts &c,
                                            const TileRef &tr, int64_t a_begin, int n_ant,
                                            const double *nodes, bool fx) {
  if (ATMAX == 1 || at == 1)
    run_item<F, P, MED, 1>(rec, b_first, b_end, an, c, tr, a_begin, n_ant, nodes, fx);
  else if (at == 2)
    run_item<F, P, MED, 2>(rec, b_first, b_end, an, c, tr, a_begin, n_ant, nodes, fx);
  else
    run_item<F, P, MED, 3>(rec, b_first, b_end, an, c, tr, a_begin, n_ant, nodes, fx);
}

// Persistent workgroups: take the items of one group until its counter
// passes the group's last one. Every workgroup leaves the loop once the
// counter has handed out the group's range, so the grid always drains.
// HEAVY: the group's two media (0: uniform, exponential; 1: tabulated,
// spherical). FF: the one formalism compiled in, or -1 for a run-time switch
// between both. ATMAX: the widest tile compiled in (1 or 3).
// nodes: 2 kGl doubles of LDS for a spherical shower's quadrature rule.
template <int P, int HEAVY, int FF, int ATMAX>
__device__ __forceinline__ void take_items(const BatchArgs &b, int group, lds<acc_t> *tile,
                                           int *cur, double *nodes) {
  const int first = b.group_begin[group], last = b.group_begin[group + 1];
  for (;;) {
    __syncthreads();   // everyone has read cur and flushed the previous tile
    if (threadIdx.x == 0) *cur = first + atomicAdd(b.counter + group, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(*cur);
    if (it >= last) break;
    const WorkItem w = b.items[it];
    const ShowerDesc &sd = b.sh[w.shower];
    const Consts c = shower_consts(sd, b);
    AntPtrs an = sd.an;
    an.x = uniform(an.x);
    an.y = uniform(an.y);
    an.z = uniform(an.z);
    an.t_start = uniform(an.t_start);
    an.m = uniform(an.m);
    const int at = ATMAX == 1 ? 1 : uniform(sd.at), seg_len = uniform(sd.seg_len);
    const int64_t a_begin = (int64_t)w.atile * at;
    const int n_ant = (int)min((int64_t)at, an.m - a_begin);
    const int lo = w.seg * seg_len;
    const int hi = min(lo + seg_len, c.n_bins);
    const int row_len = (hi - lo) * 3;
    const int f = FF >= 0 ? FF : uniform(sd.formalism);
    const int stride = (seg_len + tile_pad(f)) * 3;
    for (int i = threadIdx.x; i < at * stride; i += blockDim.x) tile[i] = 0.0;
    // mixed ZHS showers with a fixed-point unit: int64 tile (zero bits are 0)
    const double fx_inv = P == 1 && f == 1 ? uniform(b.fx[2 * w.shower + 1]) : 0.0;
    const bool fx = fx_inv > 0.0;
    const int front = tile_front(f) * 3;
    const TileRef tr{tile, stride, lo, (double)lo, (double)hi, fx_inv, front};
    if (HEAVY && c.medium == 3 && threadIdx.x < 2 * kGl)
      nodes[threadIdx.x] =
          threadIdx.x < kGl ? sd.c.gl_s[threadIdx.x] : sd.c.gl_w[threadIdx.x - kGl];
    __syncthreads();
    const double *rec = b.rec + uniform(sd.rec_block0) * (kRec * 64);
    const int64_t per_split = uniform(sd.blocks_per_split);
    const int64_t b_first =
        (int64_t)w.split * per_split + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t b_end = min(uniform(sd.n_blocks), (int64_t)(w.split + 1) * per_split);
    constexpr int M0 = HEAVY ? 2 : 0, M1 = HEAVY ? 3 : 1;   // this kernel's two media
    const bool m1 = c.medium == M1;
    if (FF != 1 && f == 0) {
      if (m1)
        run_item_at<ATMAX, 0, P, M1>(at, rec, b_first, b_end, an, c, tr, a_begin, n_ant, nodes,
                                     false);
      else
        run_item_at<ATMAX, 0, P, M0>(at, rec, b_first, b_end, an, c, tr, a_begin, n_ant, nodes,
                                     false);
    } else if (FF != 0) {
      if (m1)
        run_item_at<ATMAX, 1, P, M1>(at, rec, b_first, b_end, an, c, tr, a_begin, n_ant, nodes,
                                     fx);
      else
        run_item_at<ATMAX, 1, P, M0>(at, rec, b_first, b_end, an, c, tr, a_begin, n_ant, nodes,
                                     fx);
    }
    __syncthreads();
    const int64_t slot_len = uniform(sd.slot_len);
    const int64_t slot =
        ((int64_t)w.atile * uniform(sd.n_segs) + w.seg) * uniform(sd.splits) + w.split;
    acc_t *dst = b.partial + uniform(sd.part0) + slot * slot_len;
    for (int a = 0; a < n_ant; ++a) {
      const lds<acc_t> *src = tile + a * stride + front;
      for (int i = threadIdx.x; i < row_len; i += blockDim.x)
        dst[(int64_t)a * seg_len * 3 + i] =
            fx ? __longlong_as_double(
                     fold_front(reinterpret_cast<const lds<long long> *>(src), i, front))
               : fold_front(src, i, front);
    }
  }
}

// Any formalism and tile width, switched at run time: the union of their
// live registers (about 185 VGPRs) allows two waves per SIMD, hence at most
// 512 threads per workgroup. HEAVY = 0 takes group 0 (the uniform and
// exponential media), HEAVY = 1 group 2 (the tabulated and spherical ones),
// so that the common case keeps its registers.
template <int P, int HEAVY>
__global__ void __launch_bounds__(512) batch_deposit_kernel(BatchArgs b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int cur;
  __shared__ double nodes[HEAVY ? 2 * kGl : 1];
  take_items<P, HEAVY, -1, 3>(b, HEAVY ? kGroupHeavy : kGroupLight, (lds<acc_t> *)smem, &cur,
                              nodes);
}

// One-antenna tiles of the uniform and exponential media in one formalism F
// (group 0 Endpoint, group 1 ZHS): without the formalism and tile-width
// switches the registers fit 1024-thread workgroups, four waves per SIMD, as
// in the single-plan deposit.
template <int P, int F>
__global__ void __launch_bounds__(1024) batch_deposit_one_kernel(BatchArgs b) {
  extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
  __shared__ int cur;
  take_items<P, 0, F, 1>(b, F == 0 ? kGroupLight : kGroupLightZhs, (lds<acc_t> *)smem, &cur,
                         nullptr);
}

// One workgroup per (shower, antenna, segment): traces += sum over the
// shower's splits (in index order) of the slots, prefix-scanned for ZHS.
template <int P>
__global__ void __launch_bounds__(kMergeThreads) batch_merge_kernel(BatchArgs b) {
  using T = typename Prec<P>::out;
  const MergeTask mt = b.merges[blockIdx.x];
  const ShowerDesc &s = b.sh[mt.shower];
  const int atile = mt.antenna / s.at, ai = mt.antenna % s.at;
  const int lo = mt.seg * s.seg_len;
  const int nb = min(lo + s.seg_len, s.c.n_bins) - lo;
  const acc_t *part = b.partial + s.part0 +
                      ((int64_t)atile * s.n_segs + mt.seg) * s.splits * s.slot_len +
                      (int64_t)ai * s.seg_len * 3;
  T *out = reinterpret_cast<T *>(s.traces) + ((size_t)mt.antenna * s.c.n_bins + lo) * 3;
  const double unit = P == 1 && s.formalism == RT_ZHS ? b.fx[2 * mt.shower] : 0.0;
  if (s.formalism == RT_ENDPOINT)
    merge_segment<0, T>(part, s.slot_len, s.splits, out, nb, 1.0);
  else if (unit > 0.0)
    merge_segment<1, T>(reinterpret_cast<const long long *>(part), s.slot_len, s.splits, out, nb,
                        unit);
  else
    merge_segment<1, T>(part, s.slot_len, s.splits, out, nb, 1.0);
}

}  // namespace rt

// ------------------------------------------------------------------ host side

struct rt_batch {
  int precision = 0;
  int device = 0;
  int block = 512;             // 1024: one-antenna tiles, per-formalism kernels
  int grid = 1;                // persistent workgroups of each deposit kernel
  bool direct = false;
  size_t lds_bytes = 0;
  std::vector<rt::ShowerDesc> sh;
  std::vector<rt::WorkItem> items;
  std::vector<rt::MergeTask> merges;
  std::vector<int64_t> cum;
  std::vector<rt::FxChunk> fx_chunks;   // mixed ZHS showers' bound-reduction chunks
  int32_t group_begin[rt::kGroups + 1] = {0, 0, 0, 0};   // items, grouped
  int64_t total_blocks = 0, total_partial = 0, total_pairs = 0;
  int64_t total_tab = 0;       // doubles of the tabulated showers' F tables
  // the device tables (shower descriptors, work items, merge tasks,
  // cumulative record blocks, item counters) live at the start of the
  // caller's workspace; host_tables is their image, copied there by the
  // launches (offsets: tab_off[]), and tables_ws the workspace that last
  // received it
  std::vector<unsigned char> host_tables;
  size_t tab_off[6] = {0, 0, 0, 0, 0, 0};
  size_t tables_bytes = 0;
  void *tables_ws = nullptr;
  hipStream_t cap_stream = nullptr;   // created when a graph is first built
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void *cap_ws = nullptr;
  hipEvent_t ev_start = nullptr, ev_stop = nullptr;
};

namespace rt {

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

static size_t record_bytes(const rt_batch &b) {
  return align256((size_t)b.total_blocks * kRec * 64 * sizeof(double));
}

static size_t partial_bytes(const rt_batch &b) {
  return align256((size_t)b.total_partial * sizeof(acc_t));
}

static size_t tab_bytes(const rt_batch &b) {
  return align256((size_t)b.total_tab * sizeof(double));
}

// per shower {unit, 1 / unit}, then per bound-reduction chunk {sum, max}
static size_t fx_bytes(const rt_batch &b) {
  return align256(b.sh.size() * 2 * sizeof(double)) +
         align256(b.fx_chunks.size() * 2 * sizeof(double));
}

// the batch's tables, records, partial slots, the F tables of the tabulated
// showers, then the fixed-point region
size_t batch_workspace_bytes(const rt_batch &b) {
  return b.tables_bytes + record_bytes(b) + partial_bytes(b) + tab_bytes(b) + fx_bytes(b);
}

// The host image of the device tables, each part 256-byte aligned: shower
// descriptors, work items, merge tasks, cumulative record blocks, the kGroups
// item counters (reset by every launch) and the fixed-point chunks.
static void build_table_image(rt_batch &b) {
  const size_t sizes[6] = {b.sh.size() * sizeof(ShowerDesc), b.items.size() * sizeof(WorkItem),
                           b.merges.size() * sizeof(MergeTask), b.cum.size() * sizeof(int64_t),
                           kGroups * sizeof(int), b.fx_chunks.size() * sizeof(FxChunk)};
  const void *src[6] = {b.sh.data(), b.items.data(), b.merges.data(), b.cum.data(), nullptr,
                        b.fx_chunks.data()};
  size_t off = 0;
  for (int i = 0; i < 6; ++i) {
    b.tab_off[i] = off;
    off += align256(sizes[i]);
  }
  b.tables_bytes = off;
  b.host_tables.assign(off, 0);
  for (int i = 0; i < 6; ++i)
    if (sizes[i] && src[i]) std::memcpy(b.host_tables.data() + b.tab_off[i], src[i], sizes[i]);
}

static BatchArgs batch_args(const rt_batch &b, void *workspace) {
  BatchArgs a;
  char *ws = reinterpret_cast<char *>(workspace);
  a.sh = reinterpret_cast<const ShowerDesc *>(ws + b.tab_off[0]);
  a.items = reinterpret_cast<const WorkItem *>(ws + b.tab_off[1]);
  a.merges = reinterpret_cast<const MergeTask *>(ws + b.tab_off[2]);
  a.cum_blocks = reinterpret_cast<const int64_t *>(ws + b.tab_off[3]);
  a.counter = reinterpret_cast<int *>(ws + b.tab_off[4]);
  a.fx_chunks = reinterpret_cast<const FxChunk *>(ws + b.tab_off[5]);
  a.n_showers = (int32_t)b.sh.size();
  a.n_items = (int32_t)b.items.size();
  a.n_fx_chunks = (int32_t)b.fx_chunks.size();
  for (int g = 0; g <= kGroups; ++g) a.group_begin[g] = b.group_begin[g];
  char *data = ws + b.tables_bytes;
  a.rec = reinterpret_cast<double *>(data);
  a.partial = reinterpret_cast<double *>(data + record_bytes(b));
  a.tables = reinterpret_cast<double *>(data + record_bytes(b) + partial_bytes(b));
  a.fx = reinterpret_cast<double *>(data + record_bytes(b) + partial_bytes(b) + tab_bytes(b));
  a.fx_part = a.fx + align256(b.sh.size() * 2 * sizeof(double)) / sizeof(double);
  a.total_blocks = b.total_blocks;
  return a;
}

using BatchKernel = void (*)(BatchArgs);

// The deposit kernel of an item group and its workgroup size.
static BatchKernel deposit_fn(const rt_batch &b, int group, int *threads) {
  const bool one = b.block == 1024 && group != kGroupHeavy;
  *threads = one ? 1024 : std::min(b.block, 512);
  if (b.precision == RT_FP64) {
    if (one)
      return group == kGroupLight ? batch_deposit_one_kernel<0, 0> : batch_deposit_one_kernel<0, 1>;
    return group == kGroupHeavy ? batch_deposit_kernel<0, 1> : batch_deposit_kernel<0, 0>;
  }
  if (one)
    return group == kGroupLight ? batch_deposit_one_kernel<1, 0> : batch_deposit_one_kernel<1, 1>;
  return group == kGroupHeavy ? batch_deposit_kernel<1, 1> : batch_deposit_kernel<1, 0>;
}

static bool is_heavy(int medium) { return medium == RT_TABULATED || medium == RT_SPHERICAL; }

static int item_group(const rt_batch &b, const ShowerDesc &d) {
  if (is_heavy(d.c.medium)) return kGroupHeavy;
  return b.block == 1024 && d.formalism == RT_ZHS ? kGroupLightZhs : kGroupLight;
}

// reset counters, F tables, records, the persistent deposits of each item
// group, merge
static hipError_t batch_enqueue(const rt_batch &b, void *workspace, hipStream_t stream,
                                hipEvent_t ev0, hipEvent_t ev1) {
  if (b.items.empty()) return hipSuccess;
  BatchArgs a = batch_args(b, workspace);
  batch_reset_kernel<<<1, 64, 0, stream>>>(a.counter);
  if (b.total_tab > 0) batch_tables_kernel<<<(unsigned)b.sh.size(), 64, 0, stream>>>(a);
  const unsigned pblocks = (unsigned)std::min<int64_t>((b.total_blocks * 64 + 255) / 256, 1 << 16);
  if (b.precision == RT_FP64) {
    batch_prepare_kernel<0><<<pblocks, 256, 0, stream>>>(a);
  } else {
    batch_prepare_kernel<1><<<pblocks, 256, 0, stream>>>(a);
    // fixed-point units of the mixed ZHS showers (0 for the others)
    if (!b.fx_chunks.empty())
      batch_fx_part_kernel<<<(unsigned)b.fx_chunks.size(), kFxThreads, 0, stream>>>(a);
    batch_fx_unit_kernel<<<(unsigned)((b.sh.size() + 63) / 64), 64, 0, stream>>>(a);
  }
  if (ev0) (void)hipEventRecord(ev0, stream);
  for (int g = 0; g < kGroups; ++g) {
    if (b.group_begin[g + 1] == b.group_begin[g]) continue;
    int threads = 0;
    const BatchKernel k = deposit_fn(b, g, &threads);
    hipLaunchKernelGGL(k, dim3(b.grid), dim3(threads), b.lds_bytes, stream, a);
  }
  if (ev1) (void)hipEventRecord(ev1, stream);
  if (b.precision == RT_FP64)
    batch_merge_kernel<0><<<(unsigned)b.merges.size(), kMergeThreads, 0, stream>>>(a);
  else
    batch_merge_kernel<1><<<(unsigned)b.merges.size(), kMergeThreads, 0, stream>>>(a);
  return hipGetLastError();
}

// Tiles, splits, work items and merge tasks of a batch. Returns "" or an
// error text.
static std::string batch_plan(rt_batch &b, const rt_shower *showers, int32_t n, int precision,
                              double k, const rt_batch_options *opt, int num_cus,
                              size_t lds_block, size_t lds_cu) {
  b.precision = precision;
  b.block = (opt && opt->block_threads > 0) ? opt->block_threads : 512;
  b.direct = opt && opt->direct_launch != 0;
  const int items_per_cu = (opt && opt->items_per_cu > 0) ? opt->items_per_cu : 4;
  const int at_cap = (opt && opt->max_antennas_per_tile > 0) ? opt->max_antennas_per_tile : 3;
  const size_t row_bytes = 3 * sizeof(acc_t);
  const size_t budget = lds_block - 256;   // room for the kernel's own LDS words

  b.sh.resize(n);
  int64_t max_slot = 0;
  for (int s = 0; s < n; ++s) {
    const rt_shower &in = showers[s];
    ShowerDesc &d = b.sh[s];
    const int B = in.det.n_bins;
    const rt_tiling *user = (opt && opt->per_shower) ? &opt->per_shower[s] : nullptr;
    // a tile row holds a segment's bins plus the formalism's padding bins
    const int pad = tile_pad(in.formalism);
    const int max_bins = (int)(budget / row_bytes - pad) / 64 * 64;
    int seg = user && user->bins_per_segment > 0 ? std::min(user->bins_per_segment, B) : B;
    if (seg > max_bins) {   // equal segments, multiples of 64
      int segs = (B + max_bins - 1) / max_bins;
      seg = ((B + segs - 1) / segs + 63) / 64 * 64;
    }
    const size_t tile_row = (size_t)(seg + pad) * row_bytes;
    int at = user && user->antennas_per_block > 0 ? user->antennas_per_block
                                                  : std::min<int>(at_cap, (int)(budget / tile_row));
    at = (int)std::max<int64_t>(1, std::min<int64_t>({(int64_t)at, 3, in.det.n_antennas}));
    if ((size_t)at * tile_row > budget)
      return "the LDS tile of shower " + std::to_string(s) + " does not fit";
    d.tr = track_ptrs(in.tracks);
    d.an = ant_ptrs(in.det);
    d.traces = in.traces;
    d.formalism = in.formalism;
    d.at = at;
    d.seg_len = seg;
    d.n_segs = (B + seg - 1) / seg;
    d.n_atiles = (int)((in.det.n_antennas + at - 1) / at);
    d.n_blocks = (in.tracks.n + 63) / 64;
    d.slot_len = (int64_t)at * seg * 3;
    rt_fill_consts(in.det, in.med, k, d.c);
    const Consts &c = d.c;
    d.tab_off = -1;
    if (c.medium == RT_TABULATED) {   // 256-byte aligned table of n_tab doubles
      d.tab_off = b.total_tab;
      b.total_tab += ((int64_t)c.n_tab + 31) / 32 * 32;
    }
    if (d.n_blocks > 0) max_slot = std::max(max_slot, (int64_t)at * (seg + pad) * 3);
    b.total_pairs += in.tracks.n * in.det.n_antennas;
  }
  b.lds_bytes = (size_t)std::max<int64_t>(max_slot, 1) * sizeof(acc_t);
  // the run-time-switched kernels hold two waves per SIMD (512 threads per
  // CU), the one-antenna kernels four (1024 threads)
  const int per_cu = (int)std::max<size_t>(1, std::min<size_t>(lds_cu / (b.lds_bytes + 256),
                                                               512 / std::min(b.block, 512)));
  b.grid = num_cus * per_cu;
  // Track splits: items of similar cost (track x antenna evaluations, which
  // every bin segment repeats), about items_per_cu of them per compute unit,
  // counted apart for the two deposit kernels (their pairs cost differently).
  double group_cost[kGroups] = {0.0, 0.0, 0.0};
  for (const ShowerDesc &d : b.sh)
    group_cost[item_group(b, d)] += (double)d.n_blocks * 64 * d.at * d.n_atiles * d.n_segs;
  b.cum.assign(n + 1, 0);
  for (int s = 0; s < n; ++s) {
    ShowerDesc &d = b.sh[s];
    const rt_tiling *user = (opt && opt->per_shower) ? &opt->per_shower[s] : nullptr;
    const double target =
        std::max(1.0, group_cost[item_group(b, d)] / ((double)b.grid * items_per_cu));
    int64_t splits = user && user->track_splits > 0
                         ? user->track_splits
                         : (int64_t)std::ceil((double)d.n_blocks * 64 * d.at / target);
    splits = std::max<int64_t>(1, std::min<int64_t>(splits, d.n_blocks));
    d.blocks_per_split = std::max<int64_t>(1, (d.n_blocks + splits - 1) / splits);
    d.splits = d.n_blocks == 0 ? 0 : (int32_t)((d.n_blocks + d.blocks_per_split - 1) / d.blocks_per_split);
    d.rec_block0 = b.cum[s];
    b.cum[s + 1] = b.cum[s] + d.n_blocks;
    d.fx_chunk0 = (int32_t)b.fx_chunks.size();
    d.fx_chunks = 0;
    if (precision == RT_MIXED && d.formalism == RT_ZHS)
      for (int64_t b0 = 0; b0 < d.n_blocks; b0 += kFxChunkBlocks, ++d.fx_chunks)
        b.fx_chunks.push_back(FxChunk{s, 0, b0, std::min(kFxChunkBlocks, d.n_blocks - b0)});
    d.part0 = b.total_partial;
    b.total_partial += (int64_t)d.n_atiles * d.n_segs * d.splits * d.slot_len;
  }
  b.total_blocks = b.cum[n];
  // Work items, the uniform and exponential media first, each group longest
  // first; equal costs keep shower order, so the items of one shower run side
  // by side and share its records in the caches.
  std::vector<std::pair<int64_t, WorkItem>> all;
  for (int s = 0; s < n; ++s) {
    const ShowerDesc &d = b.sh[s];
    for (int t = 0; t < d.n_atiles; ++t)
      for (int g = 0; g < d.n_segs; ++g)
        for (int p = 0; p < d.splits; ++p) {
          int64_t blocks = std::min<int64_t>(d.n_blocks, (int64_t)(p + 1) * d.blocks_per_split) -
                           (int64_t)p * d.blocks_per_split;
          int64_t ants = std::min<int64_t>(d.at, d.an.m - (int64_t)t * d.at);
          all.push_back({blocks * ants, WorkItem{s, t, g, p}});
        }
  }
  if (all.size() > (size_t)INT32_MAX - 1024) return "too many work items";
  auto group = [&b](const WorkItem &w) { return item_group(b, b.sh[w.shower]); };
  std::stable_sort(all.begin(), all.end(),
                   [&group](const std::pair<int64_t, WorkItem> &x,
                            const std::pair<int64_t, WorkItem> &y) {
                     const int gx = group(x.second), gy = group(y.second);
                     return gx != gy ? gx < gy : x.first > y.first;
                   });
  b.items.reserve(all.size());
  int64_t count[kGroups] = {0, 0, 0};
  for (auto &x : all) {
    b.items.push_back(x.second);
    ++count[group(x.second)];
  }
  b.group_begin[0] = 0;
  for (int g = 0; g < kGroups; ++g) b.group_begin[g + 1] = b.group_begin[g] + (int32_t)count[g];
  for (int s = 0; s < n; ++s) {
    if (b.sh[s].n_blocks == 0) continue;
    for (int64_t a = 0; a < b.sh[s].an.m; ++a)
      for (int g = 0; g < b.sh[s].n_segs; ++g) b.merges.push_back(MergeTask{s, (int32_t)a, g, 0});
  }
  // one merge workgroup of kMergeThreads per (shower, antenna, segment): the
  // launch must stay below 2^32 threads
  if (b.merges.size() * kMergeThreads > (size_t)UINT32_MAX) return "too many merge tasks";
  return "";
}

static void release(rt_batch *b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap_stream) (void)hipStreamDestroy(b->cap_stream);
  delete b;
}

}  // namespace rt

extern "C" {

int rt_batch_create(rt_batch **batch, const rt_shower *showers, int32_t n_showers, int precision,
                    double k, const rt_batch_options *options) {
  if (!batch) return rt_fail(RT_E_INVALID, "batch output pointer is NULL");
  *batch = nullptr;
  if (!showers || n_showers < 1) return rt_fail(RT_E_INVALID, "need at least one shower");
  const bool one_antenna = options && options->block_threads == 1024;
  if (options) {
    const int bt = options->block_threads;
    if (bt != 0 && bt != 1024 && (bt < 64 || bt > 512 || bt % 64))
      return rt_fail(RT_E_INVALID,
                     "block_threads must be a multiple of 64 in [64, 512], or 1024 with "
                     "max_antennas_per_tile 1");
    if (options->items_per_cu < 0) return rt_fail(RT_E_INVALID, "items_per_cu must be >= 0");
    if (options->max_antennas_per_tile < 0 || options->max_antennas_per_tile > 3)
      return rt_fail(RT_E_INVALID, "max_antennas_per_tile must be in [0, 3]");
    if (one_antenna && options->max_antennas_per_tile != 1)
      return rt_fail(RT_E_INVALID, "block_threads 1024 needs max_antennas_per_tile 1");
  }
  for (int32_t s = 0; s < n_showers; ++s) {
    const rt_shower &sh = showers[s];
    const std::string where = "shower " + std::to_string(s) + ": ";
    int st = rt_check_setup(&sh.det, &sh.med, sh.formalism, precision, k);
    if (st == RT_OK) st = rt_check_tracks(&sh.tracks, sh.det.n_antennas);
    if (st != RT_OK) return rt_fail(st, where + rt_last_error());
    if (sh.tracks.n >= ((int64_t)1 << 31))
      return rt_fail(RT_E_UNSUPPORTED, where + "at most 2^31 - 1 tracks per shower");
    if (sh.tracks.n > 0 && !sh.traces) return rt_fail(RT_E_INVALID, where + "traces is NULL");
    if (options && options->per_shower) {
      const rt_tiling &t = options->per_shower[s];
      if (t.antennas_per_block < 0 || t.antennas_per_block > 3 || t.track_splits < 0 ||
          t.bins_per_segment < 0 ||
          (t.bins_per_segment > 0 && t.bins_per_segment % 64 && t.bins_per_segment != sh.det.n_bins))
        return rt_fail(RT_E_INVALID, where + "per-shower tiling out of range (antennas_per_block "
                                             "0-3, bins_per_segment a multiple of 64 or n_bins)");
      if (one_antenna && t.antennas_per_block > 1)
        return rt_fail(RT_E_INVALID, where + "block_threads 1024 takes one-antenna tiles only");
    }
  }
  int dev = 0, cus = 0;
  size_t lds_block = 0, lds_cu = 0;
  int st = rt_device_info(&dev, &cus, &lds_block, &lds_cu);
  if (st != RT_OK) return st;
  rt_batch *b = new (std::nothrow) rt_batch();
  if (!b) return rt_fail(RT_E_INVALID, "out of host memory");
  b->device = dev;
  std::string err = rt::batch_plan(*b, showers, n_showers, precision, k, options, cus, lds_block,
                                   lds_cu);
  if (!err.empty()) {
    delete b;
    return rt_fail(RT_E_UNSUPPORTED, err);
  }
  rt::build_table_image(*b);
  (void)hipGetLastError();
  hipError_t e = hipSuccess;
  for (int g = 0; g < rt::kGroups && e == hipSuccess; ++g) {
    int threads = 0;
    e = hipFuncSetAttribute((const void *)rt::deposit_fn(*b, g, &threads),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)b->lds_bytes);
  }
  if (e != hipSuccess) {
    rt::release(b);
    return rt_hip_fail(e, "setting up the batch kernels");
  }
  *batch = b;
  return RT_OK;
}

int rt_batch_destroy(rt_batch *batch) {
  if (batch) rt::release(batch);
  return RT_OK;
}

int rt_batch_workspace_bytes(const rt_batch *batch, size_t *bytes) {
  if (!batch || !bytes) return rt_fail(RT_E_INVALID, "batch or bytes is NULL");
  *bytes = rt::batch_workspace_bytes(*batch);
  return RT_OK;
}

int rt_batch_get_info(const rt_batch *batch, int64_t *n_items, int32_t *n_workgroups,
                      int64_t *lds_bytes, int64_t *pairs) {
  if (!batch) return rt_fail(RT_E_INVALID, "batch is NULL");
  if (n_items) *n_items = (int64_t)batch->items.size();
  if (n_workgroups) *n_workgroups = batch->grid;
  if (lds_bytes) *lds_bytes = (int64_t)batch->lds_bytes;
  if (pairs) *pairs = batch->total_pairs;
  return RT_OK;
}

int rt_batch_set_timing_events(rt_batch *batch, void *start_event, void *stop_event) {
  if (!batch) return rt_fail(RT_E_INVALID, "batch is NULL");
  if ((start_event == nullptr) != (stop_event == nullptr))
    return rt_fail(RT_E_INVALID, "give both events or neither");
  batch->ev_start = (hipEvent_t)start_event;
  batch->ev_stop = (hipEvent_t)stop_event;
  return RT_OK;
}

int rt_batch_launch(rt_batch *batch, void *workspace, size_t workspace_bytes, void *stream) {
  if (!batch) return rt_fail(RT_E_INVALID, "batch is NULL");
  const size_t need = rt::batch_workspace_bytes(*batch);
  if (need > 0 && (!workspace || workspace_bytes < need))
    return rt_fail(RT_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes, got " +
                                       std::to_string(workspace ? workspace_bytes : 0));
  if (batch->items.empty()) return RT_OK;   // every shower is empty
  hipStream_t s = (hipStream_t)stream;
  (void)hipGetLastError();
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (s) {
    hipError_t e = hipStreamIsCapturing(s, &cap);
    if (e != hipSuccess) return rt_hip_fail(e, "querying the stream's capture state");
  }
  // the tables: copied into the workspace on the launch stream before every
  // launch outside a capture (the host image persists until
  // rt_batch_destroy); a launch inside the caller's capture reuses the copy
  // an earlier launch left in this workspace
  if (cap == hipStreamCaptureStatusNone) {
    hipError_t e = hipMemcpyAsync(workspace, batch->host_tables.data(), batch->tables_bytes,
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return rt_hip_fail(e, "copying the batch tables");
    batch->tables_ws = workspace;
  } else if (batch->tables_ws != workspace) {
    return rt_fail(RT_E_INVALID,
                   "a launch inside a stream capture needs the batch tables in its workspace: "
                   "launch once with this workspace outside the capture first");
  }
  const bool timed = batch->ev_start != nullptr;
  if (batch->direct || timed || cap != hipStreamCaptureStatusNone) {
    hipError_t e = rt::batch_enqueue(*batch, workspace, s, batch->ev_start, batch->ev_stop);
    batch->ev_start = batch->ev_stop = nullptr;
    if (e != hipSuccess) return rt_hip_fail(e, "launching the batch kernels");
    return RT_OK;
  }
  if (!batch->exec || batch->cap_ws != workspace) {
    if (!batch->cap_stream) {
      hipError_t e = hipStreamCreateWithFlags(&batch->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return rt_hip_fail(e, "creating the capture stream");
    }
    if (batch->exec) (void)hipGraphExecDestroy(batch->exec);
    if (batch->graph) (void)hipGraphDestroy(batch->graph);
    batch->exec = nullptr;
    batch->graph = nullptr;
    hipError_t e = hipStreamBeginCapture(batch->cap_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return rt_hip_fail(e, "beginning the graph capture");
    hipError_t el = rt::batch_enqueue(*batch, workspace, batch->cap_stream, nullptr, nullptr);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(batch->cap_stream, &g);
    if (el != hipSuccess || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rt_hip_fail(el != hipSuccess ? el : e, "capturing the batch kernels");
    }
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      (void)hipGraphDestroy(g);
      return rt_hip_fail(e, "instantiating the batch graph");
    }
    batch->graph = g;
    batch->exec = x;
    batch->cap_ws = workspace;
  }
  hipError_t e = hipGraphLaunch(batch->exec, s);
  if (e != hipSuccess) return rt_hip_fail(e, "launching the batch graph");
  return RT_OK;
}

}  // extern "C"
