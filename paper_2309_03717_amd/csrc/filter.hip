// filter.hip -- the track filter: the check each track passes before the
// antenna loop (§2, Fig. 1: the radio process first decides whether a track
// is relevant to the radio calculation). Kept tracks are compacted, in their
// input order, into caller buffers, so that dropped tracks take no lane in
// the deposits.
//
// A track is kept when every field is finite, |qw| > qw_min, and it can
// radiate: it moves (some velocity component is nonzero) and it is not a
// point (its end differs from its start in position or time). With
// qw_min = 0 every dropped track contributes exactly nothing to either
// formalism (non-finite tracks are skipped by definition, qw = 0 and beta = 0
// give zero amplitudes, a point's two Endpoint impulses cancel in one bin and
// its ZHS box has zero integral).
//
// Kernels: filter_count_kernel (kept tracks per workgroup), filter_scan_kernel
// (one workgroup: exclusive prefix sums of the counts, and the total) and
// filter_scatter_kernel (each workgroup writes its kept tracks from its
// offset on, in order).
#include "rt_internal.h"

namespace rt {

constexpr int kFilterBlock = 256;   // tracks per workgroup, one per thread
constexpr int kScanThreads = 1024;

struct FilterIn {
  const double *x0, *y0, *z0, *t0, *x1, *y1, *z1, *t1;
  const void *bx, *by, *bz, *qw;
  int64_t n;
};

struct FilterOut {
  double *x0, *y0, *z0, *t0, *x1, *y1, *z1, *t1;
  void *bx, *by, *bz, *qw;
};

template <typename In>
__device__ __forceinline__ bool keep_track(const FilterIn &t, int64_t i, double qw_min) {
  const double x0 = t.x0[i], y0 = t.y0[i], z0 = t.z0[i], t0 = t.t0[i];
  const double x1 = t.x1[i], y1 = t.y1[i], z1 = t.z1[i], t1 = t.t1[i];
  const double bx = (double)((const In *)t.bx)[i], by = (double)((const In *)t.by)[i];
  const double bz = (double)((const In *)t.bz)[i], qw = (double)((const In *)t.qw)[i];
  const bool finite = isfinite(x0) && isfinite(y0) && isfinite(z0) && isfinite(t0) &&
                      isfinite(x1) && isfinite(y1) && isfinite(z1) && isfinite(t1) &&
                      isfinite(bx) && isfinite(by) && isfinite(bz) && isfinite(qw);
  const bool moves = bx != 0.0 || by != 0.0 || bz != 0.0;
  const bool extends = x1 != x0 || y1 != y0 || z1 != z0 || t1 != t0;
  return finite && fabs(qw) > qw_min && moves && extends;
}

// Kept tracks before this thread's within its workgroup, and the workgroup's
// total (wave ballots, then the waves' counts in LDS).
__device__ __forceinline__ int block_prefix(bool keep, int *total) {
  __shared__ int wave_count[kFilterBlock / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const uint64_t ballot = __ballot(keep);
  const int below = __popcll(ballot & ((1ull << lane) - 1));
  if (lane == 0) wave_count[wave] = __popcll(ballot);
  __syncthreads();
  int before = 0, sum = 0;
  for (int w = 0; w < kFilterBlock / 64; ++w) {
    if (w < wave) before += wave_count[w];
    sum += wave_count[w];
  }
  *total = sum;
  return before + below;
}

template <typename In>
__global__ void __launch_bounds__(kFilterBlock) filter_count_kernel(FilterIn t, double qw_min,
                                                                  int64_t *counts) {
  const int64_t i = (int64_t)blockIdx.x * kFilterBlock + threadIdx.x;
  const bool keep = i < t.n && keep_track<In>(t, i, qw_min);
  int total = 0;
  block_prefix(keep, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Exclusive prefix sums of nb counts, in chunks of kScanThreads, and the
// total into *n_kept.
__global__ void __launch_bounds__(kScanThreads) filter_scan_kernel(const int64_t *counts,
                                                                   int64_t nb, int64_t *offsets,
                                                                   int64_t *n_kept) {
  __shared__ int64_t buf[kScanThreads];
  int64_t carry = 0;
  for (int64_t base = 0; base < nb; base += kScanThreads) {
    const int64_t j = base + threadIdx.x;
    const int64_t v = j < nb ? counts[j] : 0;
    buf[threadIdx.x] = v;
    __syncthreads();
    for (int s = 1; s < kScanThreads; s <<= 1) {   // inclusive scan
      const int64_t add = (int)threadIdx.x >= s ? buf[threadIdx.x - s] : 0;
      __syncthreads();
      buf[threadIdx.x] += add;
      __syncthreads();
    }
    if (j < nb) offsets[j] = carry + buf[threadIdx.x] - v;
    carry += buf[kScanThreads - 1];
    __syncthreads();   // buf is rewritten by the next chunk
  }
  if (threadIdx.x == 0) *n_kept = carry;
}

template <typename In>
__global__ void __launch_bounds__(kFilterBlock) filter_scatter_kernel(FilterIn t, FilterOut o,
                                                                    double qw_min,
                                                                    const int64_t *offsets) {
  const int64_t i = (int64_t)blockIdx.x * kFilterBlock + threadIdx.x;
  const bool keep = i < t.n && keep_track<In>(t, i, qw_min);
  int total = 0;
  const int local = block_prefix(keep, &total);
  if (!keep) return;
  const int64_t d = offsets[blockIdx.x] + local;
  o.x0[d] = t.x0[i];
  o.y0[d] = t.y0[i];
  o.z0[d] = t.z0[i];
  o.t0[d] = t.t0[i];
  o.x1[d] = t.x1[i];
  o.y1[d] = t.y1[i];
  o.z1[d] = t.z1[i];
  o.t1[d] = t.t1[i];
  ((In *)o.bx)[d] = ((const In *)t.bx)[i];
  ((In *)o.by)[d] = ((const In *)t.by)[i];
  ((In *)o.bz)[d] = ((const In *)t.bz)[i];
  ((In *)o.qw)[d] = ((const In *)t.qw)[i];
}

__global__ void filter_zero_kernel(int64_t *n_kept) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *n_kept = 0;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t filter_workspace_bytes(int64_t n) {
  const int64_t nb = (n + kFilterBlock - 1) / kFilterBlock;
  return 2 * align256((size_t)std::max<int64_t>(nb, 1) * sizeof(int64_t));
}

hipError_t launch_filter(const rt_tracks &in, int precision, double qw_min, const rt_tracks &out,
                         int64_t *n_kept, void *workspace, hipStream_t stream) {
  if (in.n == 0) {
    filter_zero_kernel<<<1, 64, 0, stream>>>(n_kept);
    return hipGetLastError();
  }
  const int64_t nb = (in.n + kFilterBlock - 1) / kFilterBlock;
  int64_t *counts = reinterpret_cast<int64_t *>(workspace);
  int64_t *offsets = reinterpret_cast<int64_t *>(reinterpret_cast<char *>(workspace) +
                                                 filter_workspace_bytes(in.n) / 2);
  const FilterIn fi{in.x0, in.y0, in.z0, in.t0, in.x1, in.y1, in.z1, in.t1,
                    in.bx, in.by, in.bz, in.qw, in.n};
  const FilterOut fo{const_cast<double *>(out.x0), const_cast<double *>(out.y0),
                     const_cast<double *>(out.z0), const_cast<double *>(out.t0),
                     const_cast<double *>(out.x1), const_cast<double *>(out.y1),
                     const_cast<double *>(out.z1), const_cast<double *>(out.t1),
                     const_cast<void *>(out.bx),   const_cast<void *>(out.by),
                     const_cast<void *>(out.bz),   const_cast<void *>(out.qw)};
  if (precision == RT_FP64)
    filter_count_kernel<double><<<(unsigned)nb, kFilterBlock, 0, stream>>>(fi, qw_min, counts);
  else
    filter_count_kernel<float><<<(unsigned)nb, kFilterBlock, 0, stream>>>(fi, qw_min, counts);
  filter_scan_kernel<<<1, kScanThreads, 0, stream>>>(counts, nb, offsets, n_kept);
  if (precision == RT_FP64)
    filter_scatter_kernel<double><<<(unsigned)nb, kFilterBlock, 0, stream>>>(fi, fo, qw_min,
                                                                             offsets);
  else
    filter_scatter_kernel<float><<<(unsigned)nb, kFilterBlock, 0, stream>>>(fi, fo, qw_min,
                                                                            offsets);
  return hipGetLastError();
}

}  // namespace rt

// ------------------------------------------------------------------ C ABI

extern "C" {

int rt_filter_workspace_bytes(int64_t n_tracks, size_t *bytes) {
  if (!bytes) return rt_fail(RT_E_INVALID, "bytes is NULL");
  if (n_tracks < 0) return rt_fail(RT_E_INVALID, "n_tracks < 0");
  *bytes = rt::filter_workspace_bytes(n_tracks);
  return RT_OK;
}

int rt_filter_tracks(const rt_tracks *in, int precision, double qw_min, const rt_tracks *out,
                     int64_t *n_kept, void *workspace, size_t workspace_bytes, void *stream) {
  if (!in || !out || !n_kept) return rt_fail(RT_E_INVALID, "in, out or n_kept is NULL");
  if (precision != RT_FP64 && precision != RT_MIXED)
    return rt_fail(RT_E_INVALID, "precision must be RT_FP64 or RT_MIXED");
  if (!(qw_min >= 0.0) || qw_min == __builtin_inf())
    return rt_fail(RT_E_INVALID, "qw_min must be finite and >= 0");
  int st = rt_check_tracks(in, 0);
  if (st != RT_OK) return st;
  if (in->n > 0) {
    st = rt_check_tracks(out, 0);
    if (st != RT_OK) return rt_fail(st, std::string("out: ") + rt_last_error());
    if (out->n < in->n)
      return rt_fail(RT_E_INVALID, "out->n (the output capacity) must be >= in->n");
  }
  if (in->n > (int64_t)INT32_MAX * rt::kFilterBlock)
    return rt_fail(RT_E_UNSUPPORTED, "too many tracks for one filter call");
  const size_t need = rt::filter_workspace_bytes(in->n);
  if (!workspace || workspace_bytes < need)
    return rt_fail(RT_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
  (void)hipGetLastError();
  hipError_t e = rt::launch_filter(*in, precision, qw_min, *out, n_kept, workspace,
                                   (hipStream_t)stream);
  if (e != hipSuccess) return rt_hip_fail(e, "launching the track filter");
  return RT_OK;
}

}  // extern "C"
