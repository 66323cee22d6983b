// autotune.hip -- the autotuner's timing loop: candidate launch shapes of a
// plan or of a batch, each timed with HIP events around real launches on the
// caller's buffers (no device allocation; the calls synchronize the stream).
// Choosing candidates and caching results is left to the caller.
#include <algorithm>
#include <string>
#include <vector>

#include "rt_internal.h"

namespace {

struct Events {
  hipEvent_t a = nullptr, b = nullptr;
  ~Events() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
  hipError_t create() {
    hipError_t e = hipEventCreate(&a);
    return e == hipSuccess ? hipEventCreate(&b) : e;
  }
};

// Median of the timed repetitions (ms).
float median(std::vector<float> v) {
  std::sort(v.begin(), v.end());
  const size_t n = v.size();
  return n % 2 ? v[n / 2] : 0.5f * (v[n / 2 - 1] + v[n / 2]);
}

// Times `launch` (one warm-up, then reps repetitions between two events on
// stream); returns RT_OK and the median in *ms, or the launch's status.
template <class Launch>
int time_launches(Launch launch, int reps, hipStream_t stream, Events &ev, float *ms) {
  int st = launch();
  if (st != RT_OK) return st;
  std::vector<float> t;
  for (int r = 0; r < reps; ++r) {
    hipError_t e = hipEventRecord(ev.a, stream);
    if (e != hipSuccess) return rt_hip_fail(e, "recording the start event");
    st = launch();
    if (st != RT_OK) return st;
    e = hipEventRecord(ev.b, stream);
    if (e == hipSuccess) e = hipEventSynchronize(ev.b);
    float x = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&x, ev.a, ev.b);
    if (e != hipSuccess) return rt_hip_fail(e, "timing a candidate");
    t.push_back(x);
  }
  *ms = median(t);
  return RT_OK;
}

}  // namespace

extern "C" {

int rt_plan_autotune(rt_plan *plan, const rt_tracks *sample, void *traces, void *workspace,
                     size_t workspace_bytes, const rt_tiling *candidates, int32_t n_candidates,
                     int32_t reps, void *stream, float *ms, int32_t *best) {
  if (!plan || !sample || !traces || !candidates || n_candidates < 1 || !best)
    return rt_fail(RT_E_INVALID, "plan, sample, traces, candidates and best are required");
  if (reps < 1) return rt_fail(RT_E_INVALID, "reps must be >= 1");
  if (sample->n < 1) return rt_fail(RT_E_INVALID, "the sample needs at least one track");
  rt_tiling keep;
  keep.antennas_per_block = plan->at_user;
  keep.track_splits = plan->splits_user;
  keep.block_threads = plan->block_user;
  keep.bins_per_segment = plan->seg_user;
  keep.tracks_per_pass = plan->pass_user;
  Events ev;
  hipError_t e = ev.create();
  if (e != hipSuccess) return rt_hip_fail(e, "creating timing events");
  hipStream_t s = (hipStream_t)stream;
  *best = -1;
  float best_ms = 0.0f;
  for (int32_t i = 0; i < n_candidates; ++i) {
    float t = -1.0f;
    if (rt_plan_set_tiling(plan, &candidates[i]) == RT_OK &&
        rt::workspace_bytes(*plan, sample->n) <= workspace_bytes) {
      auto launch = [&]() {
        return rt_accumulate(plan, sample, traces, workspace, workspace_bytes, stream);
      };
      const int st = time_launches(launch, reps, s, ev, &t);
      if (st == RT_E_HIP) {
        (void)rt_plan_set_tiling(plan, &keep);
        return st;   // a device error ends the search
      }
      if (st != RT_OK) t = -1.0f;   // a shape the library refuses: skipped
    }
    if (ms) ms[i] = t;
    if (t >= 0.0f && (*best < 0 || t < best_ms)) {
      *best = i;
      best_ms = t;
    }
  }
  if (*best < 0) {
    (void)rt_plan_set_tiling(plan, &keep);
    return rt_fail(RT_E_UNSUPPORTED,
                   "no candidate could be timed (refused shapes, or a workspace too small for all)");
  }
  return rt_plan_set_tiling(plan, &candidates[*best]);
}

int rt_batch_autotune(const rt_shower *showers, int32_t n_showers, int precision, double k,
                      const rt_batch_options *candidates, int32_t n_candidates, void *workspace,
                      size_t workspace_bytes, int32_t reps, void *stream, float *ms,
                      int32_t *best) {
  if (!showers || n_showers < 1 || !candidates || n_candidates < 1 || !best)
    return rt_fail(RT_E_INVALID, "showers, candidates and best are required");
  if (reps < 1) return rt_fail(RT_E_INVALID, "reps must be >= 1");
  Events ev;
  hipError_t e = ev.create();
  if (e != hipSuccess) return rt_hip_fail(e, "creating timing events");
  hipStream_t s = (hipStream_t)stream;
  *best = -1;
  float best_ms = 0.0f;
  for (int32_t i = 0; i < n_candidates; ++i) {
    float t = -1.0f;
    rt_batch_options o = candidates[i];
    o.direct_launch = 1;   // every launch enqueues its kernels (no graph per candidate)
    rt_batch *b = nullptr;
    if (rt_batch_create(&b, showers, n_showers, precision, k, &o) == RT_OK) {
      size_t need = 0;
      (void)rt_batch_workspace_bytes(b, &need);
      if (need <= workspace_bytes) {
        auto launch = [&]() { return rt_batch_launch(b, workspace, workspace_bytes, stream); };
        const int st = time_launches(launch, reps, s, ev, &t);
        // the batch's host tables must outlive its launches' table copies
        (void)hipStreamSynchronize(s);
        if (st == RT_E_HIP) {
          (void)rt_batch_destroy(b);
          return st;
        }
        if (st != RT_OK) t = -1.0f;
      }
      (void)rt_batch_destroy(b);
    }
    if (ms) ms[i] = t;
    if (t >= 0.0f && (*best < 0 || t < best_ms)) {
      *best = i;
      best_ms = t;
    }
  }
  if (*best < 0)
    return rt_fail(RT_E_UNSUPPORTED,
                   "no candidate could be timed (refused options, or a workspace too small for all)");
  return RT_OK;
}

}  // extern "C"
