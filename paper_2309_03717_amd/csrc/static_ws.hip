// static_ws.hip -- rt_accumulate_static: the deposit call of rt_accumulate
// for callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid allocation). Its
// workspace is a fixed-size device array of this library instead of a
// caller buffer.
#include <mutex>
#include <string>

#include "rt_internal.h"

// The workspace of rt_accumulate_static on each device: records, the
// fixed-point region and the split partials of one call (every byte a call
// reads is written earlier in the same call, so nothing is cleared). Each
// device holds its own copy until the process ends.
static __device__ __align__(256) unsigned char scratch[RT_STATIC_WORKSPACE_BYTES];

namespace {

constexpr size_t kScratchBytes = RT_STATIC_WORKSPACE_BYTES;

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on device `dev` (current), looked up once.
// In host code the array's name is only a stand-in for the symbol; the
// address kernels may use is this one.
int scratch_on(int dev, void **ptr) {
  if (dev < 0 || dev >= kMaxDevices)
    return rt_fail(RT_E_UNSUPPORTED, "device index beyond " + std::to_string(kMaxDevices));
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return rt_hip_fail(e, "looking up the static workspace");
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return RT_OK;
}

}  // namespace

extern "C" {

int rt_accumulate_static(rt_plan *plan, const rt_tracks *tracks, void *traces, void *stream) {
  if (!plan) return rt_fail(RT_E_INVALID, "plan is NULL");
  int s = rt_check_tracks(tracks, plan->det.n_antennas);
  if (s != RT_OK) return s;
  if (tracks->n == 0) return RT_OK;
  if (!traces) return rt_fail(RT_E_INVALID, "traces is NULL");
  if (tracks->n >= ((int64_t)1 << 31))
    return rt_fail(RT_E_UNSUPPORTED, "at most 2^31 - 1 tracks per call");
  const size_t need = rt::workspace_bytes(*plan, tracks->n);
  if (need > kScratchBytes)
    return rt_fail(RT_E_WORKSPACE,
                   "this call needs " + std::to_string(need) + " bytes of workspace; the static "
                   "workspace holds " + std::to_string(kScratchBytes) +
                   ": pass fewer tracks per call (or use rt_accumulate with a caller buffer)");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return rt_hip_fail(e, "querying the current device");
  if (dev != plan->device)
    return rt_fail(RT_E_INVALID, "the current device is not the plan's device");
  void *ws = nullptr;
  s = scratch_on(dev, &ws);
  if (s != RT_OK) return s;
  // the same checks and launches as rt_accumulate, on the static workspace
  return rt_accumulate(plan, tracks, traces, ws, kScratchBytes, stream);
}

}  // extern "C"
