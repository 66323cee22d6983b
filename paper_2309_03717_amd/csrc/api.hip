// api.hip -- the extern "C" entry points of include/radtrace.h: argument
// validation, plan set-up and launches on the caller's stream.
#include <cmath>
#include <cstdio>
#include <new>
#include <string>

#include "rt_deposit.h"   // kMergeThreads
#include "rt_internal.h"

static thread_local std::string g_last_error;

void rt_set_error(const std::string &msg) { g_last_error = msg; }

static int fail(int status, const std::string &msg) {
  rt_set_error(msg);
  return status;
}

static bool is_finite(double x) { return std::isfinite(x); }

static int hip_fail(hipError_t e, const char *what) {
  return fail(RT_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

int rt_check_tracks(const rt_tracks *t, int64_t n_antennas) {
  if (!t) return fail(RT_E_INVALID, "tracks is NULL");
  if (t->n < 0) return fail(RT_E_INVALID, "tracks->n < 0");
  if (t->n == 0) return RT_OK;
  if (!t->x0 || !t->y0 || !t->z0 || !t->t0 || !t->x1 || !t->y1 || !t->z1 || !t->t1 || !t->bx ||
      !t->by || !t->bz || !t->qw)
    return fail(RT_E_INVALID, "a track array pointer is NULL");
  if (n_antennas > 0 && t->n > INT64_MAX / n_antennas)
    return fail(RT_E_INVALID, "n_tracks * n_antennas overflows");
  return RT_OK;
}

static int check_tracks(const rt_plan *p, const rt_tracks *t) {
  return rt_check_tracks(t, p->det.n_antennas);
}

int rt_check_setup(const rt_detector *det, const rt_medium *med, int formalism, int precision,
                   double k) {
  if (!det || !med) return fail(RT_E_INVALID, "detector or medium is NULL");
  if (det->n_antennas < 1) return fail(RT_E_INVALID, "detector needs at least one antenna");
  if (det->n_antennas > INT32_MAX)
    return fail(RT_E_UNSUPPORTED, "at most 2^31 - 1 antennas per detector");
  if (!det->x || !det->y || !det->z || !det->t_start)
    return fail(RT_E_INVALID, "an antenna array pointer is NULL");
  if (!(det->dt > 0.0) || !is_finite(det->dt)) return fail(RT_E_INVALID, "dt must be finite and > 0");
  if (det->n_bins < 1) return fail(RT_E_INVALID, "n_bins must be >= 1");
  if ((int64_t)det->n_bins * 3 > INT32_MAX / 2) return fail(RT_E_UNSUPPORTED, "n_bins too large");
  if (formalism != RT_ENDPOINT && formalism != RT_ZHS)
    return fail(RT_E_INVALID, "formalism must be RT_ENDPOINT or RT_ZHS");
  if (precision != RT_FP64 && precision != RT_MIXED)
    return fail(RT_E_INVALID, "precision must be RT_FP64 or RT_MIXED");
  if (med->kind != RT_UNIFORM && med->kind != RT_EXPONENTIAL && med->kind != RT_TABULATED &&
      med->kind != RT_SPHERICAL)
    return fail(RT_E_INVALID,
                "medium kind must be RT_UNIFORM, RT_EXPONENTIAL, RT_TABULATED or RT_SPHERICAL");
  if (!(med->n0_minus_1 >= 0.0) || !is_finite(med->n0_minus_1))
    return fail(RT_E_INVALID, "n0_minus_1 must be finite and >= 0");
  if ((med->kind == RT_EXPONENTIAL || med->kind == RT_SPHERICAL) &&
      (!(med->scale_height > 0.0) || !is_finite(med->scale_height)))
    return fail(RT_E_INVALID, "scale_height must be finite and > 0");
  if (med->kind == RT_SPHERICAL && (!(med->earth_radius >= 1000.0) || !is_finite(med->earth_radius)))
    return fail(RT_E_INVALID, "earth_radius must be finite and >= 1000 m");
  if (med->kind == RT_TABULATED) {
    if (!med->table) return fail(RT_E_INVALID, "a tabulated medium needs its table");
    if (med->n_table < 2 || med->n_table > (1 << 20))
      return fail(RT_E_INVALID, "n_table must be in [2, 1048576]");
    if (!(med->table_dz > 0.0) || !is_finite(med->table_dz) || !is_finite(med->table_z0))
      return fail(RT_E_INVALID, "table_dz must be finite and > 0, table_z0 finite");
  }
  if (!is_finite(k)) return fail(RT_E_INVALID, "k must be finite");
  return RT_OK;
}

int rt_device_info(int *dev, int *num_cus, size_t *lds_block, size_t *lds_cu) {
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    return fail(RT_E_NO_DEVICE, "no HIP device is available");
  }
  if (hipGetDevice(dev) != hipSuccess) return fail(RT_E_NO_DEVICE, "hipGetDevice failed");
  int cus = 0, lb = 0, lc = 0;
  hipError_t e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, *dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lb, hipDeviceAttributeMaxSharedMemoryPerBlock, *dev);
  if (e == hipSuccess)
    e = hipDeviceGetAttribute(&lc, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, *dev);
  if (e != hipSuccess) return hip_fail(e, "querying device attributes");
  *num_cus = cus > 0 ? cus : 1;
  *lds_block = (size_t)(lb > 0 ? lb : 65536);
  *lds_cu = (size_t)(lc > 0 ? lc : (int)*lds_block);
  return RT_OK;
}

int rt_fail(int status, const std::string &msg) { return fail(status, msg); }

// Tabulated-profile fields of the constants (zero otherwise).
static void fill_table(const rt_medium &med, rt::Consts &c) {
  c.tab = c.tabF = nullptr;
  c.n_tab = 0;
  c.tz0 = 0.0;
  c.tdz = c.tinv_dz = 1.0;
  if (med.kind == RT_TABULATED) {
    c.tab = med.table;
    c.n_tab = med.n_table;
    c.tz0 = med.table_z0;
    c.tdz = med.table_dz;
    c.tinv_dz = 1.0 / med.table_dz;
  }
}
// Nodes (ascending) and weights of the n-point Gauss-Legendre rule moved to
// [0, 1], n even: the roots of the Legendre polynomial P_n by Newton's method
// in long double from the estimate cos(pi (i - 1/4) / (n + 1/2)), P_n and
// P_n' from the three-term recurrence, weights 2 / ((1 - x^2) P_n'(x)^2);
// the rule is symmetric, so each root x > 0 gives s = (1 -+ x) / 2.
static void gauss_legendre01(int n, double *s, double *w) {
  const long double pi = 3.141592653589793238462643383279502884L;
  for (int i = 1; i <= n / 2; ++i) {
    long double x = cosl(pi * ((long double)i - 0.25L) / ((long double)n + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 64; ++it) {
      long double p0 = 1.0L, p1 = x;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (x * p1 - p0) / (x * x - 1.0L);
      const long double step = p1 / dp;
      x -= step;
      if (fabsl(step) <= 1e-19L) break;
    }
    long double p0 = 1.0L, p1 = x;
    for (int k = 2; k <= n; ++k) {
      const long double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (x * p1 - p0) / (x * x - 1.0L);
    const long double wt = 1.0L / ((1.0L - x * x) * dp * dp);   // half of 2 / (...)
    s[i - 1] = (double)((1.0L - x) * 0.5L);
    s[n - i] = (double)((1.0L + x) * 0.5L);
    w[i - 1] = w[n - i] = (double)wt;
  }
}

// Spherical-Earth fields of the constants (radius, quadrature rule; zero
// otherwise).
static void fill_sphere(const rt_medium &med, rt::Consts &c) {
  c.re = c.re2 = c.re_twice = 0.0;
  for (int k = 0; k < rt::kGl; ++k) c.gl_s[k] = c.gl_w[k] = 0.0;
  if (med.kind == RT_SPHERICAL) {
    c.re = med.earth_radius;
    c.re2 = c.re * c.re;
    c.re_twice = c.re + c.re;
    gauss_legendre01(rt::kGl, c.gl_s, c.gl_w);
  }
}

void rt_fill_consts(const rt_detector &det, const rt_medium &med, double k, rt::Consts &c) {
  c.inv_c = 1.0 / 299792458.0;
  c.inv_dt = 1.0 / det.dt;
  c.k = k;
  c.n_uniform = 1.0 + med.n0_minus_1;
  c.n0m1 = med.n0_minus_1;
  c.h = med.kind == RT_EXPONENTIAL || med.kind == RT_SPHERICAL ? med.scale_height : 1.0;
  c.n0h = c.n0m1 * c.h;
  c.nbins_d = (double)det.n_bins;
  c.n_bins = det.n_bins;
  c.medium = med.kind;
  fill_table(med, c);
  fill_sphere(med, c);
  c.n0m1_dev = nullptr;
}

int rt_hip_fail(hipError_t e, const char *what) { return hip_fail(e, what); }

extern "C" {

int rt_abi_version(void) { return RT_ABI_VERSION; }

const char *rt_status_string(int status) {
  switch (status) {
    case RT_OK: return "ok";
    case RT_E_INVALID: return "invalid argument";
    case RT_E_UNSUPPORTED: return "unsupported configuration";
    case RT_E_NO_DEVICE: return "no usable HIP device";
    case RT_E_HIP: return "HIP runtime error";
    case RT_E_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

const char *rt_last_error(void) { return g_last_error.c_str(); }

int rt_plan_create(rt_plan **plan, const rt_detector *det, const rt_medium *med, int formalism,
                   int precision, double k) {
  if (!plan) return fail(RT_E_INVALID, "plan output pointer is NULL");
  *plan = nullptr;
  int st = rt_check_setup(det, med, formalism, precision, k);
  if (st != RT_OK) return st;
  int dev = 0, cus = 0;
  size_t lds_block = 0, lds_cu = 0;
  st = rt_device_info(&dev, &cus, &lds_block, &lds_cu);
  if (st != RT_OK) return st;

  rt_plan *p = new (std::nothrow) rt_plan();
  if (!p) return fail(RT_E_INVALID, "out of host memory");
  p->det = *det;
  p->med = *med;
  p->formalism = formalism;
  p->precision = precision;
  p->k = k;
  p->device = dev;
  p->num_cus = cus;
  p->lds_per_block = lds_block;
  p->lds_per_cu = lds_cu;
  p->at_user = p->splits_user = p->block_user = p->seg_user = 0;
  p->pass_user = 0;
  p->ev_start = p->ev_stop = nullptr;
  rt_fill_consts(*det, *med, k, p->c);
  *plan = p;
  return RT_OK;
}

int rt_plan_destroy(rt_plan *plan) {
  delete plan;
  return RT_OK;
}

int rt_plan_set_tiling(rt_plan *plan, const rt_tiling *tl) {
  if (!plan || !tl) return fail(RT_E_INVALID, "plan or tiling is NULL");
  const int at = tl->antennas_per_block, splits = tl->track_splits;
  const int block = tl->block_threads, seg_in = tl->bins_per_segment;
  if (at < 0 || at > rt::kMaxTile) return fail(RT_E_INVALID, "antennas_per_block must be in [0, 8]");
  if (splits < 0) return fail(RT_E_INVALID, "track_splits must be >= 0");
  if (block != 0 && (block < 64 || block > 1024 || block % 64))
    return fail(RT_E_INVALID, "block_threads must be a multiple of 64 in [64, 1024]");
  if (seg_in < 0 || (seg_in > 0 && seg_in % 64 && seg_in != plan->det.n_bins))
    return fail(RT_E_INVALID, "bins_per_segment must be a multiple of 64 or n_bins");
  if (tl->tracks_per_pass < 0 || tl->tracks_per_pass % 64)
    return fail(RT_E_INVALID, "tracks_per_pass must be a non-negative multiple of 64");
  const size_t acc = rt::acc_bytes(plan->precision);
  const int seg = seg_in > 0 ? std::min(seg_in, plan->det.n_bins) : 0;
  // a tile row holds the segment's bins plus the formalism's padding bins
  const int pad = rt::tile_pad(plan->formalism);
  if (seg > 0 && (size_t)(seg + pad) * 3 * acc * (at > 0 ? at : 1) > plan->lds_per_block)
    return fail(RT_E_UNSUPPORTED, "tile does not fit in LDS");
  if (at > 0 && seg == 0 && (size_t)at * (plan->det.n_bins + pad) * 3 * acc > plan->lds_per_block)
    return fail(RT_E_UNSUPPORTED,
                "antennas_per_block x n_bins does not fit in LDS; also set bins_per_segment");
  plan->at_user = at;
  plan->splits_user = splits;
  plan->block_user = block;
  plan->seg_user = seg_in;
  plan->pass_user = tl->tracks_per_pass;
  return RT_OK;
}

int rt_plan_get_tiling(const rt_plan *plan, int64_t n_tracks, rt_tiling *out) {
  if (!plan || !out) return fail(RT_E_INVALID, "plan or out is NULL");
  if (n_tracks < 0) return fail(RT_E_INVALID, "n_tracks < 0");
  rt::Tiling t = rt::choose_tiling(*plan, n_tracks);
  out->antennas_per_block = t.at;
  out->track_splits = t.splits;
  out->block_threads = t.block;
  out->bins_per_segment = t.seg_len;
  out->tracks_per_pass = t.pass_tracks;
  return RT_OK;
}

int rt_plan_workspace_bytes(const rt_plan *plan, int64_t n_tracks, size_t *bytes) {
  if (!plan || !bytes) return fail(RT_E_INVALID, "plan or bytes is NULL");
  if (n_tracks < 0) return fail(RT_E_INVALID, "n_tracks < 0");
  *bytes = n_tracks == 0 ? 0 : rt::workspace_bytes(*plan, n_tracks);
  return RT_OK;
}

int rt_accumulate(rt_plan *plan, const rt_tracks *tracks, void *traces, void *workspace,
                  size_t workspace_bytes, void *stream) {
  if (!plan) return fail(RT_E_INVALID, "plan is NULL");
  int s = check_tracks(plan, tracks);
  if (s != RT_OK) return s;
  if (tracks->n == 0) return RT_OK;
  if (!traces) return fail(RT_E_INVALID, "traces is NULL");
  if (tracks->n >= ((int64_t)1 << 31))
    return fail(RT_E_UNSUPPORTED, "at most 2^31 - 1 tracks per call; stream larger inputs in chunks");
  {
    // every launch must fit the hardware grid (fewer than 2^32 threads, int
    // workgroup indices): the deposit of a pass has tiles x segments x splits
    // workgroups, the merge antennas x segments
    const rt::Tiling tl = rt::choose_tiling(*plan, tracks->n);
    const int64_t deposit = (int64_t)tl.n_atiles * tl.n_segs * tl.splits;
    const int64_t merge = plan->det.n_antennas * tl.n_segs;
    const int64_t limit = (int64_t)UINT32_MAX;
    if (deposit * tl.block > limit || merge * rt::kMergeThreads > limit)
      return fail(RT_E_UNSUPPORTED,
                  "the array needs " + std::to_string(deposit) + " deposit workgroups of " +
                      std::to_string(tl.block) + " threads per pass: split the antennas over "
                      "several plans (or set fewer track splits)");
  }
  size_t need = rt::workspace_bytes(*plan, tracks->n);
  if (!workspace || workspace_bytes < need)
    return fail(RT_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes, got " +
                                    std::to_string(workspace ? workspace_bytes : 0));
  (void)hipGetLastError();
  hipError_t e = rt::launch_forward(*plan, *tracks, traces, workspace, (hipStream_t)stream);
  plan->ev_start = plan->ev_stop = nullptr;
  if (e != hipSuccess) return hip_fail(e, "launching the deposit kernels");
  return RT_OK;
}

int rt_plan_vjp_workspace_bytes(const rt_plan *plan, int64_t n_tracks, size_t *bytes) {
  if (!plan || !bytes) return fail(RT_E_INVALID, "plan or bytes is NULL");
  if (n_tracks < 0) return fail(RT_E_INVALID, "n_tracks < 0");
  *bytes = rt::vjp_workspace_bytes(*plan, n_tracks);
  return RT_OK;
}

static int vjp_call(rt_plan *plan, const rt_tracks *tracks, const void *grad_traces,
                    double *grad_qw, double *grad_p0, double *grad_p1, double *grad_n0m1,
                    void *workspace, size_t workspace_bytes, void *stream);

int rt_zhs_vjp(rt_plan *plan, const rt_tracks *tracks, const void *grad_traces, double *grad_qw,
               double *grad_p0, double *grad_p1, double *grad_n0m1, void *workspace,
               size_t workspace_bytes, void *stream) {
  if (!plan) return fail(RT_E_INVALID, "plan is NULL");
  if (plan->formalism != RT_ZHS) return fail(RT_E_INVALID, "rt_zhs_vjp needs an RT_ZHS plan");
  return vjp_call(plan, tracks, grad_traces, grad_qw, grad_p0, grad_p1, grad_n0m1, workspace,
                  workspace_bytes, stream);
}

int rt_endpoint_vjp(rt_plan *plan, const rt_tracks *tracks, const void *grad_traces,
                    double *grad_qw, double *grad_p0, double *grad_p1, double *grad_n0m1,
                    void *workspace, size_t workspace_bytes, void *stream) {
  if (!plan) return fail(RT_E_INVALID, "plan is NULL");
  if (plan->formalism != RT_ENDPOINT)
    return fail(RT_E_INVALID, "rt_endpoint_vjp needs an RT_ENDPOINT plan");
  return vjp_call(plan, tracks, grad_traces, grad_qw, grad_p0, grad_p1, grad_n0m1, workspace,
                  workspace_bytes, stream);
}

static int vjp_call(rt_plan *plan, const rt_tracks *tracks, const void *grad_traces,
                    double *grad_qw, double *grad_p0, double *grad_p1, double *grad_n0m1,
                    void *workspace, size_t workspace_bytes, void *stream) {
  int s = check_tracks(plan, tracks);
  if (s != RT_OK) return s;
  if (!grad_traces || !grad_n0m1) return fail(RT_E_INVALID, "grad_traces or grad_n0m1 is NULL");
  if (tracks->n > 0 && (!grad_qw || !grad_p0 || !grad_p1))
    return fail(RT_E_INVALID, "a per-track gradient pointer is NULL");
  if (tracks->n >= ((int64_t)1 << 31) - 1024)
    return fail(RT_E_UNSUPPORTED, "at most 2^31 - 1025 tracks per call");
  if (plan->det.n_antennas * 256 > (int64_t)UINT32_MAX)   // one 256-thread phi workgroup each
    return fail(RT_E_UNSUPPORTED, "the adjoints take at most 16,777,215 antennas per plan");
  size_t need = rt::vjp_workspace_bytes(*plan, tracks->n);
  if (!workspace || workspace_bytes < need)
    return fail(RT_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes");
  (void)hipGetLastError();
  hipError_t e = rt::launch_vjp(*plan, *tracks, grad_traces, grad_qw, grad_p0, grad_p1, grad_n0m1,
                                workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launching the adjoint kernels");
  return RT_OK;
}

int rt_plan_set_n0m1_device(rt_plan *plan, const double *n0m1) {
  if (!plan) return fail(RT_E_INVALID, "plan is NULL");
  plan->c.n0m1_dev = n0m1;
  return RT_OK;
}

int rt_plan_set_timing_events(rt_plan *plan, void *start_event, void *stop_event) {
  if (!plan) return fail(RT_E_INVALID, "plan is NULL");
  if ((start_event == nullptr) != (stop_event == nullptr))
    return fail(RT_E_INVALID, "give both events or neither");
  plan->ev_start = (hipEvent_t)start_event;
  plan->ev_stop = (hipEvent_t)stop_event;
  return RT_OK;
}

int rt_propagate(const rt_plan *plan, const rt_tracks *tracks, double *t_arrival, int32_t *bin,
                 void *stream) {
  if (!plan) return fail(RT_E_INVALID, "plan is NULL");
  int s = check_tracks(plan, tracks);
  if (s != RT_OK) return s;
  if (tracks->n == 0 || (!t_arrival && !bin)) return RT_OK;
  (void)hipGetLastError();
  hipError_t e = rt::launch_propagate(*plan, *tracks, t_arrival, bin, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "launching the propagator kernel");
  return RT_OK;
}

}  // extern "C"
