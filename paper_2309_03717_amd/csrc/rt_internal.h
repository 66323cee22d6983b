// rt_internal.h -- host-side plan object and kernel launchers shared by the
// translation units of libradtrace.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "../../include/radtrace.h"
#include "rt_device.h"

struct rt_plan {
  rt_detector det;        // device pointers owned by the caller
  rt_medium med;
  int formalism;          // rt_formalism
  int precision;          // rt_precision
  double k;
  rt::Consts c;
  int device;
  int num_cus;
  size_t lds_per_block;   // bytes of LDS one workgroup may use
  size_t lds_per_cu;      // bytes of LDS per compute unit
  // tiling (0 = automatic)
  int at_user, splits_user, block_user, seg_user;
  int64_t pass_user;
  // one-shot profiling events around the next deposit kernel
  hipEvent_t ev_start, ev_stop;
};

namespace rt {

struct Tiling {
  int at;          // antennas per tile
  int seg_len;     // bins per segment
  int n_segs;
  int n_atiles;
  int splits;
  int block;
  int64_t pass_tracks;        // tracks per pass (a multiple of 64)
  int64_t per_split;          // tracks per split of a pass (a multiple of 64)
  int64_t blocks_per_split;   // the same in wave blocks of 64 tracks
  size_t lds_bytes;
};

// Effective launch shape of a plan for n tracks.
Tiling choose_tiling(const rt_plan &p, int64_t n);
size_t acc_bytes(int precision);
// Bytes of the per-track prepared media values for n tracks (0 if none).
size_t prep_bytes(const rt_plan &p, int64_t n);
size_t workspace_bytes(const rt_plan &p, int64_t n);

TrackPtrs track_ptrs(const rt_tracks &t);
AntPtrs ant_ptrs(const rt_detector &d);

// Launchers: enqueue on `stream`, return the hipGetLastError() status.
hipError_t launch_forward(const rt_plan &p, const rt_tracks &t, void *traces, void *workspace,
                          hipStream_t stream);
// ZHS vector-Jacobian product (adjoint.hip).
size_t vjp_workspace_bytes(const rt_plan &p, int64_t n);

// Tabulated medium: bytes of the cumulative table F at the nodes (0 for the
// other media), and the one-thread kernel that writes it (the summation
// order every lookup relies on).
size_t table_bytes(const rt_plan &p);
void launch_tab_cells(const rt_plan &p, double *cells, hipStream_t stream);
hipError_t launch_vjp(const rt_plan &p, const rt_tracks &t, const void *grad, double *g_qw,
                      double *g_p0, double *g_p1, double *g_n0, void *workspace,
                      hipStream_t stream);

hipError_t launch_propagate(const rt_plan &p, const rt_tracks &t, double *t_arrival,
                            int32_t *bin, hipStream_t stream);

}  // namespace rt

// Thread-local error text and shared argument checks (api.hip). The checks
// set the error text and return an rt_status.
void rt_set_error(const std::string &msg);
int rt_fail(int status, const std::string &msg);
int rt_hip_fail(hipError_t e, const char *what);
int rt_check_setup(const rt_detector *det, const rt_medium *med, int formalism, int precision,
                   double k);
int rt_check_tracks(const rt_tracks *t, int64_t n_antennas);
// The kernels' constants of one (detector, medium, prefactor) set-up: time
// binning, refractivity and the fields of every medium kind (zero where the
// kind does not use them). Single plans and batches both take them from here.
void rt_fill_consts(const rt_detector &det, const rt_medium &med, double k, rt::Consts &c);
// Current device, its compute units and LDS bytes per workgroup and per CU.
int rt_device_info(int *dev, int *num_cus, size_t *lds_block, size_t *lds_cu);
