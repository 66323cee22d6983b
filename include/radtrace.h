/*
 * radtrace.h -- C ABI of the MI355X (gfx950) track x antenna radio-emission
 * library.
 *
 * The computation (paper §2, "Overview of the radio module", Fig. 1): every
 * particle track is looped over every antenna of the array; for each pair a
 * straight-line propagator gives the distance R, the effective refractive
 * index n_eff of the path and the arrival time, and the formalism's field is
 * stored in the antenna's time trace. The two formalisms are the Endpoint and
 * the ZHS formalism (§1); Listing 2 (§4) builds a propagator from an
 * environment and a radio process from a detector and a propagator, which
 * is what rt_plan_create does here.
 *
 * Conventions for every entry point:
 *  - Units are SI: metres, seconds; velocities in units of c.
 *  - Array arguments documented as "device" are device pointers of the
 *    current HIP device (for example torch CUDA tensors' data_ptr()); they are
 *    owned by the caller and must stay valid until the work enqueued on
 *    `stream` has completed. "host" pointers are read before the call returns.
 *  - `stream` is a hipStream_t passed as void* (NULL: the null stream). All
 *    device work of a call is enqueued on it; no call allocates device
 *    memory, and no call except the autotuners synchronizes the stream, so
 *    calls may be captured into a HIP graph (rt_batch_launch with the
 *    condition stated there).
 *  - Every function returns an rt_status. On failure nothing is enqueued and
 *    rt_last_error() holds a description (per host thread).
 *    Invalid arguments give RT_E_INVALID; shapes the kernels do not support
 *    give RT_E_UNSUPPORTED; a HIP error at launch gives RT_E_HIP; a too-small
 *    workspace gives RT_E_WORKSPACE; no usable device gives RT_E_NO_DEVICE.
 *    Asynchronous faults surface at the caller's next synchronization.
 *  - A plan is used by one host thread at a time; different plans are
 *    independent.
 *
 * Trace layout: traces[a][k][c] for antenna a, bin k, component c (x, y, z),
 * row-major, element type double (RT_FP64) or float (RT_MIXED). Bin k of
 * antenna a covers arrival times [t_start[a] + k dt, t_start[a] + (k+1) dt);
 * a time exactly on an edge belongs to the bin above it, and times outside
 * [0, n_bins) bins are dropped (ZHS boxes are clipped to the window).
 */
#ifndef RADTRACE_H
#define RADTRACE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RT_ABI_VERSION 2

typedef enum {
  RT_OK = 0,
  RT_E_INVALID = 1,
  RT_E_UNSUPPORTED = 2,
  RT_E_NO_DEVICE = 3,
  RT_E_HIP = 4,
  RT_E_WORKSPACE = 5
} rt_status;

/* The two formalisms named in §1. */
typedef enum { RT_ENDPOINT = 0, RT_ZHS = 1 } rt_formalism;

/* RT_FP64: all arithmetic and the traces in double precision.
 * RT_MIXED: tracks carry beta and qw as float and the traces are float; the
 * arithmetic runs in double precision. Endpoint: arrival time, distance and
 * bin exactly as RT_FP64 (the same bins), amplitude from refined hardware
 * reciprocals (relative error a few 1e-15), LDS accumulation in double.
 * ZHS: arrival times to a few 1e-15 (the box is continuous in them), box
 * amplitude and weights at single-precision accuracy (hardware estimates,
 * 5e-8), LDS accumulation in 64-bit fixed point (see rt_accumulate). */
typedef enum { RT_FP64 = 0, RT_MIXED = 1 } rt_precision;

/* Refractive-index model of the environment the propagator is built from
 * (§2, Listing 2; media whose properties vary, §1):
 *   RT_UNIFORM:     n(z) = 1 + n0_minus_1
 *   RT_EXPONENTIAL: n(z) = 1 + n0_minus_1 * exp(-z / scale_height)
 *   RT_TABULATED:   n(z) = 1 + n0_minus_1 * f(z), f piecewise linear through
 *                   table[i] at table_z0 + i * table_dz, constant beyond the
 *                   first and last node (a measured or layered atmosphere)
 *   RT_SPHERICAL:   n(p) = 1 + n0_minus_1 * exp(-h(p) / scale_height) with h
 *                   the height above a spherical Earth of radius earth_radius
 *                   centred at (0, 0, -earth_radius): z = 0 is the ground at
 *                   the origin of the array frame, and the ground falls away
 *                   with horizontal distance (a curved-Earth atmosphere)
 * The straight path from height zp to an antenna at height za sees the path
 * mean of n: n_eff = 1 + n0_minus_1 * scale_height * (exp(-za/h) -
 * exp(-zp/h)) / (zp - za) for the exponential profile, 1 + n0_minus_1 *
 * (F(zp) - F(za)) / (zp - za) for the tabulated one with F the exact integral
 * of f (whole-cell trapezoids summed from the first node up, plus the part of
 * the last cell); the local index at the midpoint height when |zp - za| <
 * 1 mm. Over the spherical Earth the path mean has no closed form: it is
 * taken by 8-point Gauss-Legendre quadrature along the straight path from the
 * emission point P to the antenna X,
 *   n_eff = 1 + n0_minus_1 * sum_k w_k exp(-h(P + s_k (X - P)) / scale_height)
 * with the nodes s_k and weights w_k of the rule on [0, 1] (ascending s_k,
 * sum w_k = 1; accurate to double rounding for these profiles), and h(q) =
 * rho2 / (sqrt(rho2 + R^2) + R), rho2 = (qx^2 + qy^2) + qz (qz + 2R), which is
 * |q - C| - R without cancellation. Plans, adjoints and batches accept every
 * medium. */
typedef enum {
  RT_UNIFORM = 0,
  RT_EXPONENTIAL = 1,
  RT_TABULATED = 2,
  RT_SPHERICAL = 3
} rt_medium_kind;

typedef struct {
  int32_t kind;          /* rt_medium_kind */
  double n0_minus_1;     /* refractivity scale, >= 0 (at z = 0 if exponential
                            or spherical) */
  double scale_height;   /* metres, > 0 (exponential and spherical only) */
  const double *table;   /* device, n_table finite values (tabulated only); the
                            plan keeps the pointer: it must outlive the plan */
  int32_t n_table;       /* 2 .. 1048576 (tabulated only) */
  double table_z0;       /* height of table[0] (m) */
  double table_dz;       /* node spacing (m), > 0 */
  double earth_radius;   /* metres, finite and >= 1000 (spherical only) */
} rt_medium;

/* The antenna collection (§2, "detector" in Listing 2). Device arrays of
 * n_antennas doubles. The plan keeps these pointers: they must outlive it. */
typedef struct {
  int64_t n_antennas;
  const double *x, *y, *z;   /* device: antenna positions (m) */
  const double *t_start;     /* device: time of the left edge of bin 0 (s) */
  double dt;                 /* bin width (s), > 0 */
  int32_t n_bins;            /* bins per trace, >= 1 */
} rt_detector;

/* Straight particle tracks, structure of arrays, n of each (device).
 * Track i starts at (x0,y0,z0) at time t0 and ends at (x1,y1,z1) at t1 with
 * constant velocity (bx,by,bz) (units of c); qw is its charge (units of e)
 * times its statistical weight. bx..qw are double for RT_FP64 plans and float
 * for RT_MIXED plans. Non-finite inputs produce no contribution. */
typedef struct {
  int64_t n;
  const double *x0, *y0, *z0, *t0;
  const double *x1, *y1, *z1, *t1;
  const void *bx, *by, *bz, *qw;
} rt_tracks;

typedef struct rt_plan rt_plan;   /* opaque; host-side metadata only */

/* Version of this ABI (RT_ABI_VERSION). */
int rt_abi_version(void);

/* Static description of a status code. */
const char *rt_status_string(int status);

/* Description of the last failure on this host thread ("" if none). */
const char *rt_last_error(void);

/* A radio process for one detector, medium, formalism and precision (the
 * analogue of make_radio_process_CoREAS / _ZHS of Listing 2, with a HIP
 * stream in place of a thread count). k is the field prefactor:
 * e / (4 pi eps0 c) = 4.80320471518522e-18 V s for SI fields (1 for unit
 * tests). The plan reads no device memory; it chooses a tiling from the
 * device's compute-unit count and LDS size, which rt_plan_set_tiling can
 * override.
 * Output: *plan (host object, free with rt_plan_destroy). */
int rt_plan_create(rt_plan **plan, const rt_detector *det, const rt_medium *med,
                   int formalism, int precision, double k);

/* Frees a plan (NULL is accepted). Does not touch device memory. */
int rt_plan_destroy(rt_plan *plan);

/* Launch shape of the deposit kernels. In rt_plan_set_tiling a zero field
 * keeps the automatic choice.
 *  antennas_per_block: antennas whose traces one workgroup keeps in LDS (1-8)
 *  track_splits: track ranges per pass, merged in fixed order afterwards
 *  block_threads: workgroup size, a multiple of 64 in [64, 1024] (automatic:
 *                 1024, four waves per SIMD beside one trace tile per CU)
 *  bins_per_segment: bins per LDS trace segment, a multiple of 64 (or
 *                    n_bins); segments split long traces across workgroups
 *  tracks_per_pass: a call deposits its tracks in consecutive passes of at
 *                   most this many tracks (a multiple of 64), so that the
 *                   per-track records of a pass stay resident in the
 *                   last-level cache while every antenna tile streams them
 * Results do not depend on the tiling beyond floating-point summation
 * order (RT_MIXED ZHS calls: not at all, see rt_accumulate); bins never
 * change. */
typedef struct {
  int32_t antennas_per_block;
  int32_t track_splits;
  int32_t block_threads;
  int32_t bins_per_segment;
  int64_t tracks_per_pass;
} rt_tiling;

/* Overrides the launch shape (tiling: host, read during the call). */
int rt_plan_set_tiling(rt_plan *plan, const rt_tiling *tiling);

/* The launch shape the plan uses for a call with n_tracks tracks (out:
 * host). */
int rt_plan_get_tiling(const rt_plan *plan, int64_t n_tracks, rt_tiling *out);

/* Device workspace (bytes) rt_accumulate needs for a call with n_tracks
 * tracks. */
int rt_plan_workspace_bytes(const rt_plan *plan, int64_t n_tracks, size_t *bytes);

/* The hot loop (§2): for every track and every antenna, propagate both ends,
 * then add the formalism's contribution into traces (device, [M][n_bins][3],
 * += so that track chunks can be streamed in consecutive calls):
 *   Endpoint: at each end an impulse  s k qw [r x (r x beta)] /
 *             ((1 - n_src beta.r) R dt)  in the bin of that end's arrival,
 *             s = +1 at the start and -1 at the end, n_src the local index.
 *   ZHS:      the segment's vector potential, a box between the two arrival
 *             times whose time integral is k qw beta_perp (t1 - t0) / R_mid
 *             (beta_perp and R_mid at the segment midpoint), averaged over
 *             every bin it overlaps.
 * workspace: device, >= rt_plan_workspace_bytes(plan, tracks->n) bytes, used
 * as scratch by this call only. tracks->n == 0 is a no-op; at most 2^31 - 1
 * tracks per call (RT_E_UNSUPPORTED beyond: stream larger inputs in
 * chunks). Partial traces of track splits are merged in a fixed order (no
 * float atomics in global memory), so a call is repeatable for a fixed
 * tiling up to the order of LDS additions within a workgroup. RT_MIXED ZHS
 * calls accumulate in 64-bit fixed point instead: every deposit is rounded to
 * a power-of-two unit chosen per call from the tracks (so that no sum can
 * overflow) and summed exactly, which makes their traces bitwise identical
 * for any tiling, launch and repetition; a call whose tracks admit no such
 * unit (a track midpoint inside the antennas' bounding box, or one track
 * whose deposit bound dwarfs the others) accumulates in double like the
 * other modes. */
int rt_accumulate(rt_plan *plan, const rt_tracks *tracks, void *traces, void *workspace,
                  size_t workspace_bytes, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the call
 * of rt_accumulate with the workspace taken from a device array of
 * RT_STATIC_WORKSPACE_BYTES bytes that the library holds on each device until
 * the process ends, so the caller passes only the tracks and the traces (as
 * for rt_accumulate: device, [M][n_bins][3], +=). The call allocates
 * nothing. A call whose workspace (rt_plan_workspace_bytes) exceeds the array
 * returns RT_E_WORKSPACE with the sizes in rt_last_error (pass fewer tracks
 * per call). The current device must be the plan's (RT_E_INVALID
 * otherwise). Every call on one device uses the same array: calls that
 * overlap in time on one device (two streams, two host threads) race and
 * must be serialised by the caller; consecutive calls on one stream are
 * safe. Results equal those of rt_accumulate with the same tiling. */
#define RT_STATIC_WORKSPACE_BYTES ((size_t)64 << 20)
int rt_accumulate_static(rt_plan *plan, const rt_tracks *tracks, void *traces, void *stream);

/* Refractivity in device memory (the differentiable workflow, where n0 - 1
 * is a device tensor that changes between calls): with n0m1 non-NULL, every
 * later call on this plan (rt_accumulate, rt_propagate, the VJPs) reads
 * n0 - 1 from that device double when its kernels run, in place of
 * med->n0_minus_1 of rt_plan_create, so no host copy of it is needed;
 * NULL returns to med->n0_minus_1. The pointer is kept by the plan and must
 * stay valid while work of those calls can run; the value is not validated
 * (it should be finite and >= 0, as for rt_medium). The medium kind, scale
 * height, table and Earth radius stay those of rt_plan_create (§1: the
 * environment the propagator is built from). */
int rt_plan_set_n0m1_device(rt_plan *plan, const double *n0m1);

/* Profiling aid: the next rt_accumulate call on this plan records
 * start_event on its stream immediately before its deposit kernel and
 * stop_event immediately after it, then forgets both. The events are
 * hipEvent_t handles passed as void*, created and owned by the caller (with
 * timing enabled); NULL for both clears a pending request. */
int rt_plan_set_timing_events(rt_plan *plan, void *start_event, void *stop_event);

/* The propagator alone (§2; the "simple" radio propagator of Listing 2) for
 * every (end e, track i, antenna a), stored at index (e * n + i) * M + a:
 *   t_arrival (device double, may be NULL): arrival time (s)
 *   bin (device int32, may be NULL): bin index, -1 outside the window.
 * These are the exact times and bins rt_accumulate uses. */
int rt_propagate(const rt_plan *plan, const rt_tracks *tracks, double *t_arrival, int32_t *bin,
                 void *stream);

/* The track filter (§2, Fig. 1: each track is checked for relevance to the
 * radio calculation before the antenna loop). Copies the tracks of `in` that
 * can radiate to the first n_kept entries of `out`, in their input order:
 * a track is kept when every field is finite, |qw| > qw_min, some velocity
 * component is nonzero and its end differs from its start in position or
 * time. With qw_min = 0 every dropped track contributes exactly nothing to
 * either formalism, so rt_accumulate on the kept tracks equals it on all of
 * them up to floating-point summation order; qw_min > 0 also drops the
 * tracks of smaller weight, by choice.
 *   in: device tracks (n >= 0; bx, by, bz, qw double for RT_FP64, float for
 *       RT_MIXED)
 *   out: device arrays of the same types whose capacity out->n is >= in->n;
 *        must not overlap `in`
 *   n_kept: device, one int64, written with the number of kept tracks (read
 *           it after the stream reaches this call)
 *   workspace: device, >= rt_filter_workspace_bytes(in->n) bytes, used by
 *              this call only
 * Errors: RT_E_INVALID (NULL pointers, qw_min negative or not finite, a
 * capacity below in->n), RT_E_WORKSPACE, RT_E_UNSUPPORTED (more than
 * (2^31 - 1) * 256 tracks). */
int rt_filter_tracks(const rt_tracks *in, int precision, double qw_min, const rt_tracks *out,
                     int64_t *n_kept, void *workspace, size_t workspace_bytes, void *stream);

/* Device workspace (bytes) rt_filter_tracks needs for n_tracks tracks. */
int rt_filter_workspace_bytes(int64_t n_tracks, size_t *bytes);

/* Device workspace (bytes) rt_zhs_vjp or rt_endpoint_vjp (by the plan's
 * formalism) needs for n_tracks tracks. */
int rt_plan_vjp_workspace_bytes(const rt_plan *plan, int64_t n_tracks, size_t *bytes);

/* Vector-Jacobian product of the ZHS traces (the differentiable form of the
 * ZHS deposit of rt_accumulate; plan must be RT_ZHS). Given the upstream
 * gradient grad_traces = dL/dA of a scalar loss L with respect to the traces
 * (device, [M][n_bins][3], the plan's trace type), writes the exact
 * derivatives of L with respect to each track's weight qw, its start point P0
 * and end point P1, and the refractivity n0_minus_1, with the velocity and
 * the emission times t0, t1 held fixed (piecewise: the derivative of a box
 * edge that sits exactly on a bin edge is the right derivative):
 *   grad_qw   device double [n]
 *   grad_p0   device double [3][n]  (x, y, z rows)
 *   grad_p1   device double [3][n]
 *   grad_n0m1 device double [1]     (sum over this call's tracks)
 * All outputs are overwritten; for streamed chunks the caller sums grad_n0m1.
 * Tracks with a non-finite field get zero gradients. The per-track gradients
 * do not depend on any launch shape; grad_n0m1 is summed in a fixed order.
 * workspace: device, >= rt_plan_vjp_workspace_bytes(plan, tracks->n). */
int rt_zhs_vjp(rt_plan *plan, const rt_tracks *tracks, const void *grad_traces, double *grad_qw,
               double *grad_p0, double *grad_p1, double *grad_n0m1, void *workspace,
               size_t workspace_bytes, void *stream);

/* Vector-Jacobian product of the Endpoint traces (plan must be RT_ENDPOINT):
 * the derivatives of L = sum grad_traces * E with respect to each track's
 * qw, start point P0, end point P1 and n0_minus_1, with the velocity, the
 * emission times and the bin each impulse lands in held fixed (the bin is a
 * piecewise-constant function of the parameters; the jumps where an arrival
 * crosses a bin edge are not part of the derivative). Through the impulse
 * s k qw [r x (r x beta)] / ((1 - n_src beta.r) R dt): the distance and
 * direction to every antenna, and n_src = 1 + n0_minus_1 exp(-z_P / h) (its
 * height derivative enters the z component). Arguments, layouts, outputs and
 * errors as rt_zhs_vjp; workspace >= rt_plan_vjp_workspace_bytes. */
int rt_endpoint_vjp(rt_plan *plan, const rt_tracks *tracks, const void *grad_traces,
                    double *grad_qw, double *grad_p0, double *grad_p1, double *grad_n0m1,
                    void *workspace, size_t workspace_bytes, void *stream);

/* Autotuner (the launch shapes of the hot loop chosen by measurement: tile
 * width, track splits, workgroup size, bin segments, pass length). Times
 * each of the n_candidates tilings (host array) with HIP events around real
 * rt_accumulate calls on the caller's sample tracks: one warm-up call, then
 * reps >= 1 timed calls, median kept. A candidate the plan refuses, or whose
 * workspace (rt_plan_workspace_bytes with that tiling) exceeds
 * workspace_bytes, is skipped (time -1). traces (device, [M][n_bins][3]) is
 * scratch: it receives the sum of every timed call. Outputs: ms (host,
 * n_candidates floats, may be NULL) and *best (host), the index of the
 * fastest; the plan keeps that tiling (its previous tiling when none could
 * be timed: RT_E_UNSUPPORTED). This call synchronizes `stream` (it reads the
 * events) and allocates no device memory. Choosing candidates and caching
 * the result per workload are the caller's (the Python binding keeps a JSON
 * cache keyed by device and shapes). */
int rt_plan_autotune(rt_plan *plan, const rt_tracks *sample, void *traces, void *workspace,
                     size_t workspace_bytes, const rt_tiling *candidates, int32_t n_candidates,
                     int32_t reps, void *stream, float *ms, int32_t *best);

/* ------------------------------------------------------------------ batches
 *
 * Many independent showers in one launch. Each shower is one call of §2's
 * loop (its own detector, medium, formalism and tracks; the tracks of one
 * shower never reach another shower's antennas); a batch runs all of them
 * with persistent deposit kernels whose workgroups take work items
 * (antenna tile x bin segment x track split of some shower) from a shared
 * counter, longest first (one kernel for the uniform and exponential media,
 * a second for the tabulated and spherical ones when the batch has any),
 * followed by one merge kernel. Per-shower results
 * are those of rt_accumulate on that shower alone up to floating-point
 * summation order; bins never change. */
typedef struct {
  rt_detector det;   /* as for rt_plan_create; n_bins * 3 doubles of a tile
                        segment must fit in LDS after splitting (any n_bins) */
  rt_medium med;
  int32_t formalism; /* rt_formalism */
  rt_tracks tracks;  /* device; n < 2^31; n == 0 allowed */
  void *traces;      /* device, [M][n_bins][3] of the batch precision; += */
} rt_shower;

/* Launch shape of a batch (a zeroed struct, or NULL, keeps every automatic
 * choice):
 *  block_threads: workgroup size of the persistent kernels, a multiple of 64
 *                 in [64, 512] (0: 512), or 1024 together with
 *                 max_antennas_per_tile 1: one-antenna tiles, taken by one
 *                 kernel per formalism for the uniform and exponential
 *                 media (the tabulated and spherical media keep 512)
 *  items_per_cu: work items per compute unit that the track splits aim for
 *                (0: 4); more items balance better, fewer merge less
 *  max_antennas_per_tile: cap on the antennas one item keeps in LDS, 1-3
 *                         (0: 3)
 *  direct_launch: 0 captures the batch's kernels into a HIP graph on the
 *                 first rt_batch_launch (and again when the workspace
 *                 changes) and replays it; 1 enqueues the kernels on every
 *                 launch. A launch on a stream that the caller is capturing
 *                 always enqueues directly into the caller's capture.
 *  per_shower: NULL, or n_showers tilings overriding antennas_per_block
 *              (1-3), track_splits and bins_per_segment per shower (0 keeps
 *              the automatic choice; block_threads and tracks_per_pass are
 *              ignored) */
typedef struct {
  int32_t block_threads;
  int32_t items_per_cu;
  int32_t max_antennas_per_tile;
  int32_t direct_launch;
  const rt_tiling *per_shower;
} rt_batch_options;

typedef struct rt_batch rt_batch;   /* opaque; host object */

/* Plans a batch of n_showers >= 1 showers (showers, options: host, read
 * during the call) for the current device, in one precision (RT_FP64 or
 * RT_MIXED, as for rt_plan_create) and with one field prefactor k. The batch
 * keeps every device pointer of `showers`; to run new inputs, overwrite those
 * buffers and launch again. The work-item, merge and shower tables (a few
 * bytes per item) are built on the host; the launches copy them into the
 * workspace. Reads and allocates no device memory. Output: *batch (free
 * with rt_batch_destroy). */
int rt_batch_create(rt_batch **batch, const rt_shower *showers, int32_t n_showers, int precision,
                    double k, const rt_batch_options *options);

/* Frees a batch, its host tables and its graph (NULL is accepted). The
 * caller makes sure no launch of it is still running (a launch copies the
 * host tables asynchronously). */
int rt_batch_destroy(rt_batch *batch);

/* Device workspace (bytes) rt_batch_launch needs (the batch's tables, the
 * per-track records of all showers, one partial-trace slot per work item and
 * the cumulative integral of every tabulated shower's profile at its
 * nodes). */
int rt_batch_workspace_bytes(const rt_batch *batch, size_t *bytes);

/* Statistics of the plan (out: host; any pointer may be NULL): work items,
 * persistent workgroups, LDS bytes per workgroup and track x antenna pairs. */
int rt_batch_get_info(const rt_batch *batch, int64_t *n_items, int32_t *n_workgroups,
                      int64_t *lds_bytes, int64_t *pairs);

/* traces += contribution of the shower's tracks, for every shower (on
 * `stream`, see rt_batch_options.direct_launch for graphs). workspace:
 * device, >= rt_batch_workspace_bytes bytes. A launch outside a stream
 * capture first copies the batch's tables from host memory into the start of
 * the workspace on `stream`; a launch on a stream the caller is capturing
 * reuses the tables an earlier launch left in the same workspace (so launch
 * once outside the capture with that workspace first; RT_E_INVALID
 * otherwise), and the caller's graph replays rely on them staying there.
 * Launches of one batch that overlap in time race on the workspace. */
int rt_batch_launch(rt_batch *batch, void *workspace, size_t workspace_bytes, void *stream);

/* Autotuner of batches: plans the showers with each of the n_candidates
 * launch shapes (host array of rt_batch_options; direct_launch is forced to
 * 1) and times whole rt_batch_launch calls on the caller's workspace (one
 * warm-up, then reps >= 1 timed launches, median kept). Candidates the
 * planner refuses or whose workspace exceeds workspace_bytes are skipped
 * (time -1). The showers' traces are scratch: they receive every timed
 * launch. Outputs: ms (host, may be NULL), *best (host, the fastest index);
 * RT_E_UNSUPPORTED when none could be timed. Synchronizes `stream`;
 * allocates no device memory. */
int rt_batch_autotune(const rt_shower *showers, int32_t n_showers, int precision, double k,
                      const rt_batch_options *candidates, int32_t n_candidates, void *workspace,
                      size_t workspace_bytes, int32_t reps, void *stream, float *ms,
                      int32_t *best);

/* Profiling aid: the next rt_batch_launch enqueues its kernels directly (not
 * through the graph) and records start_event before and stop_event after its
 * persistent deposit kernel, then forgets both (hipEvent_t as void*, created
 * and owned by the caller); NULL for both clears a pending request. */
int rt_batch_set_timing_events(rt_batch *batch, void *start_event, void *stop_event);

#ifdef __cplusplus
}
#endif

#endif /* RADTRACE_H */
