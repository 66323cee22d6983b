"""Benchmark of the track x antenna radio-emission loop on one MI355X.

Workload: 1e8 straight tracks (streamed in chunks of 2^22, all resident in
HBM before timing) x 4096 antennas on a 64 x 64 grid of 50 m spacing,
exponential refractivity, 4096 bins of 0.2 ns x 3 components, mixed
precision (float beta, qw and traces; the arithmetic is double precision);
one step is the Endpoint pass plus the ZHS pass over all tracks. The metric
is antenna-track pairs per second over both formalisms.

With --workload batched it measures instead 256 independent showers in one
persistent, graph-replayed launch per step (launch shape from the autotuner).

Prints one JSON line on stdout (progress goes to stderr). The roofline entry
is for the dominant deposit kernel, timed with HIP events recorded on its own
stream around every launch; the fp64 entry times the same deposits in FP64
mode on the first chunks (mixed vs FP64); the CPU baseline is the FP64 oracle
on a bounded sample of the same workload on this host's cores.
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "antenna-track pairs/sec (Endpoint, ZHS), % FP32 VALU peak; mixed vs FP64"

# Algorithmic floating-point operations of the definition per pair (add, sub,
# mul, div and sqrt count 1 each; comparisons, conversions and index
# arithmetic are not counted), split into the part every pair needs (the
# arrival-time chain, which decides whether the pair lands in the window) and
# the part only pairs that land need (amplitude and deposit). Per-track and
# per-antenna work is excluded. Every one of these operations executes in
# double precision in both modes: RT_MIXED differs in its inputs (float beta
# and qw), its outputs (float traces) and its refined-reciprocal divisions, not
# in the width of its arithmetic, so no FP32 work is counted.
OPS = {
    # per track end: timing 14; amplitude and deposit 21 (beta.d 5, the Doppler
    # numerator 2, (beta.d)/R^2 1, d q - beta 6, s k qw / (num dt) 1, a V 3,
    # three accumulating adds)
    "endpoint": {"timing_per_end": 14, "amp_per_end": 21},
    # per pair: timing of both ends 28; box 61 (midpoint geometry 27, box
    # height 4, edges 4, deposit values 14, twelve accumulating adds)
    "zhs": {"timing": 28, "box": 61},
}
# Spherical Earth: the path mean of n per track end by 8-point quadrature, 19
# FP64 operations per node (the node point 6, rho^2 5, the radius sum and its
# sqrt 2, the height quotient 2, the exponent quotient 1, exp 1, the weighted
# sum 2) and 2 to scale the sum: 154 per end on top of the timing chain.
SPHERICAL_TIMING_PER_END = 8 * 19 + 2
# MI355X published FP64 vector peak (an FMA counts as two operations); the
# published FP32 vector peak (157.3e12) needs packed FP32 instructions, which
# this build does not use, and no counted operation executes in FP32.
FP64_PEAK = 78.6e12
# VALU issue rate, a diagnostic: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane
# instructions per second (one wave64 instruction takes 4 cycles on a SIMD).
VALU_ISSUE_PEAK = 256 * 4 * 16 * 2.4e9

# Stored hardware-counter figures per deposit launch of 2^20 tracks on this
# workload, from counter runs of the kernels whose sources hash to
# COUNTERS_HASH: HBM bytes from FETCH_SIZE and WRITE_SIZE (KiB per dispatch,
# scaled by what the same counters read for a 1 GiB device copy: FETCH_SIZE
# reads half the copied bytes, WRITE_SIZE all of them), and SQ_INSTS_VALU
# (wave instructions per dispatch). They are reported, labelled as stored,
# only while the kernel sources and the launch shape are the measured ones;
# otherwise null.
COUNTER_SOURCES = ("rt_device.h", "rt_deposit.h", "forward.hip")
COUNTERS_HASH = "c3588e4b4cbd6da9"
COUNTERS_PROFILE = {"traffic": "profiles/deposit_grid4096_mixed_hbm_bytes.md",
                    "valu": "profiles/deposit_grid4096_mixed_counters.md"}
TRAFFIC_SCALE = {"fetch": 1048576.0 / 524304.4, "write": 1048576.0 / 1048576.0}
TRAFFIC_KIB = {"endpoint": {"fetch": 16921235.0, "write": 1572864.0},
               "zhs": {"fetch": 11875037.5, "write": 3145728.0}}
SQ_INSTS_VALU = {"endpoint": 7.512e9, "zhs": 7.841e9}
COUNTERS_PASS = 1 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cores():
    """Host threads this process may run on (all of them are used by the CPU
    oracle baselines)."""
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:
        return os.cpu_count() or 1


def in_window_fractions(rt, plan, dtr, n_sample):
    """Fraction of track ends (Endpoint) and of boxes (ZHS) that land in the
    window, from the library's own propagator on a sample of tracks."""
    import torch
    t, b = plan.propagate(dtr.slice(0, n_sample))
    torch.cuda.synchronize()
    ends_in = float((b >= 0).double().mean().item())
    # a box overlaps iff u_hi >= 0 and u_lo < B; with both ends outside on
    # opposite sides it still overlaps (rare); count via the arrival times
    tau = plan.det.t_start.view(1, -1)
    dt = plan.det.dt
    u = (t - tau) / dt
    lo = torch.minimum(u[0], u[1])
    hi = torch.maximum(u[0], u[1])
    box_in = float(((hi >= 0) & (lo < plan.det.n_bins)).double().mean().item())
    del t, b, u, lo, hi
    return ends_in, box_in


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, "paper_2309_03717_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_counters(formalism, tiling):
    """The stored counter figures of one deposit launch (HBM bytes, VALU
    wave instructions), or None when the kernel sources or the launch shape
    differ from those the counters were taken on."""
    if kernel_source_hash() != COUNTERS_HASH or tiling[4] != COUNTERS_PASS:
        return None
    k = TRAFFIC_KIB[formalism]
    return {"traffic": 1024.0 * (k["fetch"] * TRAFFIC_SCALE["fetch"]
                                 + k["write"] * TRAFFIC_SCALE["write"]),
            "valu_insts": SQ_INSTS_VALU[formalism]}


def ops_per_pair(formalism, ends_in, box_in, medium="exponential"):
    """Algorithmic operations per pair at the measured landing fractions (all
    of them executed in double precision)."""
    o = OPS[formalism]
    extra = 2 * SPHERICAL_TIMING_PER_END if medium == "spherical" else 0
    if formalism == "endpoint":
        return 2 * (o["timing_per_end"] + ends_in * o["amp_per_end"]) + extra
    return o["timing"] + box_in * o["box"] + extra


def cpu_baseline(workload, n_sample, medium=None):
    import oracle
    oracle._load()
    cores = host_cores()
    tr = workload.tracks(n_sample).to_mixed().widened()
    secs = {}
    for f in ("endpoint", "zhs"):
        t0 = time.perf_counter()
        oracle.traces(f, tr, workload.array, medium or workload.medium, k=1.0, n_threads=cores)
        secs[f] = time.perf_counter() - t0
        log(f"cpu baseline {f}: {secs[f]:.2f} s on {cores} threads")
    pairs = tr.n * workload.array.m
    return {"value": 2 * pairs / (secs["endpoint"] + secs["zhs"]), "unit": "pairs/s",
            "cores": cores, "kind": "oracle",
            "sample": f"first {tr.n} tracks of the {workload.n_tracks}-track workload x all "
                      f"{workload.array.m} antennas, Endpoint and ZHS each, FP64 oracle on the "
                      f"same float32-rounded beta/qw",
            "seconds": {k: round(v, 3) for k, v in secs.items()}}


def shower_ops(rt, dev_showers, n_sample=2048):
    """Algorithmic operations of a batch (all executed in double precision),
    from each shower's own in-window fractions (library propagator on its
    first tracks)."""
    ops = 0.0
    for det, md, f, dtr in dev_showers:
        if dtr.n == 0:
            continue
        plan = rt.Plan(det, md, f, "mixed")
        ends_in, box_in = in_window_fractions(rt, plan, dtr, min(dtr.n, n_sample))
        ops += ops_per_pair(f, ends_in, box_in) * dtr.n * det.m
    return ops


def bench_batched(args):
    """256 independent showers (track counts log-uniform in 1e4..1e6, 16..512
    antennas, 2048..8192 bins, both formalisms and media) in one persistent,
    graph-replayed launch per step, launch shape from the autotuner."""
    import torch
    from paper_2309_03717_amd import autotune
    from paper_2309_03717_amd import radtrace as rt
    from paper_2309_03717_amd import workloads as W

    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    showers = W.batched_showers(args.showers, max_tracks=args.tracks)
    dev = []
    for i, sh in enumerate(showers):
        tr = sh.tracks(mixed=True)
        dev.append((rt.DeviceDetector.from_array(sh.array), sh.medium, sh.formalism,
                    rt.DeviceTracks.from_tracks(tr)))
        if i % 64 == 63:
            log(f"generated {i + 1}/{len(showers)} showers ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    n_tracks = sum(d[3].n for d in dev)
    log(f"inputs resident: {len(dev)} showers, {n_tracks} tracks ({time.perf_counter() - t0:.1f} s)")

    if args.batch_options:
        bt, at, ipc = (int(x) for x in args.batch_options.split(","))
        opt = rt.BatchOptions(block_threads=bt, max_antennas_per_tile=at, items_per_cu=ipc)
        log(f"options given: {opt}")
    else:
        opt, timings, cached = autotune.tune_batch(dev, "mixed", k=rt.K_SI,
                                                   sample_tracks=args.tune_sample, log=log)
        log(f"autotuned options {opt} ({'cache' if cached else f'{len(timings)} candidates timed'})")
    batch = rt.Batch(dev, "mixed", k=rt.K_SI, options=opt)
    log(f"batch: {batch.info}, workspace {batch.workspace.numel() / 1e9:.2f} GB")

    def step():
        batch.zero_traces()
        batch.launch()

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(args.steps):
        step()
    stop.record()
    torch.cuda.synchronize()
    ms_step = start.elapsed_time(stop) / args.steps
    log(f"timed {args.steps} graph steps: {ms_step:.1f} ms/step")
    # deposit kernel alone: the same launches enqueued directly with events
    durs = []
    for _ in range(args.steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        batch.zero_traces()
        batch.set_timing_events(a, b)
        batch.launch()
        durs.append((a, b))
    torch.cuda.synchronize()
    kernel_ms = sum(a.elapsed_time(b) for a, b in durs) / len(durs)
    pairs = batch.pairs
    ops = shower_ops(rt, dev)
    achieved = ops / (kernel_ms / 1e3) / 1e12
    peak = FP64_PEAK / 1e12
    out = {"metric": METRIC, "value": pairs / (ms_step / 1e3), "unit": "pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"batched-{len(dev)}-showers" + (f"[max {args.tracks}]" if args.tracks else ""),
                      "n_showers": len(dev), "n_tracks": n_tracks, "pairs": pairs,
                      "precision": "mixed", "options": vars(opt), "launch": "hipGraph replay",
                      "items": batch.info["items"], "workgroups": batch.info["workgroups"]},
           "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                        "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                        "peak_kind": "published FP64 vector peak (all arithmetic is FP64)",
                        "kernel": "batch_deposit_kernel<mixed>", "kernel_ms_avg": round(kernel_ms, 3),
                        "flops_per_pair": round(ops / pairs, 3)}}
    if not args.no_cpu_baseline:
        import oracle
        oracle._load()
        cores = host_cores()
        k = min(args.cpu_sample or 48, len(showers))
        t1 = time.perf_counter()
        cpu_pairs = 0
        for sh, d in zip(showers[:k], dev[:k]):
            tr = sh.tracks(mixed=True).widened()
            oracle.traces(sh.formalism, tr, sh.array, sh.medium, k=1.0, n_threads=cores)
            cpu_pairs += tr.n * sh.array.m
        secs = time.perf_counter() - t1
        log(f"cpu baseline: {secs:.2f} s on {cores} threads")
        out["cpu_baseline"] = {"value": cpu_pairs / secs, "unit": "pairs/s", "cores": cores,
                               "kind": "oracle", "seconds": round(secs, 3),
                               "sample": f"the first {k} showers of the batch, all their tracks and "
                                         f"antennas ({cpu_pairs} pairs), FP64 oracle"}
    print(json.dumps(out), flush=True)


def bench_shower(args):
    """Shower-like, time-ordered tracks (workloads.shower_tracks) on the
    4096-antenna grid, mixed precision, both formalisms, against random
    tracks of the grid workload with the same count: the lanes of a wave now
    land in neighbouring bins, which stresses the LDS accumulation."""
    import torch
    from paper_2309_03717_amd import radtrace as rt
    from paper_2309_03717_amd import workloads as W

    torch.cuda.set_device(0)
    w = W.config(2)
    n = args.tracks or (1 << 24)
    chunk = w.chunk
    det = rt.DeviceDetector.from_array(w.array)
    plans = {f: rt.Plan(det, w.medium, f, "mixed", k=rt.K_SI) for f in ("endpoint", "zhs")}
    res = {}
    for kind in ("shower", "random"):
        chunks = []
        for lo in range(0, n, chunk):
            m = min(chunk, n - lo)
            t = (W.shower_tracks(W.SHOWER_SEED, m, start=lo) if kind == "shower"
                 else w.tracks(m, start=lo)).to_mixed()
            chunks.append(rt.DeviceTracks.from_tracks(t))
        traces = {f: plans[f].new_traces() for f in plans}
        for f in plans:   # warm-up
            plans[f].accumulate(chunks[0], traces[f])
        torch.cuda.synchronize()
        for f, plan in plans.items():
            evs = []
            for _ in range(args.steps):
                traces[f].zero_()
                for c in chunks:
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    rt.rt_plan_set_timing_events(plan.handle, a, b)
                    plan.accumulate(c, traces[f])
                    evs.append((a, b))
            torch.cuda.synchronize()
            ms = sum(a.elapsed_time(b) for a, b in evs) / args.steps
            res.setdefault(kind, {})[f] = {"deposit_ms": round(ms, 3),
                                           "pairs_per_s": n * w.array.m / (ms / 1e3)}
        log(f"{kind}: {res[kind]}")
        del chunks
    tot = {k: 2 * n * w.array.m / sum(v[f]["deposit_ms"] for f in v) * 1e3 for k, v in res.items()}
    out = {"metric": "antenna-track pairs/sec (Endpoint, ZHS), shower-like vs random tracks",
           "value": tot["shower"], "unit": "pairs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": 1, "ms_per_step": round(sum(v["deposit_ms"] for v in res["shower"].values()), 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"shower-{n}trk-grid4096-expn-mixed", "n_tracks": n,
                      "n_antennas": w.array.m},
           "random_tracks_value": tot["random"], "per_kind": res}
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Differentiable workload: 1e6 tracks x 64 antennas (8 x 8 grid, 75 m),
    4096 bins x 0.1 ns, exponential medium, mixed precision. One step is the
    forward traces plus the vector-Jacobian product of a trace loss, for the
    ZHS and the Endpoint formalism; the metric counts forward + adjoint
    pairs."""
    import torch
    from paper_2309_03717_amd import radtrace as rt
    from paper_2309_03717_amd import workloads as W

    torch.cuda.set_device(0)
    w = W.config(3)
    n = args.tracks or w.n_tracks
    tr = w.tracks(n, mixed=True)
    dtr = rt.DeviceTracks.from_tracks(tr)
    det = rt.DeviceDetector.from_array(w.array)
    plans = {f: rt.Plan(det, w.medium, f, "mixed") for f in ("zhs", "endpoint")}
    grad = torch.randn((w.array.m, w.array.n_bins, 3), device="cuda", dtype=torch.float32,
                       generator=torch.Generator(device="cuda").manual_seed(3))
    torch.cuda.synchronize()
    times = {}

    def step(record):
        for f, plan in plans.items():
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            ev[0].record()
            plan.traces(dtr)
            ev[1].record()
            plan.vjp(dtr, grad)
            ev[2].record()
            if record:
                times.setdefault(f, []).append(ev)

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        step(True)
    b.record()
    torch.cuda.synchronize()
    ms_step = a.elapsed_time(b) / args.steps
    pairs = n * w.array.m
    per = {}
    for f, evs in times.items():
        fw = sum(e[0].elapsed_time(e[1]) for e in evs) / len(evs)
        bw = sum(e[1].elapsed_time(e[2]) for e in evs) / len(evs)
        per[f] = {"forward_ms": round(fw, 3), "vjp_ms": round(bw, 3),
                  "forward_pairs_per_s": pairs / (fw / 1e3), "vjp_pairs_per_s": pairs / (bw / 1e3)}
    out = {"metric": "antenna-track pairs/sec, forward + adjoint (ZHS, Endpoint)",
           "value": 2 * 2 * pairs / (ms_step / 1e3), "unit": "pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": w.name if n == w.n_tracks else f"{w.name}[{n}]",
                      "n_tracks": n, "n_antennas": w.array.m, "n_bins": w.array.n_bins,
                      "precision": "mixed"},
           "per_formalism": per}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_adjoint(w, min(args.cpu_sample or (1 << 19), n), grad)
    print(json.dumps(out), flush=True)


def cpu_baseline_adjoint(workload, n_sample, grad):
    """The FP64 oracle's forward traces plus its vector-Jacobian product, both
    formalisms, on the first n_sample tracks (the same float-rounded inputs and
    upstream gradient), in the bench's unit: forward + adjoint pairs/s."""
    import oracle
    oracle._load()
    cores = host_cores()
    tr = workload.tracks(n_sample).to_mixed().widened()
    g = grad.double().cpu().numpy()
    secs = {}
    for f, vjp in (("zhs", oracle.zhs_vjp), ("endpoint", oracle.endpoint_vjp)):
        t0 = time.perf_counter()
        oracle.traces(f, tr, workload.array, workload.medium, n_threads=cores)
        vjp(tr, workload.array, workload.medium, g, n_threads=cores)
        secs[f] = time.perf_counter() - t0
        log(f"cpu baseline {f} forward + vjp: {secs[f]:.2f} s on {cores} threads")
    pairs = tr.n * workload.array.m
    return {"value": 2 * 2 * pairs / (secs["zhs"] + secs["endpoint"]), "unit": "pairs/s",
            "cores": cores, "kind": "oracle",
            "sample": f"first {tr.n} tracks x all {workload.array.m} antennas, forward traces + "
                      f"VJP of both formalisms, FP64 oracle on the same float32-rounded inputs",
            "seconds": {k: round(v, 3) for k, v in secs.items()}}


def bench_oracle(args):
    """The FP64 oracle alone on the host (no GPU): the grid workload's first
    args.cpu_sample tracks x all 4096 antennas, both formalisms, at 1, 2, 4,
    8, 16 and all host threads, the latter also with the antenna
    bunch sizes {1, 4, 16, 64} (the paper's unit of work per thread) beside
    the default ceil(M / threads); then the whole 16-antenna, star and
    differentiable workloads at all host threads. Reported for context: the
    oracle is the reference, not a tuned CPU code."""
    import oracle
    from paper_2309_03717_amd import workloads as W
    oracle._load()
    cores = host_cores()
    w = W.config(2)
    tr = w.tracks(args.cpu_sample or (1 << 14)).to_mixed().widened()
    pairs = tr.n * w.array.m
    runs = []
    sweep = sorted({1, 2, 4, 8, 16} & set(range(1, cores + 1)) | {cores})
    plan = [(t, 0) for t in sweep] + [(cores, b) for b in (1, 4, 16, 64)]
    for threads, bunch in plan:
        secs = {}
        for f in ("endpoint", "zhs"):
            t0 = time.perf_counter()
            oracle.traces(f, tr, w.array, w.medium, k=1.0, n_threads=threads, bunch=bunch)
            secs[f] = time.perf_counter() - t0
        rate = 2 * pairs / (secs["endpoint"] + secs["zhs"])
        runs.append({"threads": threads, "bunch": bunch or -(-w.array.m // threads),
                     "pairs_per_s": rate, "seconds": {k: round(v, 3) for k, v in secs.items()}})
        log(f"oracle {threads} threads, bunch {runs[-1]['bunch']}: {rate / 1e6:.1f} M pairs/s")
    # the whole small workloads at every host thread (default bunches)
    whole = {}
    for k in (0, 1, 3):
        wk = W.config(k)
        tk = wk.tracks(mixed=True).widened()
        secs = {}
        for f in ("endpoint", "zhs"):
            t0 = time.perf_counter()
            oracle.traces(f, tk, wk.array, wk.medium, k=1.0, n_threads=cores)
            secs[f] = time.perf_counter() - t0
        whole[wk.name] = {"pairs": tk.n * wk.array.m,
                          "pairs_per_s": 2 * tk.n * wk.array.m / (secs["endpoint"] + secs["zhs"]),
                          "seconds": {f: round(v, 3) for f, v in secs.items()}}
        log(f"oracle {wk.name}: {whole[wk.name]['pairs_per_s'] / 1e6:.1f} M pairs/s")
    best = max(r["pairs_per_s"] for r in runs)
    one = next(r for r in runs if r["threads"] == 1 and r["bunch"] == w.array.m)
    allt = next(r for r in runs if r["threads"] == cores and r["bunch"] == -(-w.array.m // cores))
    print(json.dumps({"metric": "oracle antenna-track pairs/sec (Endpoint, ZHS), host CPU",
                      "value": best, "unit": "pairs/s", "n_gpus": 0, "steps": 1, "warmup": 0,
                      "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": f"{w.name}[{tr.n}]", "n_antennas": w.array.m,
                                 "host_threads": cores},
                      "speedup_all_threads": round(allt["pairs_per_s"] / one["pairs_per_s"], 2),
                      "runs": runs, "whole_workloads": whole}), flush=True)


def bench_copy(args):
    """Calibration for hardware byte counters: a plain device-to-device copy
    of a known size (args.copy_mib MiB read and written per launch)."""
    import torch
    torch.cuda.set_device(0)
    n = args.copy_mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(args.warmup):
        dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(args.steps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / args.steps
    print(json.dumps({"metric": "device copy bandwidth (read + write)", "value": 2 * n / (ms / 1e3),
                      "unit": "B/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
                      "ms_per_step": round(ms, 4), "higher_is_better": True,
                      "bytes_read_per_launch": n, "bytes_written_per_launch": n,
                      "config": {"workload": f"copy-{args.copy_mib}MiB"}}), flush=True)


def bench_stream(args):
    """The grid workload with the tracks in pinned host memory, as a CPU
    cascade hands them over: every 2^22-track chunk is copied to the device
    (streaming.HostTrackStream: copy stream, two device buffers) while the
    previous chunk deposits, and both formalisms run on each copied chunk.
    The value is end to end: every host-to-device copy is inside the timed
    region. The same run times the device-resident deposits for the ratio, and
    the stream with the track filter on every chunk (threshold 0: every
    synthetic track is kept, so the same pairs; the difference is the filter
    and the one-chunk lag of the deposits behind it)."""
    import torch
    from paper_2309_03717_amd import radtrace as rt
    from paper_2309_03717_amd import streaming as S
    from paper_2309_03717_amd import workloads as W

    torch.cuda.set_device(0)
    w = W.config(2)
    n_total = args.tracks or w.n_tracks
    chunk = w.chunk
    t0 = time.perf_counter()
    host = []
    for lo in range(0, n_total, chunk):
        host.append(S.pinned_chunk(w.tracks(min(chunk, n_total - lo), start=lo, mixed=True)))
        if len(host) % 6 == 1:
            log(f"pinned {lo + host[-1]['x0'].numel()}/{n_total} tracks "
                f"({time.perf_counter() - t0:.1f} s)")
    det = rt.DeviceDetector.from_array(w.array)
    plans = [rt.Plan(det, w.medium, f, "mixed", k=rt.K_SI) for f in ("endpoint", "zhs")]
    traces = [p.new_traces() for p in plans]
    for p in plans:
        p.workspace(chunk)
    st = S.HostTrackStream(plans, chunk)
    host_bytes = sum(t.numel() * t.element_size() for c in host for t in c.values())

    # raw host-to-device rate of one chunk's fields, for context
    dev = {f: torch.empty_like(host[0][f], device="cuda") for f in W.TRACK_FIELDS}
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for f in W.TRACK_FIELDS:
        dev[f].copy_(host[0][f], non_blocking=True)
    b.record()
    torch.cuda.synchronize()
    chunk_bytes = sum(t.numel() * t.element_size() for t in host[0].values())
    h2d_gbps = chunk_bytes / (a.elapsed_time(b) / 1e3) / 1e9
    del dev

    def streamed():
        for t in traces:
            t.zero_()
        for c in host:
            st.push(c, traces)

    for i in range(args.warmup):
        streamed()
        st.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    start.record()
    for _ in range(args.steps):
        streamed()
    stop.record()
    st.synchronize()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - wall0) / args.steps
    ms_step = start.elapsed_time(stop) / args.steps
    log(f"streamed: {ms_step:.1f} ms/step")

    # the same deposits from device-resident chunks (one step), for the ratio
    resident = []
    for c in host:
        resident.append(rt.DeviceTracks(**{f: c[f].to("cuda") for f in W.TRACK_FIELDS}))
    torch.cuda.synchronize()
    start.record()
    for t in traces:
        t.zero_()
    for dt in resident:
        for p, t in zip(plans, traces):
            p.accumulate(dt, t)
    stop.record()
    torch.cuda.synchronize()
    ms_res = start.elapsed_time(stop)
    del resident

    stf = S.HostTrackStream(plans, chunk, qw_min=0.0)

    def filtered():
        for t in traces:
            t.zero_()
        for c in host:
            stf.push(c, traces)
        stf.flush()

    filtered()
    stf.synchronize()
    kept0 = stf.kept
    torch.cuda.synchronize()
    start.record()
    for _ in range(args.steps):
        filtered()
    stop.record()
    stf.synchronize()
    torch.cuda.synchronize()
    ms_filt = start.elapsed_time(stop) / args.steps
    if stf.kept - kept0 != args.steps * n_total:
        raise RuntimeError(f"the filter kept {stf.kept - kept0} of {args.steps * n_total} tracks")
    log(f"streamed with the track filter: {ms_filt:.1f} ms/step")
    pairs = 2 * n_total * w.array.m
    out = {"metric": "antenna-track pairs/sec (Endpoint + ZHS), tracks streamed from host memory",
           "value": pairs / (ms_step / 1e3), "unit": "pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": f"grid4096-{n_total}trk-expn-mixed-host-streamed",
                      "n_tracks": n_total, "n_antennas": w.array.m, "chunk": chunk,
                      "host_bytes_per_step": host_bytes},
           "wall_ms_per_step": round(wall * 1e3, 3),
           "h2d_GBps_one_chunk": round(h2d_gbps, 2),
           "resident_value": pairs / (ms_res / 1e3),
           "streamed_over_resident": round(ms_res / ms_step, 4),
           "filtered_value": pairs / (ms_filt / 1e3),
           "filtered_over_streamed": round(ms_step / ms_filt, 4)}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--tracks", type=int, default=None,
                    help="override the track count (smaller runs for profiling)")
    ap.add_argument("--formalisms", default="endpoint,zhs")
    ap.add_argument("--cpu-sample", type=int, default=None,
                    help="tracks (showers for batched) the CPU oracle baseline runs on; "
                         "defaults sized for about 10-15 s of oracle work on 16 threads: "
                         "grid 2^19 tracks (2^18 in the tabulated and spherical media), "
                         "adjoint 2^19 tracks, batched 48 showers, oracle sweep 2^14 tracks")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tiling", default=None, help="at,splits,block,seg,pass override")
    ap.add_argument("--workload", default="grid4096",
                    choices=["grid4096", "batched", "adjoint", "shower", "stream", "copy",
                             "oracle"],
                    help="grid4096: 1e8 tracks x 4096 antennas (default); batched: 256 showers; "
                         "adjoint: forward + VJP on 1e6 tracks x 64 antennas; "
                         "shower: shower-like vs random tracks on the grid; "
                         "stream: the grid workload copied from pinned host memory (plain, "
                         "device-resident and filtered legs); "
                         "copy: byte-counter calibration; oracle: the CPU oracle alone "
                         "at 1 and all host threads and several antenna bunch sizes")
    ap.add_argument("--copy-mib", type=int, default=1024, help="copy: MiB per launch")
    ap.add_argument("--showers", type=int, default=256, help="batched: number of showers")
    ap.add_argument("--medium", default="exponential",
                    choices=["exponential", "layered", "spherical"],
                    help="grid4096: the exponential profile (default), the tabulated "
                         "two-layer atmosphere, or the exponential profile over a spherical "
                         "Earth (path mean by quadrature per pair)")
    ap.add_argument("--fp64-chunks", type=int, default=2,
                    help="grid4096: chunks of the workload also timed in FP64 mode (0: none)")
    ap.add_argument("--tune-sample", type=int, default=1 << 16,
                    help="batched: tracks per shower the autotuner times candidates on")
    ap.add_argument("--batch-options", default=None,
                    help="batched: block_threads,max_antennas_per_tile,items_per_cu "
                         "instead of the autotuner's choice")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(antenna sharding across GPUs is described in the design notes)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
        return
    if args.workload == "copy":
        bench_copy(args)
        return
    if args.workload == "oracle":
        bench_oracle(args)
        return
    if args.workload == "adjoint":
        bench_adjoint(args)
        return
    if args.workload == "stream":
        bench_stream(args)
        return
    if args.workload == "shower":
        bench_shower(args)
        return

    import torch
    from paper_2309_03717_amd import radtrace as rt
    from paper_2309_03717_amd import workloads as W

    torch.cuda.set_device(0)
    w = W.config(2)
    n_total = args.tracks or w.n_tracks
    chunk = w.chunk
    formalisms = args.formalisms.split(",")

    # ---- inputs resident in HBM before timing
    t0 = time.perf_counter()
    fields = {f: [] for f in W.TRACK_FIELDS}
    for lo in range(0, n_total, chunk):
        part = w.tracks(min(chunk, n_total - lo), start=lo, mixed=True)
        for f in W.TRACK_FIELDS:
            fields[f].append(torch.from_numpy(getattr(part, f)).to("cuda", non_blocking=False))
        if (lo // chunk) % 6 == 0:
            log(f"generated {lo + part.n}/{n_total} tracks ({time.perf_counter() - t0:.1f} s)")
    chunks = [rt.DeviceTracks(**{f: fields[f][c] for f in W.TRACK_FIELDS})
              for c in range(len(fields["x0"]))]
    det = rt.DeviceDetector.from_array(w.array)
    medium = {"exponential": w.medium, "layered": W.layered_air(),
              "spherical": W.SPHERICAL_AIR}[args.medium]
    plans = {f: rt.Plan(det, medium, f, "mixed", k=rt.K_SI) for f in formalisms}
    if args.tiling:
        for p in plans.values():
            p.set_tiling(*[int(x) for x in args.tiling.split(",")])
    traces = {f: plans[f].new_traces() for f in formalisms}
    for f in formalisms:
        plans[f].workspace(chunk)
    torch.cuda.synchronize()
    log(f"inputs resident: {n_total} tracks in {len(chunks)} chunks, "
        f"{sum(c.n for c in chunks) * 80 / 1e9:.2f} GB ({time.perf_counter() - t0:.1f} s)")

    kernel_events = {f: [] for f in formalisms}

    def step(record):
        for f in formalisms:
            traces[f].zero_()
            for c in chunks:
                if record:
                    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    rt.rt_plan_set_timing_events(plans[f].handle, s, e)
                    kernel_events[f].append((s, e))
                plans[f].accumulate(c, traces[f])

    for i in range(args.warmup):
        step(False)
        torch.cuda.synchronize()
        log(f"warmup step {i + 1}/{args.warmup} done")
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    start.record()
    for i in range(args.steps):
        step(True)
        if i == 0:
            pass
    stop.record()
    torch.cuda.synchronize()
    ms_total = start.elapsed_time(stop)
    ms_step = ms_total / args.steps
    log(f"timed {args.steps} steps: {ms_step:.1f} ms/step")

    pairs_per_formalism = n_total * w.array.m
    value = len(formalisms) * pairs_per_formalism / (ms_step / 1e3)

    # ---- per-kernel durations and the roofline of the dominant kernel
    ends_in, box_in = in_window_fractions(rt, plans[formalisms[0]], chunks[0],
                                          min(chunks[0].n, 1 << 13))
    per = {}
    for f in formalisms:
        # one event pair spans the deposit launches of all passes of a call
        passes = -(-chunk // plans[f].tiling(chunk)[4])
        durs = [s.elapsed_time(e) / passes for s, e in kernel_events[f]]
        n_launch = len(durs)
        avg_ms = sum(durs) / n_launch
        ops = ops_per_pair(f, ends_in, box_in, args.medium)
        pairs_per_launch = pairs_per_formalism * args.steps / (n_launch * passes)
        achieved = ops * pairs_per_launch / (avg_ms / 1e3)
        per[f] = {"kernel_ms_avg": avg_ms, "launches": n_launch * passes,
                  "kernel_ms_total_per_step": sum(durs) * passes / args.steps,
                  "pairs_per_s_kernel": pairs_per_launch / (avg_ms / 1e3),
                  "pairs_per_launch": pairs_per_launch,
                  "flops_per_pair": round(ops, 3),
                  "achieved_tflops": achieved / 1e12,
                  "fp64_peak_frac": achieved / FP64_PEAK,
                  "fp32_valu_peak_frac": 0.0}
    dom = max(formalisms, key=lambda f: per[f]["kernel_ms_total_per_step"])
    achieved = per[dom]["achieved_tflops"]
    peak = FP64_PEAK / 1e12
    stored = (stored_counters(dom, plans[dom].tiling(chunk))
              if n_total >= chunk and args.medium == "exponential" else None)
    kms = per[dom]["kernel_ms_avg"]
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(peak, 3),
                "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                "peak_kind": "published FP64 vector peak: every counted operation executes "
                             "in FP64 (none in FP32, so the FP32 VALU fraction is 0)",
                "traffic": None if stored is None else round(stored["traffic"]),
                "traffic_source": None if stored is None else
                f"stored counter runs ({COUNTERS_PROFILE['traffic']}), kernel sources "
                f"{COUNTERS_HASH}: FETCH_SIZE + WRITE_SIZE, copy-calibrated, bytes per launch",
                "traffic_rate_GBps": None if stored is None else
                round(stored["traffic"] / (kms / 1e3) / 1e9, 1),
                "kernel": f"deposit_kernel<{dom},mixed,{medium.kind}>",
                "kernel_ms_avg": round(kms, 3),
                "pairs_per_launch": per[dom]["pairs_per_launch"],
                "flops_per_pair": per[dom]["flops_per_pair"],
                "in_window": {"endpoint_ends": round(ends_in, 4), "zhs_boxes": round(box_in, 4)},
                "valu_issue_diagnostic": None if stored is None else {
                    "lane_instructions_per_s": stored["valu_insts"] * 64 / (kms / 1e3),
                    "peak": VALU_ISSUE_PEAK, "unit": "lane-instructions/s",
                    "frac": round(stored["valu_insts"] * 64 / (kms / 1e3) / VALU_ISSUE_PEAK, 4),
                    "source": f"stored SQ_INSTS_VALU ({COUNTERS_PROFILE['valu']})"}}

    out = {"metric": METRIC, "value": value, "unit": "pairs/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "io": "tracks: FP64 points and times, FP32 beta and qw; traces FP32",
           "data": "synthetic",
           "config": {"workload": (w.name if n_total == w.n_tracks else f"{w.name}[{n_total}]")
                      + ("" if args.medium == "exponential" else "+" + args.medium),
                      "n_tracks": n_total, "n_antennas": w.array.m, "n_bins": w.array.n_bins,
                      "dt_ns": w.array.dt * 1e9,
                      "medium": {"exponential": "exponential", "layered": "tabulated (layered)",
                                 "spherical": "exponential over a spherical Earth"}[args.medium],
                      "precision": "mixed", "formalisms": formalisms, "chunk": chunk,
                      "tiling": {f: plans[f].tiling(chunk) for f in formalisms}},
           "per_formalism": {f: {"pairs_per_s": pairs_per_formalism / (per[f]["kernel_ms_total_per_step"] / 1e3),
                                 **{k: (round(v, 4) if isinstance(v, float) else v)
                                    for k, v in per[f].items()}} for f in formalisms},
           "roofline": roofline}
    out["track_filter"] = filter_leg(rt, chunks[0])
    if args.fp64_chunks > 0:
        out["fp64"] = fp64_leg(rt, det, medium, chunks[:args.fp64_chunks], formalisms,
                               w.array.m, {f: out["per_formalism"][f]["pairs_per_s"]
                                           for f in formalisms})
    if not args.no_cpu_baseline:
        # the spherical and tabulated media's oracle takes 2.5-3x longer per pair
        default = 1 << 19 if args.medium == "exponential" else 1 << 18
        out["cpu_baseline"] = cpu_baseline(w, min(args.cpu_sample or default, n_total), medium)
    print(json.dumps(out), flush=True)


def filter_leg(rt, chunk, reps=5):
    """The track filter (rt_filter_tracks, qw_min = 0) on one chunk, timed
    with HIP events outside the timed steps: its cost beside the deposits and
    its HBM rate (each track read twice, kept ones written once)."""
    import torch
    from paper_2309_03717_amd import workloads as W
    prec = rt.RT_MIXED
    src = chunk.struct(prec)
    out = rt.DeviceTracks(**{f: torch.empty_like(getattr(chunk, f)) for f in W.TRACK_FIELDS})
    dst = out.struct(prec)
    n_kept = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = torch.empty(max(rt.rt_filter_workspace_bytes(chunk.n), 256), dtype=torch.uint8,
                     device="cuda")
    rt.rt_filter_tracks(src, prec, 0.0, dst, n_kept, ws)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        rt.rt_filter_tracks(src, prec, 0.0, dst, n_kept, ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    kept = int(n_kept.item())
    per_track = sum(getattr(chunk, f).element_size() for f in W.TRACK_FIELDS)
    moved = (2 * chunk.n + kept) * per_track
    return {"tracks": chunk.n, "kept": kept, "ms": round(ms, 4),
            "GBps": round(moved / (ms / 1e3) / 1e9, 1)}


def fp64_leg(rt, det, medium, chunks, formalisms, m, mixed_rate):
    """The same deposits in FP64 mode (every operation in double, double
    traces) on the first chunks of the workload, with the float32-rounded beta
    and qw of the mixed inputs widened: kernel pairs/s per formalism (HIP events
    around the deposits, one warm-up call first) and the mixed/FP64 ratio."""
    import torch
    from paper_2309_03717_amd import workloads as W
    wide = [rt.DeviceTracks(**{f: (getattr(c, f).double() if f in W.BETA_W_FIELDS
                                   else getattr(c, f)) for f in W.TRACK_FIELDS})
            for c in chunks]
    res = {"tracks": sum(c.n for c in wide), "note": "first chunks of the workload, "
           "kernel time of the deposits, same inputs as the mixed run widened to double"}
    for f in formalisms:
        plan = rt.Plan(det, medium, f, "fp64", k=rt.K_SI)
        tr = plan.new_traces()
        plan.accumulate(wide[0], tr)
        torch.cuda.synchronize()
        ev = []
        for c in wide:
            s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            rt.rt_plan_set_timing_events(plan.handle, s, e)
            plan.accumulate(c, tr)
            ev.append((s, e))
        torch.cuda.synchronize()
        ms = sum(s.elapsed_time(e) for s, e in ev)
        rate = res["tracks"] * m / (ms / 1e3)
        res[f] = {"pairs_per_s": rate, "kernel_ms": round(ms, 3),
                  "mixed_over_fp64": round(mixed_rate[f] / rate, 3),
                  "tiling": plan.tiling(wide[0].n)}
        log(f"fp64 {f}: {rate / 1e9:.1f} G pairs/s ({ms:.1f} ms for {res['tracks']} tracks)")
        del plan, tr
    del wide
    torch.cuda.empty_cache()
    return res


if __name__ == "__main__":
    main()
