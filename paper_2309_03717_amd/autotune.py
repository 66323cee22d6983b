"""Launch-shape autotuner for batches and single plans.

The library's autotuners (rt_plan_autotune, rt_batch_autotune) time the
candidate shapes on the device with HIP events around real launches (same
inputs, direct launches, warm-up first); this module chooses the candidates,
re-times the best families on the whole workload when a sample was timed, and
keeps the fastest in a JSON cache keyed by the device (architecture and
compute-unit count) and a signature of the workload's shapes, so that later
runs of the same shapes reuse it without timing anything. The cache file is
written atomically (temporary file + rename).
"""
from __future__ import annotations

import hashlib
import itertools
import json
import os
import tempfile
import time
from typing import Callable, Dict, Iterable, List, Optional, Sequence, Tuple

import torch

DEFAULT_CACHE = os.environ.get(
    "RADTRACE_TUNE_CACHE",
    os.path.join(os.path.expanduser("~"), ".cache", "paper_2309_03717_amd", "tuning.json"))


# ------------------------------------------------------------------ cache
class TuningCache:
    """A JSON object {key: {"best": ..., "timings": [...], "when": ...}}."""

    def __init__(self, path: Optional[str] = None):
        self.path = path or DEFAULT_CACHE
        self.data: Dict[str, dict] = {}
        if os.path.exists(self.path):
            try:
                with open(self.path) as f:
                    self.data = json.load(f)
            except (OSError, ValueError):
                self.data = {}   # unreadable cache: start afresh

    def get(self, key: str):
        e = self.data.get(key)
        return None if e is None else e["best"]

    def put(self, key: str, best, timings) -> None:
        self.data[key] = {"best": best, "timings": timings, "when": time.time()}
        d = os.path.dirname(os.path.abspath(self.path))
        os.makedirs(d, exist_ok=True)
        fd, tmp = tempfile.mkstemp(dir=d, prefix=".tuning", suffix=".json")
        with os.fdopen(fd, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def device_key() -> str:
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(p, "gcnArchName", p.name)
    return f"{arch}/{p.multi_processor_count}cu"


def signature(parts: Iterable) -> str:
    return hashlib.sha1(json.dumps(list(parts)).encode()).hexdigest()[:16]


def tune(key: str, candidates: Sequence, measure: Optional[Callable[[object], float]] = None,
         cache: Optional[TuningCache] = None, log: Optional[Callable[[str], None]] = None,
         final_measure: Optional[Callable[[object], float]] = None, finalists: int = 3,
         family: Callable[[object], object] = lambda c: json.dumps(c),
         measure_all: Optional[Callable[[Sequence], Sequence]] = None):
    """The candidate with the smallest measure(candidate) (seconds), cached
    under key. A candidate whose measurement raises (for example a shape the
    library rejects) is skipped. measure_all(candidates) may replace measure:
    one call returning the seconds of every candidate (None for a skipped
    one). With final_measure (say, the whole workload where measure times a
    sample), the fastest candidate of each of the `finalists` fastest
    families (family(candidate): candidates that differ only in a minor knob
    share one) is timed again by it and the fastest of those wins. Returns
    (best, timings, from_cache)."""
    cache = cache if cache is not None else TuningCache()
    hit = cache.get(key)
    if hit is not None:
        return hit, None, True
    timings: List[Tuple[object, float]] = []
    if measure_all is not None:
        for c, t in zip(candidates, measure_all(list(candidates))):
            if t is None:
                if log:
                    log(f"  {c}: skipped (refused, or beyond the workspace)")
                continue
            timings.append((c, t))
            if log:
                log(f"  {c}: {t * 1e3:.3f} ms")
    for c in (candidates if measure_all is None else ()):
        try:
            t = measure(c)
        except (RuntimeError, ValueError) as e:
            if log:
                log(f"  {c}: rejected ({e})")
            continue
        timings.append((c, t))
        if log:
            log(f"  {c}: {t * 1e3:.3f} ms")
    if not timings:
        raise RuntimeError("no candidate launch shape could be measured")
    best = min(timings, key=lambda ct: ct[1])[0]
    if final_measure is not None and finalists > 1 and len(timings) > 1:
        final, seen = [], set()
        for c, _ in sorted(timings, key=lambda ct: ct[1]):
            fam = family(c)
            if fam in seen:
                continue
            seen.add(fam)
            if len(seen) > finalists:
                break
            t = final_measure(c)
            final.append((c, t))
            if log:
                log(f"  final {c}: {t * 1e3:.3f} ms")
        best = min(final, key=lambda ct: ct[1])[0]
    cache.put(key, best, [[c, t] for c, t in timings])
    return best, timings, False


# ------------------------------------------------------------------ batches
BATCH_BLOCKS = (256, 512)
BATCH_AT = (1, 2, 3)
BATCH_ITEMS = (2, 4, 8)


def batch_key(showers, precision: str) -> str:
    shapes = [(f, md.kind, det.m, det.n_bins, tr.n) for det, md, f, tr in showers]
    return f"batch/{device_key()}/{precision}/{signature(shapes)}"


def tune_batch(showers, precision: str = "mixed", k: float = 1.0,
               cache_path: Optional[str] = None, candidates=None, sample_tracks: Optional[int] = None,
               reps: int = 2, log=None):
    """BatchOptions for the showers (list of (DeviceDetector, medium,
    formalism, DeviceTracks)). Candidates are (block_threads, max antennas
    per tile, items per CU) triples (1024 threads with one-antenna tiles
    among them); sample_tracks times each candidate on
    the first tracks of every shower only. The result launches through a HIP
    graph."""
    from . import radtrace as rt
    key = batch_key(showers, precision)
    cands = candidates or ([list(c) for c in itertools.product(BATCH_BLOCKS, BATCH_AT, BATCH_ITEMS)]
                           + [[1024, 1, i] for i in BATCH_ITEMS])
    sample = showers
    if sample_tracks is not None:
        sample = [(d, m, f, t.slice(0, min(t.n, sample_tracks))) for d, m, f, t in showers]

    def options(c):
        return rt.BatchOptions(block_threads=c[0], max_antennas_per_tile=c[1], items_per_cu=c[2])

    def timed(showers_, cs, reps_):   # one rt_batch_autotune call over the candidates
        return rt.rt_batch_autotune(showers_, precision, k, [options(c) for c in cs], reps_)

    # shapes within a percent on the sample can order differently on the
    # whole batch: the best of the three best (workgroup size, tile width)
    # families are timed again on all tracks
    def final(c):
        t = timed(showers, [c], 1)[0]
        if t is None:
            raise RuntimeError(f"{c} could not be timed on the whole batch")
        return t

    best, timings, cached = tune(key, cands, None, TuningCache(cache_path), log,
                                 final_measure=final if sample is not showers else None,
                                 family=lambda c: (c[0], c[1]),
                                 measure_all=lambda cs: timed(sample, cs, reps))
    return rt.BatchOptions(block_threads=best[0], max_antennas_per_tile=best[1],
                           items_per_cu=best[2]), timings, cached


# ------------------------------------------------------------------ single plans
PLAN_BLOCKS = (256, 512, 1024)
PLAN_PASSES = (1 << 19, 1 << 20, 1 << 21)
# track-split multiples of the automatic count tried at the automatic block
# size and pass length: time-ordered track streams (a shower's) keep the
# workgroups of an XCD sharing their records in L2 better with shorter splits
PLAN_SPLIT_FACTORS = (2,)


def plan_candidates(auto_tiling):
    """Default candidates of tune_plan: the automatic tile at every block size
    and pass length, then the automatic block size and pass length with twice
    the automatic track splits. auto_tiling is the plan's automatic
    (antennas_per_block, track_splits, block_threads, bins_per_segment,
    tracks_per_pass) for the tuned call."""
    cands = [[0, 0, b, 0, p] for b in PLAN_BLOCKS for p in PLAN_PASSES]
    splits, block, pass_len = auto_tiling[1], auto_tiling[2], auto_tiling[4]
    for f in PLAN_SPLIT_FACTORS:
        c = [0, splits * f, block, 0, pass_len]
        if c not in cands:
            cands.append(c)
    return cands


def plan_key(plan, n_tracks: int) -> str:
    shapes = [plan.formalism, plan.precision, plan.medium.kind, plan.det.m, plan.det.n_bins,
              int(n_tracks).bit_length()]
    return f"plan/{device_key()}/{signature(shapes)}"


def tune_plan(plan, tracks, cache_path: Optional[str] = None, candidates=None, reps: int = 2,
              log=None):
    """Sets and returns the fastest (antennas_per_block, track_splits,
    block_threads, bins_per_segment, tracks_per_pass) tiling of a Plan for
    calls like plan.accumulate(tracks); candidates default to plan_candidates
    of the plan's automatic tiling."""
    from . import radtrace as rt
    key = plan_key(plan, tracks.n)
    if not candidates:
        plan.set_tiling()   # the automatic tiling, whatever was set before
        candidates = plan_candidates(list(plan.tiling(tracks.n)))
    cands = candidates
    best, timings, cached = tune(key, cands, None, TuningCache(cache_path), log,
                                 measure_all=lambda cs: rt.rt_plan_autotune(plan, tracks, cs, reps))
    plan.set_tiling(*best)
    return list(best), timings, cached
