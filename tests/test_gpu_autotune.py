"""The plan autotuner (rt_plan_autotune through autotune.tune_plan): every
candidate timed on the device, the fastest set on the plan and cached, and
the tuned plan's traces unchanged (the tiling moves summation order only)."""
import numpy as np
import pytest

from paper_2309_03717_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_03717_amd import radtrace
    return radtrace


def test_plan_autotune_times_sets_and_caches(rt, tmp_path):
    import torch
    from paper_2309_03717_amd import autotune
    w = W.config(1)
    det = rt.DeviceDetector.from_array(w.array)
    plan = rt.Plan(det, w.medium, "zhs", "mixed")
    dtr = rt.DeviceTracks.from_tracks(w.tracks(50_000, mixed=True))
    ref = plan.traces(dtr).cpu().numpy()
    cands = [[0, 0, 256, 0, 0], [0, 0, 1024, 0, 0], [0, 3, 512, 0, 1 << 14],
             [9, 0, 0, 0, 0]]   # the last one is refused (at most 8 antennas per tile)
    path = str(tmp_path / "tune.json")
    best, timings, cached = autotune.tune_plan(plan, dtr, cache_path=path, candidates=cands)
    assert not cached and best in cands[:3] and len(timings) == 3
    assert list(plan.tiling(dtr.n))[2] == (best[2] or 1024)
    got = plan.traces(dtr).cpu().numpy()
    np.testing.assert_array_equal(got, ref)   # fixed-point ZHS: the same bits for any tiling
    best2, _, cached2 = autotune.tune_plan(plan, dtr, cache_path=path, candidates=cands)
    assert cached2 and best2 == best
    torch.cuda.synchronize()


def test_plan_autotune_skips_candidates_beyond_the_workspace(rt):
    """The C entry point with a workspace sized for one candidate only: the
    others are skipped (time -1 -> None) and the fitting one is chosen."""
    import ctypes as C
    import torch
    w = W.config(0)
    det = rt.DeviceDetector.from_array(w.array)
    plan = rt.Plan(det, w.medium, "endpoint", "fp64")
    dtr = rt.DeviceTracks.from_tracks(w.tracks(20_000))
    small = rt.rt_tiling(0, 1, 256, 0, 0)    # one split: the smallest workspace
    big = rt.rt_tiling(0, 64, 256, 0, 0)     # 64 splits of partials
    rt.rt_plan_set_tiling(plan.handle, *small.as_tuple())
    need = rt.rt_plan_workspace_bytes(plan.handle, dtr.n)
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    scratch = plan.new_traces()
    cands = (rt.rt_tiling * 2)(big, small)
    ms = (C.c_float * 2)()
    best = C.c_int32(-1)
    st = rt._lib.rt_plan_autotune(plan.handle, C.byref(dtr.struct(rt.RT_FP64)), scratch.data_ptr(),
                                  ws.data_ptr(), need, cands, 2, 2,
                                  torch.cuda.current_stream().cuda_stream, ms, C.byref(best))
    assert st == rt.RT_OK, rt.rt_last_error()
    assert ms[0] == -1.0 and ms[1] > 0 and best.value == 1
    assert plan.tiling(dtr.n)[1] == 1


def test_plan_autotune_default_candidates(rt, tmp_path):
    """tune_plan without candidates: the automatic tile at every block size and
    pass length plus twice the automatic split count, all timed; the winner is
    set on the plan and leaves the fixed-point ZHS traces bit for bit."""
    import torch
    from paper_2309_03717_amd import autotune
    w = W.config(1)
    det = rt.DeviceDetector.from_array(w.array)
    plan = rt.Plan(det, w.medium, "zhs", "mixed")
    dtr = rt.DeviceTracks.from_tracks(w.tracks(50_000, mixed=True))
    plan.set_tiling(0, 5, 256, 0, 0)   # replaced by the automatic tiling first
    ref = plan.traces(dtr).cpu().numpy()
    plan.set_tiling()
    auto = list(plan.tiling(dtr.n))
    best, timings, cached = autotune.tune_plan(plan, dtr, cache_path=str(tmp_path / "t.json"))
    cands = autotune.plan_candidates(auto)
    assert not cached and len(timings) == len(cands) and best in cands
    assert all(t > 0 for _, t in timings)
    assert list(plan.tiling(dtr.n))[2] == (best[2] or auto[2])
    np.testing.assert_array_equal(plan.traces(dtr).cpu().numpy(), ref)
    torch.cuda.synchronize()
