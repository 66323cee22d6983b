"""GPU parity of the batched persistent launch (rt_batch_*), through the C ABI.

Each shower of a batch must give what the FP64 oracle gives for that shower
alone (bins exact, so the bars are those of the single-plan path: 1e-5
relative L2 per antenna in FP64 mode, the stated mixed bound otherwise) and
what a single plan gives for it up to summation order. Graph replays
(with eager work between them), launches captured by the caller, launch
shape overrides, empty and non-finite showers, and the workspace check are
covered too.
"""
import math

import numpy as np
import pytest

from paper_2309_03717_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_BOUND = 1e-5
MIXED_BOUND = 1e-6


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_03717_amd import radtrace
    return radtrace


def rel_l2(gpu, ref):
    m = ref.shape[0]
    num = np.linalg.norm((gpu - ref).reshape(m, -1), axis=1)
    den = np.linalg.norm(ref.reshape(m, -1), axis=1)
    assert np.all(num[den == 0] == 0), "GPU wrote into an antenna the oracle leaves empty"
    return np.where(den > 0, num / np.where(den > 0, den, 1), 0.0)


def small_showers(n=10, max_tracks=2000):
    """The first n showers of the 256-shower workload, capped at max_tracks."""
    return W.batched_showers(n, max_tracks=max_tracks)


def host_tracks(sh, precision):
    return sh.tracks(mixed=(precision == "mixed"))


def device_showers(rt, showers, precision, tracks=None):
    out = []
    for i, sh in enumerate(showers):
        tr = tracks[i] if tracks is not None else host_tracks(sh, precision)
        out.append((rt.DeviceDetector.from_array(sh.array), sh.medium, sh.formalism,
                    rt.DeviceTracks.from_tracks(tr)))
    return out


def oracle_of(orc, sh, tracks, precision):
    tr = tracks.widened() if precision == "mixed" else tracks
    return orc.traces(sh.formalism, tr, sh.array, sh.medium, n_threads=8)


def fetch(traces):
    import torch
    torch.cuda.synchronize()
    return [t.double().cpu().numpy() for t in traces]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_matches_oracle_per_shower(rt, orc, precision):
    showers = small_showers()
    kinds = {(s.formalism, s.medium.kind) for s in showers}
    assert len(kinds) >= 3, kinds   # the sample mixes formalisms and media
    tracks = [host_tracks(s, precision) for s in showers]
    b = rt.Batch(device_showers(rt, showers, precision, tracks), precision)
    got = fetch(b.launch())
    bound = FP64_BOUND if precision == "fp64" else MIXED_BOUND
    worst = 0.0
    for sh, tr, g in zip(showers, tracks, got):
        ref = oracle_of(orc, sh, tr, precision)
        assert np.abs(ref).max() > 0
        e = rel_l2(g, ref).max()
        worst = max(worst, e)
        assert e <= bound, (sh.index, sh.formalism, sh.medium.kind, e)
    print(precision, "worst per-antenna rel L2", worst, b.info)


class Shower:
    """A hand-built shower of a batch: array, medium, formalism, tracks."""

    def __init__(self, index, formalism, medium, array, tracks):
        self.index, self.formalism, self.medium, self.array = index, formalism, medium, array
        self._tracks = tracks

    def tracks(self, mixed=False):
        return self._tracks.to_mixed() if mixed else self._tracks


def tilted_star(medium):
    """The 160-antenna star with antenna heights 0 .. 190 m."""
    x, y, _ = W.star_layout(8, 20, 25.0)
    z = (np.arange(x.size) % 20) * 10.0
    return W.make_array(x, y, z, medium, 0.1e-9, 4096)


def heavy_mix():
    """Showers of every medium in one batch: the tabulated profile and the
    spherical Earth (the star at several heights; the inclined shower over a
    14-km grid with 8192 bins, hence several bin segments) between ordinary
    uniform and exponential showers."""
    layered, sph = W.layered_air(), W.SPHERICAL_AIR
    light = small_showers(3, 1500)
    star_t = tilted_star(layered)
    star_s = tilted_star(sph)
    inc_tr, inc_arr = W.inclined_shower(600)
    c1 = W.config(1)
    return [
        light[0],
        Shower(101, "zhs", layered, star_t, c1.tracks(1300)),
        Shower(102, "endpoint", sph, star_s, c1.tracks(900, start=2000)),
        light[1],
        Shower(103, "zhs", sph, inc_arr, inc_tr),
        Shower(104, "endpoint", layered, star_t, c1.tracks(1100, start=5000)),
        light[2],
        Shower(105, "endpoint", sph, inc_arr, inc_tr),
    ]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_heavy_media_batch_matches_oracle(rt, orc, precision):
    """A batch holding tabulated and spherical showers among uniform and
    exponential ones: every shower against the oracle."""
    showers = heavy_mix()
    kinds = {s.medium.kind for s in showers}
    assert {"tabulated", "spherical"} <= kinds and len(kinds) >= 3, kinds
    tracks = [host_tracks(s, precision) for s in showers]
    b = rt.Batch(device_showers(rt, showers, precision, tracks), precision)
    got = fetch(b.launch())
    bound = FP64_BOUND if precision == "fp64" else MIXED_BOUND
    for sh, tr, g in zip(showers, tracks, got):
        ref = oracle_of(orc, sh, tr, precision)
        assert np.abs(ref).max() > 0, sh.index
        e = rel_l2(g, ref).max()
        print(precision, sh.index, sh.formalism, sh.medium.kind, "max rel L2", e)
        assert e <= bound, (sh.index, sh.formalism, sh.medium.kind, e)


HEAVY_OPTIONS = [dict(), dict(items_per_cu=64, max_antennas_per_tile=1),
                 dict(block_threads=128, direct_launch=1),
                 dict(block_threads=1024, max_antennas_per_tile=1)]


@pytest.mark.parametrize("opt", HEAVY_OPTIONS, ids=[str(o) for o in HEAVY_OPTIONS])
def test_heavy_media_batch_equals_single_plans(rt, opt):
    """The same showers through single plans: equal up to summation order,
    whatever the launch shape; graph replays (the F tables rebuilt each time)
    add the same traces again."""
    showers = heavy_mix()
    dev = device_showers(rt, showers, "fp64")
    b = rt.Batch(dev, "fp64", options=rt.BatchOptions(**opt))
    got = fetch(b.launch())
    again = fetch(b.launch())
    for (det, md, f, dtr), g, g2 in zip(dev, got, again):
        ref = fetch([rt.Plan(det, md, f, "fp64").traces(dtr)])[0]
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(g - ref).max() <= 1e-12 * scale, (md.kind, f)
        assert np.abs(g2 - 2 * ref).max() <= 2e-12 * scale, (md.kind, f)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_batch_equals_single_plans(rt, precision):
    showers = small_showers(8, 3000)
    tracks = [host_tracks(s, precision) for s in showers]
    dev = device_showers(rt, showers, precision, tracks)
    got = fetch(rt.Batch(dev, precision).launch())
    tol = 1e-12 if precision == "fp64" else 1e-6
    for (det, md, f, dtr), g in zip(dev, got):
        ref = fetch([rt.Plan(det, md, f, precision).traces(dtr)])[0]
        scale = max(np.abs(ref).max(), 1e-300)
        assert np.abs(g - ref).max() <= tol * scale


OPTIONS = [
    dict(block_threads=256),
    dict(block_threads=64, items_per_cu=1),
    dict(block_threads=1024, max_antennas_per_tile=1),
    dict(block_threads=1024, max_antennas_per_tile=1, items_per_cu=1, direct_launch=1),
    dict(items_per_cu=64),
    dict(max_antennas_per_tile=1),
    dict(max_antennas_per_tile=2, direct_launch=1),
]


@pytest.mark.parametrize("opt", OPTIONS, ids=[str(o) for o in OPTIONS])
def test_launch_shape_invariance(rt, opt):
    showers = small_showers(6, 2500)
    dev = device_showers(rt, showers, "fp64")
    ref = fetch(rt.Batch(dev, "fp64").launch())
    b = rt.Batch(dev, "fp64", options=rt.BatchOptions(**opt))
    got = fetch(b.launch())
    for g, r in zip(got, ref):
        assert np.abs(g - r).max() <= 1e-12 * max(np.abs(r).max(), 1e-300)


def test_per_shower_tiling_with_segments_and_splits(rt, orc):
    """Per-shower overrides: segments of 256 bins (the ZHS prefix scan
    restarts per segment with the folded carry), many track splits, one
    antenna per tile."""
    showers = small_showers(4, 3000)
    dev = device_showers(rt, showers, "fp64")
    per = [(1, 7, 256), (2, 3, 512), (3, 1, 2048), (0, 5, 1024)]
    b = rt.Batch(dev, "fp64", options=rt.BatchOptions(per_shower=per))
    got = fetch(b.launch())
    for sh, g in zip(showers, got):
        ref = oracle_of(orc, sh, host_tracks(sh, "fp64"), "fp64")
        assert rel_l2(g, ref).max() <= FP64_BOUND


def test_graph_replays_with_eager_work_between(rt):
    import torch
    showers = small_showers(8, 2000)
    dev = device_showers(rt, showers, "mixed")
    ref = fetch(rt.Batch(dev, "mixed", options=rt.BatchOptions(direct_launch=1)).launch())
    b = rt.Batch(dev, "mixed")   # graph mode
    det, md, f, dtr = dev[0]
    plan = rt.Plan(det, md, f, "mixed")
    for r in range(4):
        b.zero_traces()
        x = torch.randn(1 << 20, device="cuda").mul_(3.0).sum()   # unrelated eager work
        side = plan.traces(dtr)
        got = fetch(b.launch())
        assert torch.isfinite(x).item() and side.abs().sum().item() > 0
        for g, e in zip(got, ref):
            assert np.abs(g - e).max() <= 1e-6 * max(np.abs(e).max(), 1e-30), r


def test_launch_inside_a_caller_graph(rt):
    """A launch on a stream the caller is capturing joins the caller's graph
    (zeroing by fill kernels inside the graph, no memset nodes)."""
    import torch
    showers = small_showers(5, 1500)
    dev = device_showers(rt, showers, "mixed")
    ref = fetch(rt.Batch(dev, "mixed", options=rt.BatchOptions(direct_launch=1)).launch())
    b = rt.Batch(dev, "mixed")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm-up outside the capture
        b.zero_traces()
        b.launch()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.zero_traces()
        b.launch()
    for r in range(3):
        for t in b.traces:
            t.fill_(123.0)   # replays must overwrite this
        torch.cuda.synchronize()
        g.replay()
        got = fetch(b.traces)
        for gg, e in zip(got, ref):
            assert np.abs(gg - e).max() <= 1e-6 * max(np.abs(e).max(), 1e-30), r


def test_empty_nonfinite_and_odd_showers(rt, orc):
    """An empty shower, a shower whose tracks have non-finite fields mixed
    with good ones, one antenna with 1000 bins (not a multiple of 64)."""
    base = small_showers(3, 1500)
    tr0 = host_tracks(base[0], "fp64")
    bad = tr0.arrays()
    bad["t1"] = bad["t1"].copy()
    bad["t1"][::3] = np.inf
    bad["bx"] = bad["bx"].copy()
    bad["bx"][1::5] = np.nan
    bad_tr = W.Tracks(**bad)
    one = base[2].array
    odd = W.make_array(one.x[:1], one.y[:1], one.z[:1], base[2].medium, one.dt, 1000)
    odd_sh = W.Shower(99, base[2].seed, base[2].n_tracks, odd, base[2].medium, "zhs")
    empty_tr = tr0.slice(0, 0)
    showers = [base[0], base[1], odd_sh, base[1]]
    tracks = [bad_tr, empty_tr, host_tracks(base[2], "fp64"), host_tracks(base[1], "fp64")]
    dev = device_showers(rt, showers, "fp64", tracks)
    got = fetch(rt.Batch(dev, "fp64").launch())
    assert not np.any(got[1])
    for i in (0, 2, 3):
        ref = oracle_of(orc, showers[i], tracks[i], "fp64")
        assert np.all(np.isfinite(got[i]))
        assert rel_l2(got[i], ref).max() <= FP64_BOUND, i


@pytest.mark.parametrize("opt", [dict(), dict(block_threads=1024, max_antennas_per_tile=1)],
                         ids=["default", "one-antenna"])
def test_heavy_media_empty_and_nonfinite_showers(rt, orc, opt):
    """Heavier-media showers that are empty or carry non-finite tracks, next
    to a light shower whose group is then the only non-empty light one:
    empty showers stay zero, the others match the oracle (the bad tracks
    contribute nothing), and a batch whose only heavy shower is empty
    launches no heavy kernel."""
    mix = heavy_mix()
    lay, sph, light = mix[1], mix[2], mix[0]
    tr_lay = host_tracks(lay, "fp64")
    bad = tr_lay.arrays()
    bad["z0"] = bad["z0"].copy()
    bad["z0"][::4] = np.nan
    bad["qw"] = bad["qw"].copy()
    bad["qw"][2::7] = np.inf
    bad_tr = W.Tracks(**bad)
    empty_sph = host_tracks(sph, "fp64").slice(0, 0)
    light_tr = host_tracks(light, "fp64")
    showers = [lay, sph, light, sph]
    tracks = [bad_tr, empty_sph, light_tr, host_tracks(sph, "fp64")]
    dev = device_showers(rt, showers, "fp64", tracks)
    got = fetch(rt.Batch(dev, "fp64", options=rt.BatchOptions(**opt)).launch())
    assert not np.any(got[1])
    for i in (0, 2, 3):
        ref = oracle_of(orc, showers[i], tracks[i], "fp64")
        assert np.all(np.isfinite(got[i])) and np.abs(ref).max() > 0
        assert rel_l2(got[i], ref).max() <= FP64_BOUND, i
    only_empty = fetch(rt.Batch(device_showers(rt, [light, sph], "fp64",
                                               [light_tr, empty_sph]), "fp64").launch())
    assert not np.any(only_empty[1])
    ref = oracle_of(orc, light, light_tr, "fp64")
    assert rel_l2(only_empty[0], ref).max() <= FP64_BOUND


def test_all_empty_batch_is_a_noop(rt):
    sh = small_showers(2, 10)
    tr = [host_tracks(s, "fp64").slice(0, 0) for s in sh]
    b = rt.Batch(device_showers(rt, sh, "fp64", tr), "fp64")
    assert b.info["items"] == 0
    got = fetch(b.launch())
    assert not any(np.any(g) for g in got)


def test_workspace_too_small_and_timing_events(rt):
    import torch
    sh = small_showers(3, 1000)
    b = rt.Batch(device_showers(rt, sh, "mixed"), "mixed")
    small = torch.empty(64, dtype=torch.uint8, device="cuda")
    with pytest.raises(rt.RadtraceError) as e:
        rt.rt_batch_launch(b.handle, small)
    assert e.value.status == rt.RT_E_WORKSPACE
    a = torch.cuda.Event(enable_timing=True)
    z = torch.cuda.Event(enable_timing=True)
    b.set_timing_events(a, z)
    b.launch()
    z.synchronize()
    assert a.elapsed_time(z) > 0


def test_autotuner_picks_and_caches(rt, tmp_path):
    from paper_2309_03717_amd import autotune
    showers = small_showers(6, 2000)
    dev = device_showers(rt, showers, "mixed")
    path = str(tmp_path / "tune.json")
    cands = [[256, 1, 2], [512, 3, 4], [512, 2, 8]]
    opt, timings, cached = autotune.tune_batch(dev, "mixed", cache_path=path, candidates=cands)
    assert not cached and len(timings) == 3
    assert [opt.block_threads, opt.max_antennas_per_tile, opt.items_per_cu] in cands
    opt2, _, cached2 = autotune.tune_batch(dev, "mixed", cache_path=path, candidates=cands)
    assert cached2 and opt2 == opt
    ref = fetch(rt.Batch(dev, "mixed").launch())
    got = fetch(rt.Batch(dev, "mixed", options=opt).launch())
    for g, e in zip(got, ref):
        assert np.abs(g - e).max() <= 1e-6 * max(np.abs(e).max(), 1e-30)


def test_batch_autotune_entry_point_times_every_candidate(rt):
    """rt_batch_autotune through the binding: one time per candidate, None
    for a candidate the planner refuses (a tile wider than three antennas),
    and the showers' own traces untouched (the tuner's launches go to
    scratch traces)."""
    showers = small_showers(4, 1500)
    dev = device_showers(rt, showers, "mixed")
    cands = [rt.BatchOptions(block_threads=256, max_antennas_per_tile=1, items_per_cu=2),
             rt.BatchOptions(block_threads=512, max_antennas_per_tile=4),
             rt.BatchOptions(block_threads=1024, max_antennas_per_tile=1, items_per_cu=4)]
    times = rt.rt_batch_autotune(dev, "mixed", 1.0, cands, reps=2)
    assert len(times) == 3 and times[1] is None
    assert times[0] > 0 and times[2] > 0


def test_batch_tables_travel_in_the_workspace(rt):
    """The batch's tables live in the caller's workspace: two batches of
    different showers launched alternately on one shared workspace (each
    launch copies its own tables first) give each batch's own results."""
    import torch
    a_sh, b_sh = small_showers(3, 1000), small_showers(6, 1200)[3:]
    a = rt.Batch(device_showers(rt, a_sh, "mixed"), "mixed", options=rt.BatchOptions(direct_launch=1))
    b = rt.Batch(device_showers(rt, b_sh, "mixed"), "mixed", options=rt.BatchOptions(direct_launch=1))
    ref_a, ref_b = fetch(a.launch()), fetch(b.launch())
    shared = torch.empty(max(a.workspace.numel(), b.workspace.numel()), dtype=torch.uint8,
                         device="cuda")
    for bt in (a, b):
        bt.zero_traces()
    for _ in range(2):
        rt.rt_batch_launch(a.handle, shared)
        rt.rt_batch_launch(b.handle, shared)
    for got, ref in ((fetch(a.traces), ref_a), (fetch(b.traces), ref_b)):
        for g, e in zip(got, ref):
            np.testing.assert_allclose(g, 2 * e, rtol=0, atol=1e-5 * max(np.abs(e).max(), 1e-30))


SHAPES = [dict(), dict(block_threads=256, items_per_cu=1),
          dict(block_threads=1024, max_antennas_per_tile=1, items_per_cu=8),
          dict(max_antennas_per_tile=1, direct_launch=1)]


def test_mixed_zhs_batches_are_bitwise_identical_across_launch_shapes(rt):
    """Mixed ZHS showers accumulate in 64-bit fixed point with a unit per
    shower: every launch shape (workgroup size, tile width, items per CU,
    graph or direct) and a single plan over the same tracks give the same
    bits; the Endpoint showers agree to summation order."""
    showers = small_showers(8, 3000)
    assert {s.formalism for s in showers} == {"zhs", "endpoint"}
    tracks = [host_tracks(s, "mixed") for s in showers]
    dev = device_showers(rt, showers, "mixed", tracks)
    runs = [fetch(rt.Batch(dev, "mixed", options=rt.BatchOptions(**o)).launch()) for o in SHAPES]
    singles = [fetch([rt.Plan(det, md, f, "mixed").traces(dtr)])[0] for det, md, f, dtr in dev]
    for i, sh in enumerate(showers):
        for r in runs[1:]:
            if sh.formalism == "zhs":
                np.testing.assert_array_equal(r[i], runs[0][i], err_msg=f"shower {i}")
            else:
                assert np.abs(r[i] - runs[0][i]).max() <= 1e-6 * max(np.abs(runs[0][i]).max(), 1e-300)
        if sh.formalism == "zhs":
            np.testing.assert_array_equal(runs[0][i], singles[i], err_msg=f"shower {i} vs plan")
