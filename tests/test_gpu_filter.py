"""The track filter (rt_filter_tracks) on the GPU: the kept tracks are exactly
the numpy selection of the stated predicate, in input order, for ragged
sizes and for inputs whose counts span several scan chunks; deposits of the
kept tracks equal deposits of all tracks (qw_min = 0: every dropped track
contributes nothing) up to summation order; an all-dropped input and a
filter on another stream behave."""
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


def planted(n, precision, seed=3):
    """n star-workload tracks with droppable ones planted: zero and small
    weights, non-finite fields, points (zero length and duration), tracks at
    rest, and the kept near-misses (zero length with a duration, a duration of
    zero with a length)."""
    a = W.config(1).tracks(n).arrays()
    for f in a:
        a[f] = a[f].copy()
    rng = np.random.default_rng(seed)
    pick = lambda: rng.random(n) < 0.06
    a["qw"][pick()] = 0.0
    a["qw"][pick()] *= 1e-4
    a["x0"][pick()] = np.nan
    a["t1"][pick()] = np.inf
    a["bz"][pick()] = -np.inf
    pts = pick()
    for f in ("x", "y", "z", "t"):
        a[f + "1"][pts] = a[f + "0"][pts]
    rest = pick()
    for f in ("bx", "by", "bz"):
        a[f][rest] = 0.0
    still = pick()                                   # kept: lasts but does not move in space
    for f in ("x", "y", "z"):
        a[f + "1"][still] = a[f + "0"][still]
    instant = pick()                                 # kept: moves in no time
    a["t1"][instant] = a["t0"][instant]
    tr = W.Tracks(**a)
    return tr.to_mixed() if precision == "mixed" else tr


def expected_mask(tr, qw_min):
    f = {k: np.asarray(getattr(tr, k)).astype(np.float64) for k in W.TRACK_FIELDS}
    finite = np.all([np.isfinite(v) for v in f.values()], axis=0)
    with np.errstate(invalid="ignore"):
        moves = (f["bx"] != 0) | (f["by"] != 0) | (f["bz"] != 0)
        extends = ((f["x1"] != f["x0"]) | (f["y1"] != f["y0"]) | (f["z1"] != f["z0"])
                   | (f["t1"] != f["t0"]))
        heavy = np.abs(f["qw"]) > qw_min
    return finite & heavy & moves & extends


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n", [0, 1, 255, 256, 257, 70_001, 300_000])
def test_filter_matches_the_numpy_selection(rt, precision, n):
    tr = planted(n, precision)
    dev = rt.DeviceTracks.from_tracks(tr)
    for qw_min in (0.0, 1e-3):
        got = rt.filter_tracks(dev, precision, qw_min)
        mask = expected_mask(tr, qw_min)
        assert got.n == int(mask.sum()), (n, qw_min)
        for f in W.TRACK_FIELDS:
            want = np.asarray(getattr(tr, f))[mask]
            assert np.array_equal(getattr(got, f).cpu().numpy(), want), (f, n, qw_min)
        if n >= 1000:
            assert 0 < got.n < n                     # some of everything was planted


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_deposits_of_kept_tracks_equal_all_tracks(rt, precision):
    """With qw_min = 0 the filter drops only tracks that contribute exactly
    nothing, so the traces agree up to summation order."""
    w = W.config(1)
    tr = planted(20_000, precision, seed=5)
    dev = rt.DeviceTracks.from_tracks(tr)
    kept = rt.filter_tracks(dev, precision, 0.0)
    assert kept.n < tr.n
    det = rt.DeviceDetector.from_array(w.array)
    tol = 1e-12 if precision == "fp64" else 1e-6
    for formalism in ("endpoint", "zhs"):
        plan = rt.Plan(det, w.medium, formalism, precision)
        every = plan.traces(dev).double().cpu().numpy()
        some = plan.traces(kept).double().cpu().numpy()
        scale = np.abs(every).max()
        assert scale > 0
        assert np.abs(some - every).max() <= tol * scale, formalism


def test_all_dropped_and_another_stream(rt):
    import torch
    tr = planted(5000, "mixed")
    a = tr.arrays()
    a["qw"] = np.zeros_like(a["qw"])
    none = rt.filter_tracks(rt.DeviceTracks.from_tracks(W.Tracks(**a)), "mixed")
    assert none.n == 0
    dev = rt.DeviceTracks.from_tracks(tr)
    ref = rt.filter_tracks(dev, "mixed", 1e-3)
    side = torch.cuda.Stream()
    got = rt.filter_tracks(dev, "mixed", 1e-3, stream=side)
    assert got.n == ref.n > 0
    for f in W.TRACK_FIELDS:
        assert torch.equal(getattr(got, f), getattr(ref, f)), f
