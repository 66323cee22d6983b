"""The track filter (rt_filter_tracks) on the GPU: the kept tracks are exactly
the numpy selection of the stated predicate, in input order, for ragged
sizes and for inputs whose counts span several scan chunks; deposits of the
kept tracks equal deposits of all tracks (qw_min = 0: every dropped track
contributes nothing) up to summation order; an all-dropped input and a
filter on another stream behave; the predicate's boundaries (a weight equal
to the threshold, signed zeros, subnormal velocities, one-ulp durations)."""
import numpy as np
import pytest

from paper_2309_03717_amd import workloads as W
from helpers import expected_mask, planted

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_03717_amd import radtrace
    return radtrace


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


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_predicate_boundaries(rt, precision):
    """|qw| equal to qw_min is dropped (strict), a negative weight counts by
    its magnitude, -0.0 velocity components are at rest, a subnormal one
    moves, and a track differing from a point only in its end time is kept."""
    low = np.float64 if precision == "fp64" else np.float32
    tiny = np.finfo(low).smallest_subnormal
    n = 8
    a = W.config(1).tracks(n).arrays()
    a = {f: v.astype(low if f in ("bx", "by", "bz", "qw") else np.float64) for f, v in a.items()}
    qw_min = 0.25
    a["qw"][:] = 1.0
    a["qw"][0] = low(qw_min)                         # dropped: not above the threshold
    a["qw"][1] = low(-1.0)                           # kept: |qw| counts
    a["qw"][2] = np.nextafter(low(qw_min), low(1))   # kept: just above
    for f in ("bx", "by", "bz"):
        a[f][3] = low(-0.0)                          # dropped: at rest
    a["bx"][4], a["by"][4], a["bz"][4] = tiny, low(0), low(-0.0)   # kept: moves
    for f in ("x", "y", "z", "t"):
        a[f + "1"][5] = a[f + "0"][5]                # dropped: a point
    for f in ("x", "y", "z"):
        a[f + "1"][6] = a[f + "0"][6]
    a["t1"][6] = np.nextafter(a["t0"][6], np.inf)    # kept: lasts one ulp
    tr = W.Tracks(**a)
    want = np.array([0, 1, 1, 0, 1, 0, 1, 1], bool)
    assert np.array_equal(expected_mask(tr, qw_min), want)
    got = rt.filter_tracks(rt.DeviceTracks.from_tracks(tr), precision, qw_min)
    assert got.n == int(want.sum())
    for f in W.TRACK_FIELDS:
        assert np.array_equal(getattr(got, f).cpu().numpy(), np.asarray(getattr(tr, f))[want]), f
