"""Parity at the full workload sizes, in the launch configurations bench.py
times (default tilings: 2^20-track passes, ZHS splits of 128K tracks, one
antenna per LDS tile at 4096 bins).

Each antenna's trace depends only on that antenna, so the GPU traces of the
whole array are compared with the oracle run on a sample of the antennas
(corners, centre, edges and random ones) over every track of the chunk or
workload. Same bars as the small parity tests: 1e-5 relative L2 per antenna
in FP64 mode, the stated 1e-6 in mixed mode.
"""
import os

import numpy as np
import pytest

from paper_2309_03717_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64_BOUND = 1e-5
MIXED_BOUND = 1e-6
THREADS = max(1, min(16, len(os.sched_getaffinity(0))))


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


def sample_antennas(m, nx=None, seed=7):
    picks = {0, m - 1, m // 2}
    if nx:
        picks |= {nx - 1, m - nx, (m // nx // 2) * nx + nx // 2}
    rng = np.random.default_rng(seed)
    picks |= set(rng.choice(m, size=min(m, 3), replace=False).tolist())
    return np.array(sorted(picks))


def sub_array(arr, idx):
    return W.AntennaArray(arr.x[idx], arr.y[idx], arr.z[idx], arr.t_start[idx], arr.dt,
                          arr.n_bins)


def gpu_full(rt, arr, medium, formalism, precision, tracks, k):
    import torch
    det = rt.DeviceDetector.from_array(arr)
    plan = rt.Plan(det, medium, formalism, precision, k)
    out = plan.traces(rt.DeviceTracks.from_tracks(tracks))
    torch.cuda.synchronize()
    tiling = plan.tiling(tracks.n)
    res = out.double().cpu().numpy()
    del out, plan
    return res, tiling


@pytest.mark.parametrize("formalism", ["endpoint", "zhs"])
@pytest.mark.parametrize("which", ["first", "last"])
def test_grid4096_chunk_sampled_antennas(rt, orc, formalism, which):
    """The 4096-antenna grid, mixed precision, SI prefactor: the first chunk of
    2^22 tracks and the ragged last chunk (3,531,008 tracks), whole array on
    the GPU, eight antennas checked against the oracle."""
    w = W.config(2)
    start = 0 if which == "first" else (w.n_tracks // w.chunk) * w.chunk
    n = min(w.chunk, w.n_tracks - start)
    tr = w.tracks(n, start=start, mixed=True)
    k = 4.80320471518522e-18
    got, tiling = gpu_full(rt, w.array, w.medium, formalism, "mixed", tr, k)
    assert tiling[4] == 1 << 20 and tiling[0] == 1
    if formalism == "zhs":
        assert tiling[1] == 8
    idx = sample_antennas(w.array.m, nx=64)
    ref = orc.traces(formalism, tr.widened(), sub_array(w.array, idx), w.medium, k=k,
                     n_threads=THREADS)
    err = rel_l2(got[idx], ref)
    print(formalism, which, n, "tracks: max rel L2", err.max(), "antennas", idx.tolist())
    assert np.abs(ref).max() > 0
    assert err.max() <= MIXED_BOUND


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_star160_all_tracks_sampled_antennas(rt, orc, precision):
    """The 160-antenna star with all 1e7 tracks, both formalisms."""
    w = W.config(1)
    tr = w.tracks(mixed=(precision == "mixed"))
    idx = sample_antennas(w.array.m)
    sub = sub_array(w.array, idx)
    bound = FP64_BOUND if precision == "fp64" else MIXED_BOUND
    for f in ("endpoint", "zhs"):
        got, _ = gpu_full(rt, w.array, w.medium, f, precision, tr, 1.0)
        ref = orc.traces(f, tr.widened() if precision == "mixed" else tr, sub, w.medium,
                         n_threads=THREADS)
        err = rel_l2(got[idx], ref)
        print(f, precision, "1e7 tracks: max rel L2", err.max())
        assert err.max() <= bound


def test_adjoint_full_workload(rt, orc):
    """ZHS adjoint on all 1e6 tracks and 64 antennas (mixed inputs) against the
    oracle's adjoint for the same upstream gradient."""
    import torch
    w = W.config(3)
    tr = w.tracks(mixed=True)
    grad = np.random.default_rng(11).normal(size=(w.array.m, w.array.n_bins, 3)).astype(np.float32)
    det = rt.DeviceDetector.from_array(w.array)
    plan = rt.Plan(det, w.medium, "zhs", "mixed")
    out = plan.zhs_vjp(rt.DeviceTracks.from_tracks(tr), torch.from_numpy(grad).to("cuda"))
    torch.cuda.synchronize()
    gq, gp0, gp1, gn = [o.cpu().numpy() for o in out]
    ref = orc.zhs_vjp(tr.widened(), w.array, w.medium, grad.astype(np.float64), n_threads=THREADS)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
    errs = {"qw": rel(gq, ref["qw"]), "p0": rel(gp0, ref["p0"]), "p1": rel(gp1, ref["p1"]),
            "n0m1": rel(gn[0], ref["n0m1"])}
    print("adjoint 1e6 tracks", errs)
    for key, v in errs.items():
        assert v <= 1e-9, (key, v)


def test_batched_256_showers_sampled(rt, orc):
    """All 256 showers in one graph-replayed batch (default options); four
    showers of different kinds checked in full against the oracle."""
    import torch
    showers = W.batched_showers()
    dev, tracks = [], []
    for sh in showers:
        t = sh.tracks(mixed=True)
        tracks.append(t)
        dev.append((rt.DeviceDetector.from_array(sh.array), sh.medium, sh.formalism,
                    rt.DeviceTracks.from_tracks(t)))
    b = rt.Batch(dev, "mixed")
    b.launch()
    torch.cuda.synchronize()
    picks, seen = [], set()
    for i, sh in enumerate(showers):
        kind = (sh.formalism, sh.medium.kind)
        if kind not in seen and sh.n_tracks * sh.array.m < 3e8:
            seen.add(kind)
            picks.append(i)
    assert len(picks) == 4
    for i in picks:
        sh = showers[i]
        got = b.traces[i].double().cpu().numpy()
        ref = orc.traces(sh.formalism, tracks[i].widened(), sh.array, sh.medium,
                         n_threads=THREADS)
        err = rel_l2(got, ref)
        print("shower", i, sh.formalism, sh.medium.kind, sh.n_tracks, sh.array.m, sh.array.n_bins,
              "max rel L2", err.max())
        assert err.max() <= MIXED_BOUND


@pytest.mark.parametrize("formalism", ["endpoint", "zhs"])
def test_shower_like_stream_sampled_antennas(rt, orc, formalism):
    """A time-ordered, shower-like chunk of 2^22 tracks on the 4096-antenna
    grid (neighbouring lanes land in neighbouring bins at antennas near the
    axis): sampled antennas, centre ones included, against the oracle."""
    w = W.config(2)
    tr = W.shower_tracks(W.SHOWER_SEED, 1 << 22).to_mixed()
    k = 4.80320471518522e-18
    got, _ = gpu_full(rt, w.array, w.medium, formalism, "mixed", tr, k)
    idx = np.unique(np.concatenate([sample_antennas(w.array.m, nx=64),
                                    [2015, 2016, 2079, 2080, 2081, 2144]]))
    ref = orc.traces(formalism, tr.widened(), sub_array(w.array, idx), w.medium, k=k,
                     n_threads=THREADS)
    err = rel_l2(got[idx], ref)
    print(formalism, "shower-like: max rel L2", err.max())
    assert np.abs(ref).max() > 0
    assert err.max() <= MIXED_BOUND


@pytest.mark.parametrize("formalism", ["endpoint", "zhs"])
def test_grid4096_one_pass_every_antenna(rt, orc, formalism):
    """One 2^20-track pass of the grid workload (the launch the bench times:
    2^20-track passes, eight ZHS splits, one 4096-bin tile per workgroup in
    the XCD-major block order) over all 4096 antennas, every antenna against
    the oracle (4.3e9 pairs): mixed bound per antenna, and for the Endpoint
    the same set of nonzero bins as the oracle (no impulse misplaced)."""
    import torch
    w = W.config(2)
    tr = w.tracks(1 << 20, mixed=True)
    det = rt.DeviceDetector.from_array(w.array)
    plan = rt.Plan(det, w.medium, formalism, "mixed", 1.0)
    assert plan.tiling(tr.n)[4] == 1 << 20   # one pass
    gpu = plan.traces(rt.DeviceTracks.from_tracks(tr))
    torch.cuda.synchronize()
    gpu = gpu.cpu().numpy().astype(np.float64)
    ref = orc.traces(formalism, tr.widened(), w.array, w.medium, k=1.0, n_threads=THREADS)
    err = rel_l2(gpu, ref)
    print(f"{formalism}: 4096 antennas, max rel L2 {err.max():.3e}, median {np.median(err):.3e}")
    assert err.max() <= MIXED_BOUND
    if formalism == "endpoint":
        np.testing.assert_array_equal(gpu != 0, ref != 0)
