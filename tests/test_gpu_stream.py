"""Host-resident track streams (streaming.HostTrackStream): chunks copied
from pinned host memory on a copy stream, double-buffered, deposited by the
library's plans. The streamed traces must equal those of the same chunks
deposited from device memory (up to LDS summation order) and the oracle's.
With a filter threshold, the streamed traces equal the deposits of the numpy
selection of each chunk's kept tracks, and every kept track is counted once."""
import numpy as np
import pytest

from paper_2309_03717_amd import workloads as W
from helpers import expected_mask, planted

pytestmark = pytest.mark.gpu

CHUNK = 20000
SIZES = [CHUNK, CHUNK, 7000, CHUNK, 1]   # a ragged chunk and a single track


@pytest.fixture(scope="module")
def rt():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_03717_amd import radtrace
    return radtrace


def chunks(mixed):
    w = W.config(1)
    out, lo = [], 0
    for n in SIZES:
        out.append(w.tracks(n, start=lo, mixed=mixed))
        lo += n
    return w, out


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_streamed_chunks_equal_resident_and_oracle(rt, orc, precision):
    import torch
    from paper_2309_03717_amd import streaming as S
    w, parts = chunks(precision == "mixed")
    det = rt.DeviceDetector.from_array(w.array)
    plans = [rt.Plan(det, w.medium, f, precision) for f in ("endpoint", "zhs")]
    resident = [p.new_traces() for p in plans]
    for part in parts:
        dt = rt.DeviceTracks.from_tracks(part)
        for p, tr in zip(plans, resident):
            p.accumulate(dt, tr)
    streamed = [p.new_traces() for p in plans]
    st = S.HostTrackStream(plans, CHUNK)
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    for rep in range(2):   # two passes: the buffers are reused across calls
        # the second pass runs with another current stream: the stream's own
        # copies and buffer reuse order through its events; the traces both
        # passes add to are the caller's, so the caller orders the two streams
        if rep == 1:
            side.wait_stream(main)
        with torch.cuda.stream(side if rep == 1 else main):
            for part in parts:
                st.push(S.pinned_chunk(part), streamed)
    st.synchronize()
    torch.cuda.synchronize()
    allt = W.Tracks.concat(parts)
    for f, p, r, s in zip(("endpoint", "zhs"), plans, resident, streamed):
        r = r.double().cpu().numpy()
        s = s.double().cpu().numpy()
        scale = np.abs(r).max()
        assert scale > 0
        tol = 1e-12 if precision == "fp64" else 1e-6
        np.testing.assert_allclose(s, 2 * r, rtol=0, atol=2 * tol * scale, err_msg=f)
        ref = orc.traces(f, allt.widened() if precision == "mixed" else allt, w.array, w.medium,
                         n_threads=8)
        num = np.linalg.norm((s / 2 - ref).reshape(w.array.m, -1), axis=1)
        den = np.linalg.norm(ref.reshape(w.array.m, -1), axis=1)
        err = np.where(den > 0, num / np.where(den > 0, den, 1), 0.0).max()
        print(f, precision, "streamed vs oracle max rel L2", err)
        assert err <= (1e-5 if precision == "fp64" else 1e-6)


def planted_chunks(precision):
    """The chunk sizes above with droppable tracks planted, plus a chunk in
    which every track is dropped."""
    parts, lo = [], 0
    for i, n in enumerate(SIZES):
        parts.append(planted(n, precision, seed=10 + i, start=lo))
        lo += n
    a = planted(3000, precision, seed=9, start=lo).arrays()
    a["qw"] = np.zeros_like(a["qw"])
    parts.insert(2, W.Tracks(**a))
    return parts


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("qw_min", [0.0, 1e-3])
def test_filtered_stream_equals_deposits_of_kept_tracks(rt, precision, qw_min):
    import torch
    from paper_2309_03717_amd import streaming as S
    w = W.config(1)
    parts = planted_chunks(precision)
    det = rt.DeviceDetector.from_array(w.array)
    plans = [rt.Plan(det, w.medium, f, precision) for f in ("endpoint", "zhs")]
    ref = [p.new_traces() for p in plans]
    n_kept = 0
    for part in parts:
        mask = expected_mask(part, qw_min)
        n_kept += int(mask.sum())
        if mask.any():
            sel = W.Tracks(**{f: np.asarray(getattr(part, f))[mask] for f in W.TRACK_FIELDS})
            dt = rt.DeviceTracks.from_tracks(sel)
            for p, tr in zip(plans, ref):
                p.accumulate(dt, tr)
    assert 0 < n_kept < sum(p.n for p in parts)
    streamed = [p.new_traces() for p in plans]
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    main = torch.cuda.current_stream()
    with S.HostTrackStream(plans, CHUNK, qw_min=qw_min) as st:
        for rep in range(2):
            # the second pass runs on another stream: the first pass's last
            # chunk is flushed (deposited on its own stream) before that
            # stream waits; the last chunk of all is flushed on exit, on the
            # side stream
            if rep == 1:
                st.flush()
                side.wait_stream(main)
            with torch.cuda.stream(side if rep == 1 else main):
                for part in parts:
                    st.push(S.pinned_chunk(part), streamed)
    torch.cuda.synchronize()
    assert st.kept == 2 * n_kept
    tol = 1e-12 if precision == "fp64" else 1e-6
    for f, r, s in zip(("endpoint", "zhs"), ref, streamed):
        r = r.double().cpu().numpy()
        s = s.double().cpu().numpy()
        scale = np.abs(r).max()
        assert scale > 0
        np.testing.assert_allclose(s, 2 * r, rtol=0, atol=2 * tol * scale, err_msg=f)


def test_stream_rejects_bad_chunks(rt):
    import torch
    from paper_2309_03717_amd import streaming as S
    w, parts = chunks(True)
    det = rt.DeviceDetector.from_array(w.array)
    plan = rt.Plan(det, w.medium, "zhs", "mixed")
    st = S.HostTrackStream([plan], 1000)
    tr = [plan.new_traces()]
    small = W.config(1).tracks(10, mixed=True)
    ok = S.pinned_chunk(small)
    pageable = {f: torch.from_numpy(getattr(small, f)) for f in W.TRACK_FIELDS}
    with pytest.raises(ValueError, match="pinned"):
        st.push(pageable, tr)
    with pytest.raises(ValueError, match="max_chunk"):
        st.push(S.pinned_chunk(parts[0]), tr)
    wrong = dict(ok)
    wrong["qw"] = ok["qw"].double().pin_memory()
    with pytest.raises(ValueError, match="qw"):
        st.push(wrong, tr)
    short = dict(ok)
    short["x0"] = ok["x0"][:5].clone().pin_memory()
    with pytest.raises(ValueError, match="same length"):
        st.push(short, tr)
    with pytest.raises(ValueError, match="one trace tensor per plan"):
        st.push(ok, tr * 2)
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(ValueError, match="qw_min"):
            S.HostTrackStream([plan], 1000, qw_min=bad)
    fp64 = rt.Plan(det, w.medium, "zhs", "fp64")
    with pytest.raises(ValueError, match="precision"):
        S.HostTrackStream([plan, fp64], 1000)
    st.push(ok, tr)   # still usable after the rejections
    st.synchronize()
    assert torch.isfinite(tr[0]).all()
