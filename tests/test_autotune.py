"""The autotuner's selection and cache logic, with a synthetic timing
function (the device timing itself is covered by the GPU batch tests)."""
import json

import pytest

from paper_2309_03717_amd import autotune


def test_tune_picks_fastest_skips_rejected_and_caches(tmp_path):
    path = str(tmp_path / "t.json")
    cost = {(256, 1): 3.0, (512, 2): 1.5, (512, 3): 2.0}
    seen = []

    def measure(c):
        seen.append(tuple(c))
        if tuple(c) == (64, 9):
            raise RuntimeError("rejected by the library")
        return cost[tuple(c)]

    cands = [[256, 1], [64, 9], [512, 2], [512, 3]]
    best, timings, cached = autotune.tune("k1", cands, measure, autotune.TuningCache(path))
    assert best == [512, 2] and not cached
    assert [c for c, _ in timings] == [[256, 1], [512, 2], [512, 3]]
    data = json.load(open(path))
    assert data["k1"]["best"] == [512, 2]
    seen.clear()
    best2, timings2, cached2 = autotune.tune("k1", cands, measure, autotune.TuningCache(path))
    assert cached2 and best2 == [512, 2] and timings2 is None and not seen
    best3, _, cached3 = autotune.tune("k2", [[512, 3]], measure, autotune.TuningCache(path))
    assert best3 == [512, 3] and not cached3
    assert set(json.load(open(path))) == {"k1", "k2"}


def test_tune_with_no_measurable_candidate_raises(tmp_path):
    def measure(c):
        raise ValueError("no")
    with pytest.raises(RuntimeError):
        autotune.tune("k", [[1]], measure, autotune.TuningCache(str(tmp_path / "x.json")))


def test_unreadable_cache_starts_afresh(tmp_path):
    p = tmp_path / "bad.json"
    p.write_text("{not json")
    c = autotune.TuningCache(str(p))
    assert c.get("anything") is None
    c.put("a", [1], [[[1], 0.5]])
    assert autotune.TuningCache(str(p)).get("a") == [1]


def test_signature_depends_on_every_shape():
    a = autotune.signature([("zhs", "uniform", 16, 2048, 1000)])
    b = autotune.signature([("zhs", "uniform", 16, 2048, 1001)])
    c = autotune.signature([("endpoint", "uniform", 16, 2048, 1000)])
    assert len({a, b, c}) == 3
    assert a == autotune.signature([("zhs", "uniform", 16, 2048, 1000)])
