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


def test_finalists_are_timed_again_on_the_whole_workload(tmp_path):
    """The sample ranks (1024, 1) first by a hair; the whole workload ranks
    (512, 3) first: the final stage re-times the three best and takes its
    winner, and never times the fourth."""
    sample = {(1024, 1): 1.00, (512, 3): 1.01, (512, 2): 1.02, (256, 1): 2.0}
    whole = {(1024, 1): 10.3, (512, 3): 10.0, (512, 2): 10.2, (256, 1): 1.0}
    finals = []

    def final(c):
        finals.append(tuple(c))
        return whole[tuple(c)]

    cands = [[256, 1], [512, 2], [512, 3], [1024, 1]]
    best, timings, cached = autotune.tune("f", cands, lambda c: sample[tuple(c)],
                                          autotune.TuningCache(str(tmp_path / "f.json")),
                                          final_measure=final)
    assert best == [512, 3] and not cached
    assert sorted(finals) == [(512, 2), (512, 3), (1024, 1)]
    best2, _, _ = autotune.tune("g", cands, lambda c: sample[tuple(c)],
                                autotune.TuningCache(str(tmp_path / "g.json")))
    assert best2 == [1024, 1]   # without the final stage the sample decides


def test_finalists_come_from_distinct_families(tmp_path):
    """Three variants of one family lead the sample; the final stage takes
    only the best of them and goes on to the next families."""
    sample = {(1024, 1, 2): 1.00, (1024, 1, 4): 1.001, (1024, 1, 8): 1.002,
              (512, 3, 2): 1.01, (512, 2, 2): 1.02, (256, 1, 2): 1.03}
    whole = {(1024, 1, 2): 10.3, (512, 3, 2): 10.0, (512, 2, 2): 10.2}
    finals = []

    def final(c):
        finals.append(tuple(c))
        return whole[tuple(c)]

    best, _, _ = autotune.tune("h", [list(c) for c in sample], lambda c: sample[tuple(c)],
                               autotune.TuningCache(str(tmp_path / "h.json")),
                               final_measure=final, family=lambda c: (c[0], c[1]))
    assert best == [512, 3, 2]
    assert finals == [(1024, 1, 2), (512, 3, 2), (512, 2, 2)]


def test_plan_candidates_add_shorter_track_splits():
    """The plan autotuner's default candidates: every block size and pass
    length with the automatic tile, plus the automatic launch with twice the
    automatic split count (shorter splits suit time-ordered track streams)."""
    auto = (1, 4, 1024, 4096, 1 << 20)
    cands = autotune.plan_candidates(auto)
    base = [[0, 0, b, 0, p] for b in autotune.PLAN_BLOCKS for p in autotune.PLAN_PASSES]
    assert cands[:len(base)] == base
    assert cands[len(base):] == [[0, 8, 1024, 0, 1 << 20]]
    assert len({tuple(c) for c in cands}) == len(cands)
