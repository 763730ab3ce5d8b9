"""Host logic of the autotuner (no GPU): workload keys, cache round trip,
and the rule that a faster setting with different sizes is an error."""
import pytest

import mcs_instances as mi
from paper_1908_06418_amd import autotune


def test_workload_key_classes():
    k1 = autotune.workload_key(mi.pair_c1())
    assert k1.startswith("w32-u-n16-p") and k1.endswith("b1")
    k2 = autotune.workload_key(mi.pairs_c2(ns=(40,), ps=(0.5,), seeds=range(3)))
    assert k2.startswith("w64-u-n40-p0.5") and k2.endswith("b4")
    k3 = autotune.workload_key(mi.pairs_c3(ns=(40,), seeds=range(2)))
    assert k3.startswith("w64-dl-n40")


def test_cache_round_trip(tmp_path, monkeypatch):
    path = str(tmp_path / "t.json")
    monkeypatch.setenv("MCS_TUNING_FILE", path)
    pairs = mi.pair_c1()
    assert autotune.tuned(pairs) is None
    data = {autotune.workload_key(pairs): {"tuning": {"waves_per_cu": 2}, "kernel_ms": 1.0}}
    autotune.save_cache(data)
    assert autotune.tuned(pairs) == {"waves_per_cu": 2}


def test_pick_fastest_proven():
    ms = [{"tuning": {"a": 1}, "kernel_ms": 5.0, "sizes": [3, 4], "proven": True},
          {"tuning": {"a": 2}, "kernel_ms": 2.0, "sizes": [3, 4], "proven": True},
          {"tuning": {"a": 3}, "kernel_ms": 1.0, "sizes": [3, 4], "proven": False}]
    assert autotune.pick(ms)["tuning"] == {"a": 2}


def test_pick_rejects_disagreeing_sizes():
    ms = [{"tuning": {"a": 1}, "kernel_ms": 5.0, "sizes": [3, 4], "proven": True},
          {"tuning": {"a": 2}, "kernel_ms": 2.0, "sizes": [3, 5], "proven": True}]
    with pytest.raises(RuntimeError):
        autotune.pick(ms)


def test_workload_key_wide_rows():
    k = autotune.workload_key(mi.pairs_w(ns=(80,), seeds=range(2)))
    assert k.startswith("w128-dl-n80")


def test_staged_candidates():
    base = {"seg_lanes": 16}
    c = autotune.staged_candidates(base, "waves_per_cu", (0, 8, 12))
    assert c == [{"seg_lanes": 16}, {"seg_lanes": 16, "waves_per_cu": 8},
                 {"seg_lanes": 16, "waves_per_cu": 12}]
    # children_per_wave applies to one search per wavefront only
    assert autotune.staged_candidates(base, "children_per_wave", (8, 4)) == []
    c = autotune.staged_candidates({"seg_lanes": 64}, "children_per_wave", (8, 4))
    assert c == [{"seg_lanes": 64, "children_per_wave": 8},
                 {"seg_lanes": 64, "children_per_wave": 4}]


def test_staged_search_walks_axes(monkeypatch):
    """Coordinate descent with a fake timer: each stage keeps its fastest
    value, and a candidate timed once is not timed again."""
    calls = []

    def fake_measure(pairs, cand, time_limit_s=30.0, reps=1):
        calls.append(dict(cand))
        ms = 10.0 - (cand.get("seg_lanes") == 8) * 3 - (cand.get("waves_per_cu") == 12) * 2
        return {"tuning": dict(cand), "kernel_ms": ms, "sizes": [1, 2], "proven": True,
                "nodes": 1}

    monkeypatch.setattr(autotune, "measure", fake_measure)
    best = autotune.tune_staged([None], axes=[("seg_lanes", (16, 8)),
                                             ("waves_per_cu", (0, 12, 16))])
    assert best["tuning"] == {"seg_lanes": 8, "waves_per_cu": 12}
    assert best["kernel_ms"] == 5.0
    keys = [tuple(sorted(c.items())) for c in calls]
    assert len(keys) == len(set(keys)) == 4
