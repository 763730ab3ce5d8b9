"""The autotuner on the GPU: it times candidates through the C ABI, every
candidate gives the same sizes, and the winner is cached per workload class."""
import pytest

import mcs_instances as mi
import oracle

pytestmark = pytest.mark.gpu


def test_tune_small_grid(gpu, tmp_path, monkeypatch):
    from paper_1908_06418_amd import autotune, solve_batch
    monkeypatch.setenv("MCS_TUNING_FILE", str(tmp_path / "tuning.json"))
    pairs = [pq for pq in mi.pairs_c4(120, start=6000) if pq[0]["n"] <= 24][:32]
    want = [oracle.mcs(G, H)["size"] for G, H in pairs]
    cands = [{"waves_per_cu": w, "children_per_wave": c} for w in (1, 4) for c in (1, 8)]
    best = autotune.tune_and_store(pairs, candidates=cands, time_limit_s=60,
                                   log=lambda m: print(m["tuning"], m["kernel_ms"], flush=True))
    assert best["sizes"] == want
    assert len(best["table"]) == len(cands)
    assert best["kernel_ms"] == min(m["kernel_ms"] for m in best["table"])
    cached = autotune.tuned(pairs)
    assert cached == best["tuning"]
    res = solve_batch(pairs, time_limit_s=60, tuning=cached)
    assert [r.size for r in res] == want


def test_tune_staged_small(gpu, tmp_path):
    """Coordinate descent over layout, wavefronts and queue depth on a small
    sample: every candidate gives the oracle's sizes and the winner is at
    least as fast as every candidate of the last stage."""
    from paper_1908_06418_amd import autotune
    pairs = [pq for pq in mi.pairs_c4(120, start=6000) if pq[0]["n"] <= 24][:32]
    want = [oracle.mcs(G, H)["size"] for G, H in pairs]
    axes = [("seg_lanes", (16, 8, 64)), ("waves_per_cu", (0, 8)), ("ring_slots", (0, 4096))]
    best = autotune.tune_and_store(pairs, path=str(tmp_path / "t.json"), staged=True,
                                   axes=axes, time_limit_s=60,
                                   log=lambda m: print(m["stage"], m["tuning"], m["kernel_ms"],
                                                       flush=True))
    assert all(m["sizes"] == want for m in best["table"])
    last = [m for m in best["table"] if m["stage"] == "ring_slots"]
    assert best["kernel_ms"] <= min(m["kernel_ms"] for m in last)
    assert autotune.tuned(pairs, path=str(tmp_path / "t.json")) == best["tuning"]
