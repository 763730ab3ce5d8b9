"""Goal-directed search on the GPU (paper Sec. IV.A top-down search and
bound correction): same sizes as the oracle, valid mappings, and the goal
semantics of mcs_plan_set_goals."""
import ctypes
import json

import numpy as np
import pytest
from _report import write_report

import mcs_instances as mi
import oracle

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _pairs():
    rng = np.random.default_rng(31)
    pairs = [pq for pq in mi.pairs_c4(160, start=4000) if pq[0]["n"] <= 24][:50]
    pairs += mi.pairs_c3(ns=(40,), seeds=range(8))
    pairs += [(mi.random_small(rng, int(rng.integers(0, 14)), float(rng.uniform(0, 1)), True, 2),
               mi.random_small(rng, int(rng.integers(0, 14)), float(rng.uniform(0, 1)), True, 2))
              for _ in range(20)]
    pairs += [(mi.empty_graph(0), mi.empty_graph(3)), (mi.complete_graph(9), mi.complete_graph(9))]
    return pairs


@pytest.mark.parametrize("strategy,ratio", [("top-down", 0), ("bisect", 0), ("dead-end+1", 0),
                                            ("dead-end*2", 0), ("dead-end+1", 2),
                                            ("dead-end*2", 4)])
def test_goal_search_matches_oracle(gpu, strategy, ratio):
    from paper_1908_06418_amd import solve_goals
    pairs = _pairs()
    want = [oracle.mcs(G, H)["size"] for G, H in pairs]
    _say(f"goal search {strategy} ratio {ratio}: {len(pairs)} pairs")
    res, launches = solve_goals(pairs, strategy=strategy, node_limit=20000, time_limit_s=60,
                                with_launches=True, deadend_nodes=2000, deadend_ratio=ratio)
    for (G, H), r, w in zip(pairs, res, want):
        assert r.optimal and r.size == w
        assert len(r.mapping) == r.size and oracle.check.is_valid(G, H, r.mapping)
    assert launches >= 1


def test_dead_end_forecast_gives_valid_partial_results(gpu):
    """A plain batch with the dead-end forecast and a tiny threshold: pairs
    given up are reported unproven (MCS_LIMIT) with a valid mapping no
    larger than the optimum; pairs that finish first are exact."""
    from paper_1908_06418_amd import solve_batch
    pairs = _pairs()
    want = [oracle.mcs(G, H)["size"] for G, H in pairs]
    for tun in ({}, {"seg_lanes": 64}):
        res = solve_batch(pairs, time_limit_s=60, deadend_nodes=50, tuning=tun)
        assert any(not r.optimal for r in res)
        for (G, H), r, w in zip(pairs, res, want):
            assert r.size <= w
            assert r.size == len(r.mapping) and oracle.check.is_valid(G, H, r.mapping)
            if r.optimal:
                assert r.size == w


def test_dead_end_portfolio_and_graph(gpu):
    """The dead-end strategies with the two-order portfolio and with the
    HIP graph: a twin given up must not stop its partner."""
    from paper_1908_06418_amd import solve_goals
    pairs = _pairs()
    want = [oracle.mcs(G, H)["size"] for G, H in pairs]
    for kw in ({"ordering": "portfolio"}, {"tuning": {"use_graph": 1}}):
        res = solve_goals(pairs, strategy="dead-end*2", time_limit_s=60, deadend_nodes=500,
                          **kw)
        assert [r.size for r in res] == want, kw
        assert all(r.optimal for r in res)


def test_bisect_through_graph_drops_node_limit(gpu):
    """Bound correction with the HIP graph: the first (plain) run is node
    limited, the goal runs after it are not -- the graph's kernel node must
    take the changed parameters, or every goal run would stop at the node
    limit and end unsettled."""
    from paper_1908_06418_amd import solve_goals
    pairs = _pairs()
    want = [oracle.mcs(G, H)["size"] for G, H in pairs]
    _say(f"bisect through the graph: {len(pairs)} pairs")
    res = solve_goals(pairs, strategy="bisect", node_limit=20000, time_limit_s=60,
                      tuning={"use_graph": 1})
    for (G, H), r, w in zip(pairs, res, want):
        assert r.optimal and r.size == w
        assert oracle.check.is_valid(G, H, r.mapping)


def test_set_goals_semantics(gpu):
    """goal = optimum: found (size >= goal); goal = optimum + 1: refuted
    (size below goal, settled)."""
    from paper_1908_06418_amd import Plan
    pairs = [pq for pq in mi.pairs_c4(80, start=4500) if pq[0]["n"] <= 22][:20]
    want = [oracle.mcs(G, H)["size"] for G, H in pairs]
    plan = Plan(pairs, time_limit_s=60).upload()
    for delta in (0, 1):
        goals = (ctypes.c_int32 * len(pairs))(*[min(w + delta, min(G["n"], H["n"])) if w + delta
                                                <= min(G["n"], H["n"]) else -1
                                                for (G, H), w in zip(pairs, want)])
        st = plan.lib.mcs_plan_set_goals(plan.handle, goals, ctypes.c_void_p(plan.stream.cuda_stream))
        assert st == 0
        _say(f"set_goals delta={delta}")
        plan.run()
        res = plan.results()
        for i, (r, w) in enumerate(zip(res, want)):
            if goals[i] < 0:
                continue
            assert r.optimal
            if delta == 0:
                assert r.size >= goals[i] and r.size == w
                assert oracle.check.is_valid(*pairs[i], r.mapping)
            else:
                assert r.size < goals[i]
    plan.close()


def test_goal_search_report(gpu):
    """Time to proof of plain, top-down and bisect search on the p = 0.1
    bands, where the MCS covers most of the graph (the case the paper's
    top-down search targets)."""
    from paper_1908_06418_amd import solve_batch, solve_goals
    report = {}
    for n in (30, 35):
        pairs = mi.pairs_c2(ns=(n,), ps=(0.1,))
        row = {}
        import time
        t = time.perf_counter()
        _say(f"report n={n}: plain")
        plain = solve_batch(pairs, time_limit_s=60)
        row["plain_s"] = time.perf_counter() - t
        row["plain_proven"] = sum(r.optimal for r in plain)
        for strat in ("top-down", "bisect", "dead-end+1", "dead-end*2"):
            t = time.perf_counter()
            _say(f"report n={n}: {strat}")
            res, launches = solve_goals(pairs, strategy=strat, node_limit=200000,
                                        time_limit_s=60, with_launches=True,
                                        deadend_nodes=200000, deadend_ratio=2)
            row[f"{strat}_s"] = time.perf_counter() - t
            row[f"{strat}_launches"] = launches
            row[f"{strat}_proven"] = sum(r.optimal for r in res)
            for a, b in zip(plain, res):
                if a.optimal and b.optimal:
                    assert a.size == b.size
        report[f"c2_n{n}_p0.1"] = row
    _say("goal report: " + json.dumps(report))
    write_report("goal_report.json", report)
