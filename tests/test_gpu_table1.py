"""The paper's worked example (Sec. II.B, Table 1: two 4-vertex graphs that
the table's labels fix, tests/golden/table1.json) on the GPU: size 4, a
valid mapping, and in single-wavefront mode the oracle's node count."""
import json
import os

import pytest

import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table1_pair():
    with open(os.path.join(GOLDEN, "table1.json")) as f:
        t = json.load(f)
    idx = {v: i for i, v in enumerate(t["vertices"])}

    def graph(edges):
        rows = [0] * 4
        for a, b in edges:
            rows[idx[a]] |= 1 << idx[b]
            rows[idx[b]] |= 1 << idx[a]
        return {"n": 4, "directed": False, "rows": rows, "label": None}

    return t, graph(t["G_edges"]), graph(t["H_edges"])


@pytest.mark.parametrize("tuning", [None, {"single_wave": 1, "children_per_wave": 1,
                                            "no_reprune": 1}])
def test_table1_pair(gpu, tuning):
    from paper_1908_06418_amd import solve_batch
    t, G, H = _table1_pair()
    print(f"table 1 pair, tuning {tuning}", flush=True)
    r, = solve_batch([(G, H)], time_limit_s=30, tuning=tuning)
    assert r.optimal and r.size == t["mcs_size"] == 4
    assert oracle.check.is_valid(G, H, r.mapping)
    if tuning:
        assert r.nodes == oracle.mcs(G, H)["nodes"]
