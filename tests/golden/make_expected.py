"""Writes the stored expected MCS sizes the GPU parity tests compare against.

Calls only the oracle (plain recursive McSplit, oracle/) on the seeded
workloads of mcs_instances.  A pair the oracle cannot finish within the node
limit is stored with complete = false and its size as a lower bound.

    python tests/golden/make_expected.py c2_n30 c3 c4_1024
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mcs_instances as mi  # noqa: E402
import oracle  # noqa: E402

SETS = {
    # name: (pairs factory, oracle node limit, description)
    "c2_n30": (lambda: mi.pairs_c2(ns=(30,)), 0,
               "undirected unlabelled G(30,p), p in {0.1,0.3,0.5}, seeds 0..19"),
    "c2_n35_p01": (lambda: mi.pairs_c2(ns=(35,), ps=(0.1,)), 200_000_000,
                   "undirected unlabelled G(35,0.1), seeds 0..19"),
    "c3": (lambda: mi.pairs_c3(), 0,
           "directed vertex-labelled n in {40,50,60}, p=0.1, ceil(0.33n) labels, seeds 0..19"),
    "c4_1024": (lambda: mi.pairs_c4(1024), 20_000_000,
                "batched workload, first 1024 pairs (n ~ U{10..35}, p ~ U[0.05,0.5))"),
    "c4": (lambda: mi.pairs_c4(4096), 20_000_000,
           "batched workload, all 4096 pairs (n ~ U{10..35}, p ~ U[0.05,0.5))"),
}


def _one(args):
    i, G, H, lim = args
    t = time.time()
    r = oracle.mcs(G, H, node_limit=lim)
    return i, r["size"], r["complete"], r["nodes"], time.time() - t


def _prefix_rows(pairs, lim):
    """Rows of another stored set whose pairs are a prefix of these, made
    with the same node limit (the same oracle runs: reused, not redone)."""
    best = []
    for other, (factory, olim, _) in SETS.items():
        path = os.path.join(HERE, f"expected_{other}.json")
        if olim != lim or not os.path.exists(path):
            continue
        with open(path) as f:
            data = json.load(f)
        k = len(data["pairs"])
        if k > len(best) and k <= len(pairs) and data["digest"] == mi.workload_hash(pairs[:k]):
            best = data["pairs"]
    return best


def make(name: str, workers: int = 8) -> str:
    factory, lim, desc = SETS[name]
    pairs = factory()
    oracle._load()
    rows = [None] * len(pairs)
    done = _prefix_rows(pairs, lim) if len(pairs) > 1 else []
    rows[:len(done)] = done
    with ProcessPoolExecutor(workers) as ex:
        for i, size, complete, nodes, dt in ex.map(
                _one, [(i, G, H, lim) for i, (G, H) in enumerate(pairs) if rows[i] is None]):
            rows[i] = {"size": size, "complete": complete, "nodes": nodes,
                       "seconds": round(dt, 4)}
    out = {"workload": name, "description": desc, "node_limit": lim,
           "digest": mi.workload_hash(pairs),
           "made_by": "tests/golden/make_expected.py (oracle only)",
           "pairs": rows}
    path = os.path.join(HERE, f"expected_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    return path


if __name__ == "__main__":
    workers = int(os.environ.get("MAKE_EXPECTED_WORKERS", "8"))
    for name in sys.argv[1:] or list(SETS):
        print(make(name, workers), flush=True)
