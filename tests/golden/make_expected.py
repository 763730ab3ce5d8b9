"""Writes the stored expected MCS sizes the GPU parity tests compare against.

Calls only the oracle (plain recursive McSplit, oracle/) on the seeded
workloads of mcs_instances.  A pair the oracle cannot finish within the node
limit is stored with complete = false and its size as a lower bound.

    python tests/golden/make_expected.py c2_n30 c3 c4_1024
    python tests/golden/make_expected.py --deepen c2 1.5e9

The second form reruns a stored set's unfinished pairs under a larger node
limit (1.5e9 nodes is about 600 s of one core for this oracle).
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, as_completed

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mcs_instances as mi  # noqa: E402
import oracle  # noqa: E402

def _c2_limit(G, H):
    # G(30,p) pairs all finish (at most about 1.2e8 nodes); larger ones get a budget
    return 0 if G["n"] <= 30 else 100_000_000


SETS = {
    # name: (pairs factory, oracle node limit (an int, or a function of the
    # pair), description)
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
    "w": (lambda: mi.pairs_w(), 0,
          "directed vertex-labelled n in {80,100}, p=0.1, ceil(0.33n) labels, seeds 0..19"),
    "c2": (lambda: mi.pairs_c2(), _c2_limit,
           "undirected unlabelled G(n,p), n in {30,35,40}, p in {0.1,0.3,0.5}, seeds 0..19 "
           "(node limit: none for n = 30, 1e8 otherwise)"),
}


def _limit(lim, G, H):
    return lim(G, H) if callable(lim) else lim


def _one(args):
    i, G, H, lim = args
    t = time.time()
    r = oracle.mcs(G, H, node_limit=lim)
    return i, r["size"], r["complete"], r["nodes"], time.time() - t


def _known_rows(pairs, lim):
    """Rows other stored sets already hold for identical pairs, where the
    oracle run under this set's limit would give the same row: a finished
    run within the limit, or an unfinished one under the same limit (the
    oracle is deterministic, so these are reused, not redone)."""
    want = {}
    for i, (G, H) in enumerate(pairs):
        want.setdefault(mi.workload_hash([(G, H)]), []).append(i)
    rows = [None] * len(pairs)
    for other, (factory, olim, _) in SETS.items():
        path = os.path.join(HERE, f"expected_{other}.json")
        if not os.path.exists(path):
            continue
        with open(path) as f:
            data = json.load(f)
        opairs = factory()
        if data["digest"] != mi.workload_hash(opairs):
            continue
        for (G, H), row in zip(opairs, data["pairs"]):
            for i in want.get(mi.workload_hash([(G, H)]), []):
                mine = _limit(lim, *pairs[i])
                theirs = row.get("node_limit", _limit(olim, G, H))
                same = (row["complete"] and (mine == 0 or row["nodes"] <= mine)) or \
                       (not row["complete"] and theirs == mine)
                if same and rows[i] is None:
                    rows[i] = row
    return rows


def make(name: str, workers: int = 8) -> str:
    factory, lim, desc = SETS[name]
    pairs = factory()
    oracle._load()
    rows = [None] * len(pairs)
    rows = _known_rows(pairs, lim)
    with ProcessPoolExecutor(workers) as ex:
        for i, size, complete, nodes, dt in ex.map(
                _one, [(i, G, H, _limit(lim, G, H)) for i, (G, H) in enumerate(pairs)
                       if rows[i] is None]):
            rows[i] = {"size": size, "complete": complete, "nodes": nodes,
                       "seconds": round(dt, 4)}
    out = {"workload": name, "description": desc,
           "node_limit": lim if not callable(lim) else [_limit(lim, G, H) for G, H in pairs],
           "digest": mi.workload_hash(pairs),
           "made_by": "tests/golden/make_expected.py (oracle only)",
           "pairs": rows}
    path = os.path.join(HERE, f"expected_{name}.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=0)
    return path


def _row_limit(data, i):
    """The node limit row i of a stored set was computed under."""
    row = data["pairs"][i]
    if "node_limit" in row:
        return row["node_limit"]
    lim = data["node_limit"]
    return lim[i] if isinstance(lim, list) else lim


def _write(path, data):
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=0)
    os.replace(tmp, path)


def deepen(name: str, limit: int, workers: int = 8) -> str:
    """Rerun, under the larger node limit ``limit``, every row of a stored set
    the oracle did not finish.  Rows are taken smallest graph first (the ones
    most likely to finish) and the file is rewritten after each result, so an
    interrupted run keeps what it finished; each row records the limit it was
    computed under."""
    factory, _, _ = SETS[name]
    pairs = factory()
    path = os.path.join(HERE, f"expected_{name}.json")
    with open(path) as f:
        data = json.load(f)
    if data["digest"] != mi.workload_hash(pairs):
        raise SystemExit(f"{path} does not belong to the current {name} pairs")
    for i in range(len(pairs)):
        data["pairs"][i]["node_limit"] = _row_limit(data, i)
    todo = [i for i, r in enumerate(data["pairs"])
            if not r["complete"] and 0 < r["node_limit"] < limit]
    todo.sort(key=lambda i: (pairs[i][0]["n"] + pairs[i][1]["n"], i))
    oracle._load()
    done = 0
    with ProcessPoolExecutor(workers) as ex:
        futs = [ex.submit(_one, (i, pairs[i][0], pairs[i][1], limit)) for i in todo]
        for fut in as_completed(futs):
            i, size, complete, nodes, dt = fut.result()
            old = data["pairs"][i]
            if size < old["size"]:
                raise SystemExit(f"pair {i}: size {size} below the stored bound {old['size']}")
            data["pairs"][i] = {"size": size, "complete": complete, "nodes": nodes,
                                "seconds": round(dt, 4), "node_limit": limit}
            done += 1
            _write(path, data)
            print(f"{name} pair {i}: size {size} complete {complete} "
                  f"nodes {nodes} {dt:.1f}s ({done}/{len(todo)})", flush=True)
    return path


if __name__ == "__main__":
    workers = int(os.environ.get("MAKE_EXPECTED_WORKERS", "8"))
    args = sys.argv[1:]
    if args[:1] == ["--deepen"]:
        # --deepen NAME LIMIT: rerun a stored set's unfinished rows under LIMIT nodes
        print(deepen(args[1], int(float(args[2])), workers), flush=True)
    else:
        for name in args or list(SETS):
            print(make(name, workers), flush=True)
