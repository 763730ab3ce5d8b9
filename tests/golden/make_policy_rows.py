"""Writes the stored training rows of the learned branching policy.

Calls only the oracle (oracle/traces.py on oracle/mcsplit_oracle.c) on the
training pairs of the learned-ordering workload (mcs_instances.pairs_c5 with
train=True: n ~ U{20..30}, p alternating 0.2 / 0.4).  For each pair the
oracle proves within its node budget:
  - branching-vertex rows at the root (and, for n <= 22, at the root's
    children): every vertex of the selected class, labelled by the proof
    cost of branching on it relative to the cheapest (oracle.branch_cost);
  - partner-order rows at the root and its children: every partner w of v,
    labelled by whether an optimum still contains the node's pairs and
    (v, w) (oracle.extend).
Pairs the oracle does not finish are skipped and counted.  Rows are appended
pair by pair, so an interrupted run keeps what it finished.

    python tests/golden/make_policy_rows.py [pairs] [seconds] [workers]
"""
from __future__ import annotations

import json
import os
import sys
import time
from concurrent.futures import ProcessPoolExecutor, as_completed

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import mcs_instances as mi  # noqa: E402
import oracle  # noqa: E402
from oracle import traces  # noqa: E402

OUT = os.path.join(HERE, "policy_rows_c5_train.npz")
NODE_LIMIT = 20_000_000


def _rows(i):
    G, H = mi.pairs_c5(1, start=i, train=True)[0]
    t = time.time()
    o = oracle.mcs(G, H, node_limit=NODE_LIMIT)
    if not o["complete"]:
        return i, G["n"], None, None, time.time() - t
    depth = 1 if G["n"] <= 22 else 0
    Xb, yb = traces.branch_pair_rows(G, H, node_limit=NODE_LIMIT, depth=depth)
    Xv, yv = traces.value_pair_rows(G, H, node_limit=NODE_LIMIT, depth=1)
    return i, G["n"], Xb + Xv, yb + yv, time.time() - t


def _save(X, y, n, pair, done, skipped):
    tmp = OUT + ".tmp.npz"
    np.savez_compressed(tmp, X=np.array(X, dtype=np.float16).reshape(-1, 16),
                        y=np.array(y, dtype=np.float32), n=np.array(n, dtype=np.int8),
                        pair=np.array(pair, dtype=np.int16),
                        meta=np.array(json.dumps({
                            "made_by": "tests/golden/make_policy_rows.py (oracle only)",
                            "workload": "pairs_c5(train=True): n ~ U{20..30}, p 0.2 / 0.4",
                            "node_limit": NODE_LIMIT, "pairs_done": sorted(done),
                            "pairs_skipped": sorted(skipped)})))
    os.replace(tmp, OUT)


def main():
    count = int(sys.argv[1]) if len(sys.argv) > 1 else 400
    budget = float(sys.argv[2]) if len(sys.argv) > 2 else 3600.0
    workers = int(sys.argv[3]) if len(sys.argv) > 3 else 4
    oracle._load()
    X, y, n, pair, done, skipped = [], [], [], [], [], []
    t0 = time.time()
    with ProcessPoolExecutor(workers) as ex:
        futs = [ex.submit(_rows, i) for i in range(count)]
        for fut in as_completed(futs):
            i, ni, Xa, ya, dt = fut.result()
            if Xa is None:
                skipped.append(i)
            else:
                done.append(i)
                X += Xa
                y += ya
                n += [ni] * len(ya)
                pair += [i] * len(ya)
                _save(X, y, n, pair, done, skipped)
            print(f"pair {i} n={ni}: {'skipped' if Xa is None else len(ya)} rows, {dt:.1f}s "
                  f"({len(done)} done, {len(skipped)} skipped, {len(y)} rows)", flush=True)
            if time.time() - t0 > budget:
                for f in futs:
                    f.cancel()
                break
    _save(X, y, n, pair, done, skipped)
    print(OUT, flush=True)


if __name__ == "__main__":
    main()
