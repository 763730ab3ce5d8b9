"""ORACLE (test infrastructure only): training rows for the branching policy,
generated from oracle solutions.

For a training pair the oracle finds an optimal mapping M*.  Search nodes are
rebuilt by replaying the C oracle's class split along prefixes of M* (the
root, then random subsets of M*'s pairs of size 1 and 2, in the order the
search maps them).  At each node the class the search would select (smallest
max(|L|,|R|), ties to the smallest vertex in descending-degree order) gives
the candidates:
  - G side, every u in L: label 1 iff M* maps u;
  - H side, every w in R: label 1 iff M* maps some vertex of L to w.
Features follow oracle.policy.features.  These targets teach the policy to
branch first on what an optimum uses; the search stays exact whatever the
network says.
"""
from __future__ import annotations

import numpy as np

from . import extend, mcs, path, policy


def degree_rank(g: dict) -> dict:
    n = g["n"]
    deg = []
    for u in range(n):
        dg = bin(g["rows"][u]).count("1")
        if g["directed"]:
            dg += sum((g["rows"][j] >> u) & 1 for j in range(n))
        deg.append(dg)
    order = sorted(range(n), key=lambda u: -deg[u])  # stable: ties by index
    return {u: r for r, u in enumerate(order)}


def select_class(classes, rank_g: dict) -> int:
    return min(range(len(classes)),
               key=lambda k: (max(len(classes[k][0]), len(classes[k][1])),
                              min(rank_g[x] for x in classes[k][0])))


def node_rows(G, H, steps, mstar: dict, rank_g: dict):
    r = path(G, H, steps)
    if r is None or not r["classes"]:
        return [], []
    classes = [(set(a), set(b)) for a, b in r["classes"]]
    sel = select_class(classes, rank_g)
    L, R = classes[sel]
    d = len(steps)
    X, y = [], []
    for u in sorted(L):
        X.append(policy.features(G, u, 0, classes, sel, d, candidates=sorted(L)))
        y.append(1.0 if u in mstar else 0.0)
    used = {mstar[u] for u in L if u in mstar}
    for w in sorted(R):
        X.append(policy.features(H, w, 1, classes, sel, d, candidates=sorted(R)))
        y.append(1.0 if w in used else 0.0)
    return X, y


def pair_rows(G, H, rng: np.random.Generator, node_limit: int = 2_000_000,
              per_depth: int = 3):
    """Rows of one pair, or ([], []) if the oracle does not finish."""
    o = mcs(G, H, node_limit=node_limit)
    if not o["complete"] or o["size"] == 0:
        return [], []
    mstar = dict(o["map"])
    rank_g = degree_rank(G)
    X, y = node_rows(G, H, [], mstar, rank_g)
    pairs = list(o["map"])
    for k in (1, 2):
        for _ in range(per_depth):
            if len(pairs) < k:
                break
            idx = rng.choice(len(pairs), size=k, replace=False)
            steps = [pairs[i] for i in sorted(idx)]
            Xa, ya = node_rows(G, H, steps, mstar, rank_g)
            X += Xa
            y += ya
    return X, y


def dataset(pairs, seed: int = 0, node_limit: int = 2_000_000):
    rng = np.random.default_rng(seed)
    X, y = [], []
    for G, H in pairs:
        Xa, ya = pair_rows(G, H, rng, node_limit)
        X += Xa
        y += ya
    return np.array(X, dtype=np.float64).reshape(-1, policy.F), np.array(y, dtype=np.float64)


# ---- value-ordering rows ------------------------------------------------------
# The search's own nodes near the root: the root and each child (v0, w) of it,
# v0 being the vertex the default rule branches on (smallest vertex in
# descending-degree order of the selected class).  At each node, for every
# partner w of that node's v: label 1 iff a common induced subgraph of the
# optimal size still contains the node's pairs and (v, w) (oracle.extend).


def _node(G, H, steps, rank_g):
    r = path(G, H, steps)
    if r is None or not r["classes"]:
        return None
    classes = [(set(a), set(b)) for a, b in r["classes"]]
    sel = select_class(classes, rank_g)
    v = min(classes[sel][0], key=lambda x: rank_g[x])
    return classes, sel, v


def value_rows_at(G, H, steps, sstar, rank_g, node_limit):
    nd = _node(G, H, steps, rank_g)
    if nd is None:
        return [], [], []
    classes, sel, v = nd
    L, R = classes[sel]
    X, y, kids = [], [], []
    for w in sorted(R):
        ok = extend(G, H, steps + [(v, w)], sstar, node_limit)
        if ok is None:
            continue
        X.append(policy.features(H, w, 1, classes, sel, len(steps), candidates=sorted(R)))
        y.append(1.0 if ok else 0.0)
        kids.append(steps + [(v, w)])
    return X, y, kids


def value_pair_rows(G, H, node_limit: int = 2_000_000, depth: int = 1):
    """Value-ordering rows of one pair at the root and, for depth >= 1, at
    every child of the root; ([], []) if the oracle does not finish."""
    o = mcs(G, H, node_limit=node_limit)
    if not o["complete"] or o["size"] == 0:
        return [], []
    rank_g = degree_rank(G)
    X, y, kids = value_rows_at(G, H, [], o["size"], rank_g, node_limit)
    frontier = kids
    for _ in range(depth):
        nxt = []
        for steps in frontier:
            Xa, ya, ka = value_rows_at(G, H, steps, o["size"], rank_g, node_limit)
            if any(ya) and not all(ya):  # nodes where the order can matter
                X += Xa
                y += ya
            nxt += ka
        frontier = nxt
    return X, y


# ---- branching-vertex rows ---------------------------------------------------
# At the root and at the root's children (default branching), every vertex u
# of the selected class is a candidate for v.  Its label is the proof cost of
# branching on it relative to the best candidate: min_cost / cost(u) (1 for
# the cheapest), with the incumbent fixed at the optimum (oracle.branch_cost).


def branch_rows_at(G, H, steps, sstar, rank_g, node_limit):
    from . import branch_cost
    nd = _node(G, H, steps, rank_g)
    if nd is None:
        return [], [], []
    classes, sel, v0 = nd
    L, R = classes[sel]
    kids = [steps + [(v0, w)] for w in sorted(R)]
    if len(L) < 2:
        return [], [], kids
    cost = {}
    for u in sorted(L):
        c = branch_cost(G, H, steps, u, sstar, node_limit)
        if c is None:
            return [], [], kids
        cost[u] = c
    best = min(cost.values())
    X = [policy.features(G, u, 0, classes, sel, len(steps), candidates=sorted(L))
         for u in sorted(L)]
    y = [best / cost[u] for u in sorted(L)]
    return X, y, kids


def branch_pair_rows(G, H, node_limit: int = 2_000_000, depth: int = 1):
    """Branching-vertex rows at the root and (depth >= 1) its children."""
    o = mcs(G, H, node_limit=node_limit)
    if not o["complete"] or o["size"] == 0:
        return [], []
    rank_g = degree_rank(G)
    X, y, kids = branch_rows_at(G, H, [], o["size"], rank_g, node_limit)
    for _ in range(depth):
        nxt = []
        for steps in kids:
            Xa, ya, ka = branch_rows_at(G, H, steps, o["size"], rank_g, node_limit)
            X += Xa
            y += ya
            nxt += ka
        kids = nxt
    return X, y
