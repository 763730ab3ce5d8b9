"""Pins the oracle's node counting and its training-trace helpers to a second,
separately written implementation (the plain Python recursion of
_mcsplit_py, which shares no code with the C oracle) and to exhaustive
search.  CPU only."""
import numpy as np
import pytest
from _mcsplit_py import Counter, branch_cost, node, rank, root, select

import mcs_instances as mi
import oracle
from oracle import traces


def _pairs(seed, count, nmax=8, directed=False, nlab=0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        n1, n2 = int(rng.integers(1, nmax + 1)), int(rng.integers(1, nmax + 1))
        p = float(rng.uniform(0.1, 0.9))
        out.append((mi.random_small(rng, n1, p, directed, nlab),
                    mi.random_small(rng, n2, p, directed, nlab)))
    return out


@pytest.mark.parametrize("directed,nlab", [(False, 0), (True, 0), (False, 2), (True, 3)])
def test_oracle_node_count_matches_plain_recursion(directed, nlab):
    """The C oracle's node count (one per Solve entry) equals the Python
    recursion's on whole searches."""
    for G, H in _pairs(300 + 2 * directed + nlab, 60, 9, directed, nlab):
        r = oracle.mcs(G, H)
        c = Counter(G, H, 0)
        c.rec(root(G, H), 0)
        assert r["complete"]
        assert (r["size"], r["nodes"]) == (c.best, c.nodes), (G, H)


@pytest.mark.parametrize("directed,nlab", [(False, 0), (True, 0), (False, 2)])
def test_branch_cost_matches_plain_recursion(directed, nlab):
    """oracle.branch_cost(steps, u, incumbent) for every u of the selected
    class, at the root and at nodes one and two pairs deep, with the
    incumbent at the optimum, one below it and zero."""
    checked = 0
    for G, H in _pairs(410 + directed + nlab, 40, 8, directed, nlab):
        opt = oracle.mcs(G, H)
        if opt["size"] == 0:
            continue
        rg = rank(G)
        paths = [[]] + [opt["map"][:k] for k in (1, 2) if opt["size"] > k]
        for steps in paths:
            classes = node(G, H, steps)
            if not classes:
                continue
            L, _ = classes[select(classes, rg)]
            for inc in sorted({opt["size"], max(0, opt["size"] - 1), 0}):
                for u in sorted(L):
                    got = oracle.branch_cost(G, H, steps, u, inc)
                    assert got == branch_cost(G, H, steps, u, inc), (G, H, steps, u, inc)
                    checked += 1
    assert checked > 100


@pytest.mark.parametrize("directed,nlab", [(False, 0), (True, 2)])
def test_trace_class_choice_is_the_oracle_choice(directed, nlab):
    """traces.select_class picks the class the C oracle branches on: the C
    entry point accepts every vertex of that class as the branching vertex
    and rejects every vertex of the other classes."""
    rng = np.random.default_rng(500 + directed)
    checked = 0
    for G, H in _pairs(510 + directed, 50, 9, directed, nlab):
        opt = oracle.mcs(G, H)
        steps = []
        for _ in range(3):
            r = oracle.path(G, H, steps)
            if r is None or not r["classes"]:
                break
            classes = [(set(a), set(b)) for a, b in r["classes"]]
            sel = traces.select_class(classes, traces.degree_rank(G))
            assert sel == select([(frozenset(a), frozenset(b)) for a, b in classes], rank(G))
            for k, (L, _) in enumerate(classes):
                for u in sorted(L):
                    if k == sel:
                        oracle.branch_cost(G, H, steps, u, opt["size"], node_limit=1)
                    else:
                        with pytest.raises(ValueError):
                            oracle.branch_cost(G, H, steps, u, opt["size"], node_limit=1)
                    checked += 1
            L, R = classes[int(rng.integers(len(classes)))]
            steps = steps + [(sorted(L)[int(rng.integers(len(L)))],
                              sorted(R)[int(rng.integers(len(R)))])]
    assert checked > 200


def test_node_rows_labels_follow_an_optimal_mapping():
    """node_rows: one row per vertex of the selected class on each side; G
    rows are positive exactly for the vertices the optimal mapping uses, H
    rows exactly for their images, and the mapping is optimal by exhaustive
    search."""
    checked = 0
    for G, H in _pairs(600, 40, 8):
        o = oracle.mcs(G, H)
        if o["size"] < 2:
            continue
        assert o["size"] == oracle.brute.mcs_size(G, H)
        mstar = dict(o["map"])
        rk = traces.degree_rank(G)
        for steps in ([], o["map"][:1], o["map"][1:2]):
            X, y = traces.node_rows(G, H, steps, mstar, rk)
            classes = node(G, H, steps)
            if not classes:
                assert X == [] and y == []
                continue
            L, R = classes[select(classes, rank(G))]
            assert len(X) == len(y) == len(L) + len(R)
            gl, hl = y[:len(L)], y[len(L):]
            assert gl == [1.0 if u in mstar else 0.0 for u in sorted(L)]
            assert hl == [1.0 if w in {mstar[u] for u in L if u in mstar} else 0.0
                          for w in sorted(R)]
            # the optimum's pairs that start in the class end in it
            assert sum(gl) == sum(hl)
            checked += 1
    assert checked > 40


def test_value_rows_labels_by_exhaustive_search():
    """value_rows_at: partner w of v is positive iff some common induced
    subgraph of the optimal size contains the node's pairs and (v, w),
    decided by exhaustive search."""
    checked = 0
    for G, H in _pairs(700, 40, 7):
        o = oracle.mcs(G, H)
        if o["size"] < 2:
            continue
        rk = traces.degree_rank(G)
        for steps in ([], o["map"][:1]):
            X, y, kids = traces.value_rows_at(G, H, steps, o["size"], rk, 0)
            for row, kid in zip(y, kids):
                truth = oracle.brute.mcs_size_with(G, H, kid) >= o["size"]
                assert row == (1.0 if truth else 0.0), (G, H, kid)
                checked += 1
    assert checked > 60
