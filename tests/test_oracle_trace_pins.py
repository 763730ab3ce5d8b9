"""Pins the oracle's node counting and its training-trace helpers to a second,
separately written implementation: a plain Python recursion over vertex sets
that follows Algorithm 1 of the paper (Sec. II.B) with the readings the
oracle states -- prune when the Eq. 1 bound is at most the incumbent; the
class of smallest max(|L|, |R|), ties to the class holding the G vertex that
comes first in descending-degree order; v the first vertex of that class in
that order; partners w in descending-degree order of H; the "v unmatched"
child last; one node per entry of the recursion.  It shares no code with the
C oracle (lists and sets here, bidomain arrays there).  CPU only."""
import numpy as np
import pytest

import mcs_instances as mi
import oracle
from oracle import traces


def _adj(g, a, b):
    return (g["rows"][a] >> b) & 1


def _rank(g):
    """Position of each vertex in descending (total) degree order, ties kept
    in index order."""
    n = g["n"]
    deg = [sum(_adj(g, u, x) for x in range(n)) +
           (sum(_adj(g, x, u) for x in range(n)) if g["directed"] else 0) for u in range(n)]
    order = sorted(range(n), key=lambda u: (-deg[u], u))
    return {u: r for r, u in enumerate(order)}


def _letter(g, v, x):
    if g["directed"]:
        return (_adj(g, v, x), _adj(g, x, v))
    return _adj(g, v, x)


def _root(G, H):
    if G["n"] == 0 or H["n"] == 0:
        return []
    if G.get("label") is None:
        return [(frozenset(range(G["n"])), frozenset(range(H["n"])))]
    out = []
    for lab in sorted(set(G["label"]) & set(H["label"])):
        out.append((frozenset(u for u in range(G["n"]) if G["label"][u] == lab),
                    frozenset(w for w in range(H["n"]) if H["label"][w] == lab)))
    return out


def _split(G, H, classes, v, w):
    out = []
    for L, R in classes:
        parts = {}
        for x in L - {v}:
            parts.setdefault(_letter(G, v, x), [set(), set()])[0].add(x)
        for y in R - {w}:
            parts.setdefault(_letter(H, w, y), [set(), set()])[1].add(y)
        for a, b in parts.values():
            if a and b:
                out.append((frozenset(a), frozenset(b)))
    return out


def _drop(classes, v):
    out = []
    for L, R in classes:
        L2 = L - {v}
        if L2:
            out.append((L2, R))
    return out


def _bound(m, classes):
    return m + sum(min(len(L), len(R)) for L, R in classes)


def _select(classes, rg):
    return min(range(len(classes)),
               key=lambda k: (max(len(classes[k][0]), len(classes[k][1])),
                              min(rg[x] for x in classes[k][0])))


class _Counter:
    def __init__(self, G, H, best):
        self.G, self.H = G, H
        self.rg, self.rh = _rank(G), _rank(H)
        self.best = best
        self.nodes = 0

    def branch(self, classes, m, v, L, R):
        for w in sorted(R, key=lambda y: self.rh[y]):
            self.rec(_split(self.G, self.H, classes, v, w), m + 1)
        self.rec(_drop(classes, v), m)

    def rec(self, classes, m):
        self.nodes += 1
        if m > self.best:
            self.best = m
        if _bound(m, classes) <= self.best:
            return
        L, R = classes[_select(classes, self.rg)]
        v = min(L, key=lambda x: self.rg[x])
        self.branch(classes, m, v, L, R)


def _node(G, H, steps):
    classes = _root(G, H)
    for v, w in steps:
        assert any(v in L and w in R for L, R in classes)
        classes = _split(G, H, classes, v, w)
    return classes


def _branch_cost(G, H, steps, u, incumbent):
    """Nodes below (and including) the node reached by steps when it branches
    on u, the incumbent starting at `incumbent`."""
    c = _Counter(G, H, incumbent)
    classes = _node(G, H, steps)
    c.nodes = 1
    if _bound(len(steps), classes) > c.best:
        L, R = next((L, R) for L, R in classes if u in L)
        c.branch(classes, len(steps), u, L, R)
    return c.nodes


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
        c = _Counter(G, H, 0)
        c.rec(_root(G, H), 0)
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
        rg = _rank(G)
        paths = [[]] + [opt["map"][:k] for k in (1, 2) if opt["size"] > k]
        for steps in paths:
            classes = _node(G, H, steps)
            if not classes:
                continue
            L, _ = classes[_select(classes, rg)]
            for inc in sorted({opt["size"], max(0, opt["size"] - 1), 0}):
                for u in sorted(L):
                    got = oracle.branch_cost(G, H, steps, u, inc)
                    assert got == _branch_cost(G, H, steps, u, inc), (G, H, steps, u, inc)
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
            assert sel == _select([(frozenset(a), frozenset(b)) for a, b in classes], _rank(G))
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
        rank = traces.degree_rank(G)
        for steps in ([], o["map"][:1], o["map"][1:2]):
            X, y = traces.node_rows(G, H, steps, mstar, rank)
            classes = _node(G, H, steps)
            if not classes:
                assert X == [] and y == []
                continue
            L, R = classes[_select(classes, _rank(G))]
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
        rank = traces.degree_rank(G)
        for steps in ([], o["map"][:1]):
            X, y, kids = traces.value_rows_at(G, H, steps, o["size"], rank, 0)
            for row, kid in zip(y, kids):
                truth = oracle.brute.mcs_size_with(G, H, kid) >= o["size"]
                assert row == (1.0 if truth else 0.0), (G, H, kid)
                checked += 1
    assert checked > 60
