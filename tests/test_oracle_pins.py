"""Pins the oracle to facts other than itself: the paper's worked example
(Table 1, Eq. 1), the definition by exhaustive search, the modular-product
clique reduction, closed forms and invariants.  CPU only."""
import itertools
import json
import os

import numpy as np
import pytest

import mcs_instances as mi
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _table1():
    with open(os.path.join(GOLDEN, "table1.json")) as f:
        t = json.load(f)
    idx = {v: i for i, v in enumerate(t["vertices"])}

    def graph(edges):
        rows = [0] * 4
        for a, b in edges:
            rows[idx[a]] |= 1 << idx[b]
            rows[idx[b]] |= 1 << idx[a]
        return {"n": 4, "directed": False, "rows": rows, "label": None}

    return t, idx, graph(t["G_edges"]), graph(t["H_edges"])


def test_table1_labels_from_definition():
    """Table 1 (a)-(c): labels of the unmatched vertices along a->b, b->c, c->a."""
    t, idx, G, H = _table1()
    name = {i: v for v, i in idx.items()}
    M = []
    for step, (g, h) in enumerate(t["path"]):
        M.append((idx[g], idx[h]))
        lg, lh = oracle.labels.label_strings(G, H, M)
        got_g = {name[x]: "".join(str(b) for b in lab) for x, lab in lg.items()}
        got_h = {name[y]: "".join(str(b) for b in lab) for y, lab in lh.items()}
        assert got_g == t["labels"][step]["G"]
        assert got_h == t["labels"][step]["H"]


def _named(classes, idx):
    name = {i: v for v, i in idx.items()}
    return sorted((sorted(name[x] for x in L), sorted(name[y] for y in R)) for L, R in classes)


def test_table1_oracle_split_and_bounds():
    """The C oracle's filterDomain reproduces Table 1's classes and Eq. 1 bounds."""
    t, idx, G, H = _table1()
    for k in range(len(t["path"]) + 1):
        steps = [(idx[g], idx[h]) for g, h in t["path"][:k]]
        r = oracle.path(G, H, steps)
        assert r is not None
        assert r["bounds"] == t["bounds"][:k + 1]
        if k > 0:
            exp = sorted((sorted(L), sorted(R)) for L, R in t["classes"][k - 1])
            assert _named(r["classes"], idx) == exp


def test_table1_definition_bounds():
    t, idx, G, H = _table1()
    M = []
    bs = [oracle.labels.bound(G, H, M)]
    for g, h in t["path"]:
        M.append((idx[g], idx[h]))
        bs.append(oracle.labels.bound(G, H, M))
    assert bs == t["bounds"]


def test_table1_mcs():
    t, idx, G, H = _table1()
    r = oracle.mcs(G, H)
    assert r["size"] == t["mcs_size"] == oracle.brute.mcs_size(G, H)
    assert oracle.check.is_valid(G, H, r["map"])


def test_path_rejects_label_mismatch():
    t, idx, G, H = _table1()
    steps = [(idx[g], idx[h]) for g, h in t["path"]] + [(idx["d"], idx["d"])]
    assert oracle.path(G, H, steps) is None


@pytest.mark.parametrize("directed,nlab", [(False, 0), (True, 0), (False, 3), (True, 2)])
def test_incremental_split_matches_label_definition(directed, nlab):
    """Along random paths, the oracle's incremental classes equal the classes
    of the label strings computed from their definition."""
    rng = np.random.default_rng(7 + 3 * directed + nlab)
    for trial in range(40):
        n = int(rng.integers(2, 9))
        G = mi.random_small(rng, n, float(rng.uniform(0.1, 0.9)), directed, nlab)
        H = mi.random_small(rng, int(rng.integers(2, 9)), float(rng.uniform(0.1, 0.9)),
                            directed, nlab)
        steps, M, removed = [], [], set()
        for _ in range(6):
            cl = oracle.labels.classes(G, H, M, removed)
            if not cl:
                break
            L, R = cl[int(rng.integers(len(cl)))]
            v = sorted(L)[int(rng.integers(len(L)))]
            if rng.random() < 0.25:
                steps.append((v, None))
                removed.add(v)
            else:
                w = sorted(R)[int(rng.integers(len(R)))]
                steps.append((v, w))
                M.append((v, w))
            r = oracle.path(G, H, steps)
            assert r is not None
            exp = oracle.labels.classes(G, H, M, removed)
            assert sorted((sorted(a), sorted(b)) for a, b in r["classes"]) == \
                sorted((sorted(a), sorted(b)) for a, b in exp)
            assert r["bounds"][-1] == oracle.labels.bound(G, H, M, removed)


@pytest.mark.parametrize("directed,nlab", [(False, 0), (True, 0), (False, 2), (True, 3)])
def test_oracle_vs_brute_force(directed, nlab):
    """Exact size on random pairs with n <= 8 against the definition."""
    rng = np.random.default_rng(100 + 2 * directed + nlab)
    count = 0
    for trial in range(150):
        nG = int(rng.integers(0, 8))
        nH = int(rng.integers(0, 8))
        G = mi.random_small(rng, nG, float(rng.uniform(0, 1)), directed, nlab)
        H = mi.random_small(rng, nH, float(rng.uniform(0, 1)), directed, nlab)
        r = oracle.mcs(G, H)
        assert r["complete"]
        assert r["size"] == oracle.brute.mcs_size(G, H), (G, H)
        assert oracle.check.is_valid(G, H, r["map"])
        assert len(r["map"]) == r["size"]
        assert r["root_bound"] >= r["size"]
        count += 1
    assert count == 150


def test_oracle_vs_brute_force_n8():
    rng = np.random.default_rng(5)
    for trial in range(12):
        p = float(rng.uniform(0.2, 0.8))
        G = mi.random_small(rng, 8, p)
        H = mi.random_small(rng, 8, p)
        assert oracle.mcs(G, H)["size"] == oracle.brute.mcs_size(G, H)


@pytest.mark.parametrize("directed,nlab", [(False, 0), (True, 0), (False, 3)])
def test_oracle_vs_modular_product_clique(directed, nlab):
    """MCS = clique number of the modular product graph (n up to 10)."""
    rng = np.random.default_rng(300 + directed + nlab)
    for trial in range(8):
        n = int(rng.integers(6, 11))
        p = float(rng.uniform(0.2, 0.7))
        G = mi.random_small(rng, n, p, directed, nlab)
        H = mi.random_small(rng, int(rng.integers(6, 11)), p, directed, nlab)
        assert oracle.mcs(G, H)["size"] == oracle.clique.mcs_size(G, H)


def test_closed_forms():
    rng = np.random.default_rng(11)
    for n in range(0, 12):
        G = mi.random_small(rng, n, 0.4)
        assert oracle.mcs(G, G)["size"] == n
        perm = list(rng.permutation(n))
        assert oracle.mcs(G, mi.permute(G, perm))["size"] == n
        S = sorted(rng.choice(n, size=n // 2, replace=False).tolist()) if n else []
        assert oracle.mcs(G, mi.induced(G, S))["size"] == len(S)
    for a in range(0, 7):
        for b in range(0, 7):
            assert oracle.mcs(mi.empty_graph(a), mi.empty_graph(b))["size"] == min(a, b)
            assert oracle.mcs(mi.complete_graph(a), mi.complete_graph(b))["size"] == min(a, b)
            assert oracle.mcs(mi.complete_graph(a), mi.empty_graph(b))["size"] == min(1, a, b)
    for trial in range(10):
        H = mi.random_small(rng, 9, 0.5)
        w = oracle.clique.omega(H)
        a = oracle.clique.omega(mi.complement(H))
        for n in (1, 3, 5, 9):
            assert oracle.mcs(mi.complete_graph(n), H)["size"] == min(n, w)
            assert oracle.mcs(mi.empty_graph(n), H)["size"] == min(n, a)


def test_invariants_random():
    rng = np.random.default_rng(21)
    for trial in range(25):
        directed = bool(trial % 2)
        n1, n2 = int(rng.integers(5, 14)), int(rng.integers(5, 14))
        p = float(rng.uniform(0.15, 0.6))
        G = mi.random_small(rng, n1, p, directed)
        H = mi.random_small(rng, n2, p, directed)
        s = oracle.mcs(G, H)["size"]
        assert oracle.mcs(H, G)["size"] == s                                 # symmetry
        assert oracle.mcs(mi.complement(G), mi.complement(H))["size"] == s   # complement
        assert oracle.mcs(mi.permute(G, list(rng.permutation(n1))),
                          mi.permute(H, list(rng.permutation(n2))))["size"] == s
        labG = dict(G, label=[int(x) for x in rng.integers(0, 2, n1)])
        labH = dict(H, label=[int(x) for x in rng.integers(0, 2, n2)])
        assert oracle.mcs(labG, labH)["size"] <= s                           # labels only restrict
        if directed:
            und = lambda g: mi.from_matrix(np.maximum(mi.to_matrix(g), mi.to_matrix(g).T), False)
            # each arc pattern determines the undirected one, so this can only grow
            assert oracle.mcs(und(G), und(H))["size"] >= s


def test_workload_c1_oracle():
    (G, H), = mi.pair_c1()
    r = oracle.mcs(G, H)
    assert r["complete"] and oracle.check.is_valid(G, H, r["map"])
    assert r["size"] == 11


def test_node_limit_reports_incomplete():
    (G, H), = mi.pair_c1()
    r = oracle.mcs(G, H, node_limit=50)
    assert not r["complete"] and r["nodes"] >= 50
    assert oracle.check.is_valid(G, H, r["map"])


def test_check_mapping_rejects():
    (G, H), = mi.pair_c1()
    good = oracle.mcs(G, H)["map"]
    assert oracle.check.is_valid(G, H, good)
    bad = list(good)
    bad[0] = (bad[0][0], bad[1][1])
    assert not oracle.check.is_valid(G, H, bad)
    assert not oracle.check.is_valid(G, H, good + [(good[0][0], 15)])
    assert not oracle.check.is_valid(G, H, [(99, 0)])


@pytest.mark.parametrize("plant", [1, 2, 3, 4])
def test_planted_oracle_mistakes_are_caught(plant, tmp_path):
    """Each deliberately wrong build of the C oracle (a dropped Eq. 1 term, a
    transposed or wrong-index adjacency operand, a missing branch) disagrees
    with the exhaustive definition on some small pair."""
    import ctypes
    lib = oracle._bind(ctypes.CDLL(oracle.build_planted(plant, str(tmp_path / f"p{plant}.so"))))
    rng = np.random.default_rng(40 + plant)
    directed = plant == 2
    wrong = 0
    for trial in range(60):
        G = mi.random_small(rng, int(rng.integers(3, 8)), float(rng.uniform(0.2, 0.8)), directed)
        H = mi.random_small(rng, int(rng.integers(3, 8)), float(rng.uniform(0.2, 0.8)), directed)
        if oracle.mcs(G, H, lib=lib)["size"] != oracle.brute.mcs_size(G, H):
            wrong += 1
    assert wrong > 0


@pytest.mark.parametrize("directed", [False, True])
def test_extend_matches_forced_brute_force(directed):
    """oracle.extend(path, target) == (largest valid map containing the path
    has at least target pairs), the latter by exhaustive search."""
    rng = np.random.default_rng(60 + directed)
    checked = 0
    for trial in range(80):
        n1, n2 = int(rng.integers(3, 8)), int(rng.integers(3, 8))
        p = float(rng.uniform(0.2, 0.8))
        G = mi.random_small(rng, n1, p, directed)
        H = mi.random_small(rng, n2, p, directed)
        best = oracle.mcs(G, H)
        k = int(rng.integers(0, min(3, best["size"]) + 1))
        # a legal path: k pairs of some valid map (the oracle's, or random)
        pairs = best["map"][:k]
        if rng.random() < 0.5 and k:
            # replace the last pair by a random label-compatible one
            steps = pairs[:-1]
            r = oracle.path(G, H, steps)
            cand = [(v, w) for L, R in r["classes"] for v in L for w in R]
            if cand:
                pairs = steps + [cand[int(rng.integers(len(cand)))]]
        truth = oracle.brute.mcs_size_with(G, H, pairs)
        for target in range(0, best["size"] + 2):
            assert oracle.extend(G, H, pairs, target) == (truth >= target), (pairs, target)
            checked += 1
    assert checked > 200
