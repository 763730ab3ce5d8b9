"""Pins of the oracle on graphs of 65..254 vertices, the range the 128- and
256-bit search kernels cover (the oracle works on dense byte matrices, so nothing in
it changes at 64; these check it there against closed forms and invariants,
as the small-graph pins do below 12 vertices)."""
import numpy as np

import mcs_instances as mi
import oracle


def test_closed_forms_beyond_64():
    for a in (65, 100, 128):
        for b in (1, 64, 65, 128):
            assert oracle.mcs(mi.empty_graph(a), mi.empty_graph(b))["size"] == min(a, b)
            assert oracle.mcs(mi.complete_graph(a), mi.complete_graph(b))["size"] == min(a, b)
            assert oracle.mcs(mi.complete_graph(a), mi.empty_graph(b))["size"] == 1


def test_relabelled_copy_and_induced_subgraph_beyond_64():
    """MCS(G, pi G) = n and MCS(G, G[S]) = |S| on random graphs of 70..128
    vertices, undirected and directed, and the mapping is valid."""
    rng = np.random.default_rng(101)
    g70 = mi.random_small(rng, 70, 0.3)
    cases = [(g70, mi.permute(g70, list(rng.permutation(70))), 70)]
    # the two relabelled 128-vertex copies of the 128-bit kernel's GPU batch
    # (draws whose copies the degree order aligns quickly; a relabelled copy
    # of a dense graph with many equal degrees can take millions of nodes)
    from test_gpu_wide import _wide_batch
    wide = _wide_batch()
    cases += [(wide[9][0], wide[9][1], 128), (wide[10][0], wide[10][1], 128)]
    g100 = mi.random_small(np.random.default_rng(41), 100, 0.2)
    for S in (list(range(0, 100, 25)), [0, 1, 2, 97, 98, 99], [64, 65, 66]):
        cases.append((g100, mi.induced(g100, S), len(S)))
    for G, H, want in cases:
        r = oracle.mcs(G, H, node_limit=5_000_000)
        assert r["complete"] and r["size"] == want, (G["n"], H["n"], r["size"], want)
        assert oracle.check.is_valid(G, H, r["map"])


def test_invariants_beyond_64():
    """Symmetry and relabelling leave the size unchanged, and refining the
    labels can only shrink it, on directed labelled pairs of 66..80 vertices
    (the directed labelled workload's recipe)."""
    rng = np.random.default_rng(7)
    for trial in range(3):
        n1, n2 = int(rng.integers(66, 81)), int(rng.integers(66, 81))
        G = mi.er_graph(n1, 0.1, 1000 + 2 * trial, True, True)
        H = mi.er_graph(n2, 0.1, 1001 + 2 * trial, True, True)
        r = oracle.mcs(G, H, node_limit=5_000_000)
        assert r["complete"]
        s = r["size"]
        assert oracle.check.is_valid(G, H, r["map"])
        assert oracle.mcs(H, G)["size"] == s
        assert oracle.mcs(mi.permute(G, list(rng.permutation(n1))),
                          mi.permute(H, list(rng.permutation(n2))))["size"] == s
        fine = lambda g: dict(g, label=[2 * l + (v % 2) for v, l in enumerate(g["label"])])
        assert oracle.mcs(fine(G), fine(H))["size"] <= s


def test_w_stored_sizes_are_the_oracles():
    """tests/golden/expected_w.json belongs to mcs_instances.pairs_w() and
    holds the oracle's sizes (re-derived here for the pairs it proves
    fastest)."""
    import json
    import os
    pairs = mi.pairs_w()
    with open(os.path.join(os.path.dirname(__file__), "golden", "expected_w.json")) as f:
        exp = json.load(f)
    assert exp["digest"] == mi.workload_hash(pairs)
    rows = sorted(range(len(pairs)), key=lambda i: exp["pairs"][i]["nodes"])[:4]
    for i in rows:
        G, H = pairs[i]
        r = oracle.mcs(G, H)
        assert r["complete"] and r["size"] == exp["pairs"][i]["size"]
        assert oracle.check.is_valid(G, H, r["map"])


def test_closed_forms_to_254():
    """The range of the 256-bit search kernel: empty and complete pairs give
    min(a, b), and K_a against E_b gives 1."""
    for a in (129, 192, 193, 254):
        for b in (1, 128, 200, 254):
            assert oracle.mcs(mi.empty_graph(a), mi.empty_graph(b))["size"] == min(a, b)
            assert oracle.mcs(mi.complete_graph(a), mi.complete_graph(b))["size"] == min(a, b)
            assert oracle.mcs(mi.complete_graph(a), mi.empty_graph(b))["size"] == 1


def test_relabelled_copy_and_induced_subgraph_to_254():
    """MCS(G, pi G) = n at 150, 200 and 254 vertices (undirected and
    directed), and MCS(G, G[S]) = |S| for vertex sets that straddle the
    64-bit word boundaries; every mapping is valid."""
    cases = []
    for seed, n, p, directed in ((100, 254, 0.5, False), (100, 254, 0.3, True),
                                 (100, 200, 0.3, False), (100, 150, 0.5, False)):
        rng = np.random.default_rng(seed)
        g = mi.random_small(rng, n, p, directed)
        cases.append((g, mi.permute(g, list(rng.permutation(n))), n))
    g200 = mi.random_small(np.random.default_rng(88), 200, 0.1)
    for S in ([0, 63, 64, 127, 128, 191, 192, 199], list(range(120, 200, 9))):
        cases.append((g200, mi.induced(g200, S), len(S)))
    for G, H, want in cases:
        r = oracle.mcs(G, H, node_limit=5_000_000)
        assert r["complete"] and r["size"] == want, (G["n"], H["n"], r["size"], want)
        assert oracle.check.is_valid(G, H, r["map"])


def test_labelled_invariants_to_254():
    """Swapping G and H, and relabelling both, leave the size of labelled
    pairs of 160..254 vertices unchanged (roots of 130..250 classes)."""
    for seed, n, p, directed, nlab in ((81, 180, 0.3, True, 130), (82, 254, 0.3, True, 250),
                                       (83, 160, 0.5, False, 140)):
        rng = np.random.default_rng(seed)
        g = mi.random_small(rng, n, p, directed)
        h = mi.random_small(rng, n, p, directed)
        g["label"] = [i % nlab for i in range(n)]
        h["label"] = [int(x) % nlab for x in rng.permutation(n)]
        r = oracle.mcs(g, h, node_limit=5_000_000)
        assert r["complete"] and oracle.check.is_valid(g, h, r["map"])
        assert oracle.mcs(h, g, node_limit=5_000_000)["size"] == r["size"]
        assert oracle.mcs(mi.permute(g, list(rng.permutation(n))),
                          mi.permute(h, list(rng.permutation(n))),
                          node_limit=5_000_000)["size"] == r["size"]
