"""The alternative vertex order of Sec. IV.A (connected components, then a
bordered block-triangular order in the manner of Hellerman and Rarick), as
the oracle implements it (oracle/ordering.py): orders worked out by hand from
the paper's rules, and properties that any order must keep."""
import numpy as np
import pytest

import mcs_instances as mi
import oracle
from oracle.ordering import btf_order, components


def _graph(n, arcs, directed=False):
    rows = [0] * n
    for i, j in arcs:
        rows[i] |= 1 << j
        if not directed:
            rows[j] |= 1 << i
    return {"n": n, "directed": directed, "rows": rows, "label": None}


def test_path_by_hand():
    # P4 0-1-2-3: shortest rows {0, 3} are met once by columns 1 and 2 (tie:
    # 1); then rows {2, 3} by columns 3 and 2 (tie: 2); then rows {1, 2} by
    # columns 0 and 3 (tie: 0); then column 3.
    assert btf_order(_graph(4, [(0, 1), (1, 2), (2, 3)])) == [1, 2, 0, 3]


def test_star_by_hand():
    # the centre meets all three shortest rows (the leaves) and goes first;
    # then the centre's row is the only one left and its columns follow
    assert btf_order(_graph(4, [(0, 1), (0, 2), (0, 3)])) == [0, 1, 2, 3]


def test_components_by_hand():
    # edge {0, 5}, triangle {1, 2, 3}, isolated 4: equal ratios (1), so the
    # larger component first; the vertex without arcs last
    g = _graph(6, [(0, 5), (1, 2), (2, 3), (1, 3)])
    assert [sorted(c) for c in components(g)] == [[0, 5], [1, 2, 3], [4]]
    assert btf_order(g) == [1, 2, 3, 0, 5, 4]


def test_directed_ratio_by_hand():
    # A = {0 -> 1, 0 -> 2}: 1 non-zero row over 2 non-zero columns (0.5);
    # B = {3 -> 5, 4 -> 5}: 2 over 1 (2.0), so B first.  In B column 5 meets
    # both shortest rows; 3 and 4 are never columns and follow in index
    # order.  In A the one row is met by columns 1 then 2; 0 follows.
    g = _graph(6, [(0, 1), (0, 2), (3, 5), (4, 5)], directed=True)
    assert btf_order(g) == [5, 3, 4, 1, 2, 0]


@pytest.mark.parametrize("directed", [False, True])
def test_order_is_a_permutation_with_contiguous_components(directed):
    rng = np.random.default_rng(3)
    for _ in range(30):
        n = int(rng.integers(0, 20))
        g = mi.random_small(rng, n, float(rng.uniform(0.02, 0.4)), directed, 0)
        order = btf_order(g)
        assert sorted(order) == list(range(n))
        comp_of = {v: k for k, c in enumerate(components(g)) for v in c}
        seen = []
        for v in order:
            if not seen or seen[-1] != comp_of[v]:
                assert comp_of[v] not in seen  # each component is one block
                seen.append(comp_of[v])


@pytest.mark.parametrize("directed,nlab", [(False, 0), (True, 0), (False, 3), (True, 2)])
def test_order_does_not_change_sizes(directed, nlab):
    rng = np.random.default_rng(11)
    for _ in range(25):
        G = mi.random_small(rng, int(rng.integers(5, 13)), 0.35, directed, nlab)
        H = mi.random_small(rng, int(rng.integers(5, 13)), 0.35, directed, nlab)
        a = oracle.mcs(G, H)
        b = oracle.mcs(G, H, order="btf")
        assert a["size"] == b["size"]
        assert oracle.check.is_valid(G, H, b["map"])
