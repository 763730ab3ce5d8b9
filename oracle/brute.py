"""ORACLE (test infrastructure only): MCS by exhaustive search over injective
partial maps -- the definition of the maximum common induced subgraph
(paper Sec. II.A), usable for graphs of up to about 8 vertices.

Vertices of G are taken in index order; each is either left unmapped or mapped
to an unused vertex of H that keeps every ordered pair of mapped vertices
agreeing on adjacency (and, when labelled, has the same label).  Consistency is
hereditary, so dropping inconsistent prefixes loses no valid map.  The only
other cut is the trivial one: stop when even mapping every remaining vertex of
G could not beat the best size found.
"""
from __future__ import annotations


def _matrix(g):
    n = g["n"]
    return [[(g["rows"][i] >> j) & 1 for j in range(n)] for i in range(n)]


def mcs_size(G: dict, H: dict) -> int:
    A, B = _matrix(G), _matrix(H)
    nG, nH = G["n"], H["n"]
    lg, lh = G.get("label"), H.get("label")
    f = [-1] * nG
    used = [False] * nH
    best = 0

    def consistent(u, h):
        if lg is not None and lg[u] != lh[h]:
            return False
        for x in range(u):
            y = f[x]
            if y >= 0 and (A[u][x] != B[h][y] or A[x][u] != B[y][h]):
                return False
        return True

    def rec(u, size):
        nonlocal best
        if size > best:
            best = size
        if u == nG or size + (nG - u) <= best:
            return
        for h in range(nH):
            if not used[h] and consistent(u, h):
                f[u], used[h] = h, True
                rec(u + 1, size + 1)
                f[u], used[h] = -1, False
        rec(u + 1, size)

    rec(0, 0)
    return best


def mcs_size_with(G: dict, H: dict, forced) -> int:
    """Largest valid injective map that contains the pairs in forced (which
    must themselves be consistent), by the same exhaustive enumeration."""
    A, B = _matrix(G), _matrix(H)
    nG, nH = G["n"], H["n"]
    lg, lh = G.get("label"), H.get("label")
    fixed = dict(forced)
    f = [-1] * nG
    used = [False] * nH
    for u, h in fixed.items():
        f[u], used[h] = h, True
    best = 0

    def ok(u, h):
        if lg is not None and lg[u] != lh[h]:
            return False
        for x in range(nG):
            y = f[x]
            if x != u and y >= 0 and (A[u][x] != B[h][y] or A[x][u] != B[y][h]):
                return False
        return True

    for u, h in fixed.items():
        f[u] = -1
        if not ok(u, h):
            return -1
        f[u] = h

    def rec(u, size):
        nonlocal best
        if u == nG:
            best = max(best, size)
            return
        if size + (nG - u) <= best:
            return
        if u in fixed:
            rec(u + 1, size + 1)
            return
        for h in range(nH):
            if not used[h] and ok(u, h):
                f[u], used[h] = h, True
                rec(u + 1, size + 1)
                f[u], used[h] = -1, False
        rec(u + 1, size)

    rec(0, 0)
    return best
