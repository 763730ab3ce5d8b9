"""ORACLE (test infrastructure only): MCS as the maximum clique of the modular
product graph (the Barrow-Burstall reduction cited in the paper's introduction;
the clique encoding of Sec. IV).

Product vertices are pairs (u, h) with equal labels.  (u, h) and (u', h') are
adjacent iff u != u', h != h' and both ordered pairs agree on adjacency:
A_G(u,u') = A_H(h,h') and A_G(u',u) = A_H(h',h).  A clique is exactly a valid
injective map, so the clique number is the MCS size.  The clique number is
found by Bron-Kerbosch with Tomita pivoting over Python-int bitsets.
"""
from __future__ import annotations


def product_graph(G: dict, H: dict):
    nG, nH = G["n"], H["n"]
    lg, lh = G.get("label"), H.get("label")
    verts = [(u, h) for u in range(nG) for h in range(nH)
             if lg is None or lg[u] == lh[h]]
    idx = {p: i for i, p in enumerate(verts)}

    def a(g, i, j):
        return (g["rows"][i] >> j) & 1

    nbr = [0] * len(verts)
    for i, (u, h) in enumerate(verts):
        for (u2, h2), j in idx.items():
            if u2 != u and h2 != h and a(G, u, u2) == a(H, h, h2) \
                    and a(G, u2, u) == a(H, h2, h):
                nbr[i] |= 1 << j
    return verts, nbr


def clique_number(nbr) -> int:
    best = 0

    def expand(size, P, X):
        nonlocal best
        if P == 0 and X == 0:
            best = max(best, size)
            return
        if size + bin(P).count("1") <= best:
            return
        # pivot: vertex of P | X with most neighbours in P
        PX = P | X
        piv, pc = -1, -1
        t = PX
        while t:
            low = t & -t
            v = low.bit_length() - 1
            c = bin(P & nbr[v]).count("1")
            if c > pc:
                piv, pc = v, c
            t ^= low
        cand = P & ~nbr[piv]
        while cand:
            low = cand & -cand
            v = low.bit_length() - 1
            expand(size + 1, P & nbr[v], X & nbr[v])
            P &= ~low
            X |= low
            cand ^= low

    expand(0, (1 << len(nbr)) - 1, 0)
    return best


def mcs_size(G: dict, H: dict) -> int:
    _, nbr = product_graph(G, H)
    return clique_number(nbr)


def omega(g: dict) -> int:
    """Clique number of an undirected graph (same routine)."""
    return clique_number(list(g["rows"]))
