"""ORACLE (test infrastructure only): McSplit's labels and classes computed
from their definition (paper Sec. II.B and Table 1), not incrementally.

Given a mapping M = [(g_1, h_1), ...] (in mapping order) and a set of G vertices
removed by "v unmatched" steps, the label of an unmatched vertex x of G is the
sequence of its adjacency letters to g_1, g_2, ... (undirected: 1 adjacent,
0 not; directed: the pair (arc g_i -> x, arc x -> g_i)), preceded by its vertex
label when the graphs are labelled; likewise for H against h_1, h_2, ...
A class is the set of vertices sharing a label; classes whose label occurs on
one side only can never be matched and add 0 to Eq. 1.
"""
from __future__ import annotations


def _adj(g, i, j):
    return (g["rows"][i] >> j) & 1


def label_of(g: dict, x: int, mapped: list):
    lab = [] if g.get("label") is None else [("vertex", g["label"][x])]
    for m in mapped:
        if g["directed"]:
            lab.append((_adj(g, m, x), _adj(g, x, m)))
        else:
            lab.append(_adj(g, m, x))
    return tuple(lab)


def label_strings(G: dict, H: dict, M: list, removed=()):
    """{vertex: label} for the unmatched vertices of G and of H."""
    mg = [p[0] for p in M]
    mh = [p[1] for p in M]
    lg = {x: label_of(G, x, mg) for x in range(G["n"]) if x not in mg and x not in removed}
    lh = {y: label_of(H, y, mh) for y in range(H["n"]) if y not in mh}
    return lg, lh


def classes(G: dict, H: dict, M: list, removed=()):
    """List of (frozenset_G, frozenset_H) for labels present on both sides."""
    lg, lh = label_strings(G, H, M, removed)
    out = []
    for lab in sorted(set(lg.values()) & set(lh.values()), key=repr):
        out.append((frozenset(x for x, l in lg.items() if l == lab),
                    frozenset(y for y, l in lh.items() if l == lab)))
    return out


def bound(G: dict, H: dict, M: list, removed=()) -> int:
    """Eq. 1: |M| + sum over labels of min(#G vertices, #H vertices)."""
    lg, lh = label_strings(G, H, M, removed)
    b = len(M)
    for lab in set(lg.values()) | set(lh.values()):
        b += min(sum(1 for l in lg.values() if l == lab),
                 sum(1 for l in lh.values() if l == lab))
    return b
