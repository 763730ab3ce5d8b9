"""ORACLE (test infrastructure only): the alternative vertex order of
Sec. IV.A ("graph sorting"), written from the paper's description in plain
Python.  The host library has its own implementation; the two are compared
through the search they induce (node counts of the one-wavefront search).

The paper's procedure on the adjacency matrix of one graph:

1. Connected components (weak components for directed graphs).  Each
   component is ordered on its own and the orders are concatenated; a
   component with a larger ratio of non-zero rows to non-zero columns comes
   first.
2. Within a component, in the manner of Hellerman and Rarick: the non-zero
   rows and columns form the active submatrix; repeatedly take the column
   that meets the most shortest rows of the active submatrix (a row's length
   is its number of active columns) and move it out of the active part, to
   the left of what remains.  The order is the sequence of columns taken.

Readings where the text is silent (they are listed in the design notes):
 - ratio ties: the larger component first, then the one holding the
   smallest vertex index; components without any arc (isolated vertices)
   come last, in index order;
 - column ties: the smallest vertex index;
 - "shortest rows" are the active rows of least non-zero length; a row whose
   active length reaches 0 leaves the active submatrix;
 - vertices never taken as a column (zero columns, or columns no active row
   meets once the rows are exhausted) follow the taken ones in index order.
"""
from __future__ import annotations


def _arc(g: dict, i: int, j: int) -> bool:
    return bool((g["rows"][i] >> j) & 1)


def components(g: dict) -> list:
    """Weak connected components, each a sorted list of vertices, in order of
    their smallest vertex."""
    n = g["n"]
    seen = [False] * n
    out = []
    for s in range(n):
        if seen[s]:
            continue
        comp, stack = [], [s]
        seen[s] = True
        while stack:
            u = stack.pop()
            comp.append(u)
            for x in range(n):
                if not seen[x] and (_arc(g, u, x) or _arc(g, x, u)):
                    seen[x] = True
                    stack.append(x)
        out.append(sorted(comp))
    return out


def order_component(g: dict, comp: list) -> list:
    rows = {r for r in comp if any(_arc(g, r, c) for c in comp)}
    cols = {c for c in comp if any(_arc(g, r, c) for r in comp)}
    taken = []
    while True:
        length = {r: sum(1 for c in cols if _arc(g, r, c)) for r in rows}
        rows = {r for r in rows if length[r] > 0}
        if not rows:
            break
        least = min(length[r] for r in rows)
        shortest = [r for r in rows if length[r] == least]
        best, best_hits = None, -1
        for c in sorted(cols):
            hits = sum(1 for r in shortest if _arc(g, r, c))
            if hits > best_hits:
                best, best_hits = c, hits
        taken.append(best)
        cols.discard(best)
    return taken + [v for v in comp if v not in taken]


def btf_order(g: dict) -> list:
    """Vertex order of one graph: order[k] = the vertex placed at position k."""
    keyed = []
    for comp in components(g):
        nz_rows = sum(1 for r in comp if any(_arc(g, r, c) for c in comp))
        nz_cols = sum(1 for c in comp if any(_arc(g, r, c) for r in comp))
        if nz_rows == 0:
            keyed.append(((1, 0.0, 0, comp[0]), comp))  # no arc: last
        else:
            keyed.append(((0, -nz_rows / nz_cols, -len(comp), comp[0]), comp))
    keyed.sort(key=lambda kc: kc[0])
    order = []
    for _, comp in keyed:
        order += order_component(g, comp)
    return order
