"""A plain Python McSplit recursion over vertex sets, written apart from the
C oracle (lists and sets here, bidomain arrays there) and from the HIP path,
for tests that pin node counts and search orders: Algorithm 1 of the paper
(Sec. II.B) with the readings the oracle states -- prune when the Eq. 1
bound is at most the incumbent; the class of smallest max(|L|, |R|), ties
to the class holding the G vertex that comes first in descending-degree
order; v the first vertex of that class in that order; partners w in
descending-degree order of H; the "v unmatched" child last; one node per
entry of the recursion.  An optional scoring rule replaces the choice of v
and the order of the partners at shallow nodes, as the learned policy does
(best score first, ties to the earlier vertex in degree order)."""


def adj(g, a, b):
    return (g["rows"][a] >> b) & 1


def rank(g):
    """Position of each vertex in descending (total) degree order, ties kept
    in index order."""
    n = g["n"]
    deg = [sum(adj(g, u, x) for x in range(n)) +
           (sum(adj(g, x, u) for x in range(n)) if g["directed"] else 0) for u in range(n)]
    order = sorted(range(n), key=lambda u: (-deg[u], u))
    return {u: r for r, u in enumerate(order)}


def letter(g, v, x):
    if g["directed"]:
        return (adj(g, v, x), adj(g, x, v))
    return adj(g, v, x)


def root(G, H):
    if G["n"] == 0 or H["n"] == 0:
        return []
    if G.get("label") is None:
        return [(frozenset(range(G["n"])), frozenset(range(H["n"])))]
    out = []
    for lab in sorted(set(G["label"]) & set(H["label"])):
        out.append((frozenset(u for u in range(G["n"]) if G["label"][u] == lab),
                    frozenset(w for w in range(H["n"]) if H["label"][w] == lab)))
    return out


def split(G, H, classes, v, w):
    out = []
    for L, R in classes:
        parts = {}
        for x in L - {v}:
            parts.setdefault(letter(G, v, x), [set(), set()])[0].add(x)
        for y in R - {w}:
            parts.setdefault(letter(H, w, y), [set(), set()])[1].add(y)
        for a, b in parts.values():
            if a and b:
                out.append((frozenset(a), frozenset(b)))
    return out


def drop(classes, v):
    out = []
    for L, R in classes:
        L2 = L - {v}
        if L2:
            out.append((L2, R))
    return out


def bound(m, classes):
    return m + sum(min(len(L), len(R)) for L, R in classes)


def select(classes, rg):
    return min(range(len(classes)),
               key=lambda k: (max(len(classes[k][0]), len(classes[k][1])),
                              min(rg[x] for x in classes[k][0])))


class Counter:
    """Node counter of a search from a given node.  score(u, side, classes,
    sel, depth, candidates), if given, is used at nodes of depth <= depth_max:
    mode bit 0 -- v is the best-scored vertex of the selected class; bit 1 --
    the partners are tried best-scored first."""

    def __init__(self, G, H, best, score=None, depth_max=-1, mode=0):
        self.G, self.H = G, H
        self.rg, self.rh = rank(G), rank(H)
        self.best = best
        self.nodes = 0
        self.score, self.depth_max, self.mode = score, depth_max, mode

    def partners(self, classes, sel, m, R):
        order = sorted(R, key=lambda y: self.rh[y])
        if self.score is not None and m <= self.depth_max and self.mode & 2:
            cand = sorted(R)
            s = {y: self.score(y, 1, classes, sel, m, cand) for y in R}
            order = sorted(R, key=lambda y: (-s[y], self.rh[y]))
        return order

    def branch(self, classes, m, v, L, R, sel=None):
        if sel is None:
            sel = next(k for k, (a, _) in enumerate(classes) if v in a)
        for w in self.partners(classes, sel, m, R):
            self.rec(split(self.G, self.H, classes, v, w), m + 1)
        self.rec(drop(classes, v), m)

    def rec(self, classes, m):
        self.nodes += 1
        if m > self.best:
            self.best = m
        if bound(m, classes) <= self.best:
            return
        sel = select(classes, self.rg)
        L, R = classes[sel]
        if self.score is not None and m <= self.depth_max and self.mode & 1:
            cand = sorted(L)
            s = {u: self.score(u, 0, classes, sel, m, cand) for u in L}
            v = min(L, key=lambda x: (-s[x], self.rg[x]))
        else:
            v = min(L, key=lambda x: self.rg[x])
        self.branch(classes, m, v, L, R, sel)


def node(G, H, steps):
    classes = root(G, H)
    for v, w in steps:
        assert any(v in L and w in R for L, R in classes)
        classes = split(G, H, classes, v, w)
    return classes


def branch_cost(G, H, steps, u, incumbent):
    """Nodes below (and including) the node reached by steps when it branches
    on u, the incumbent starting at `incumbent`."""
    c = Counter(G, H, incumbent)
    classes = node(G, H, steps)
    c.nodes = 1
    if bound(len(steps), classes) > c.best:
        L, R = next((L, R) for L, R in classes if u in L)
        c.branch(classes, len(steps), u, L, R)
    return c.nodes


