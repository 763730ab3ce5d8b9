"""Seeded synthetic graph pairs for the maximum common induced subgraph search.

This module is shared by the tests, the benchmark and the oracle's callers.  It
holds no part of the search itself: it only draws random graphs.

Random numbers come from splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014): state += 0x9E3779B97F4A7C15, then
the output is the state passed through the published 64-bit mixer.  The k-th
output of a stream (k = 0, 1, ...) is therefore mix(seed + (k + 1) * gamma), so
a whole stream is computed at once with numpy's wrapping uint64 arithmetic.
A uniform double in [0, 1) is (z >> 11) * 2**-53.

The paper evaluates on the ARG database (Sec. V.A: bounded-valence and mesh
graphs, treated as undirected and unlabelled).  That database is not available
here; the Erdos-Renyi workloads below stand in for it and cover the same size
bands (fewer than 40 vertices, and 40 to 50 vertices).

Stream seed of graph g of pair i of workload c: (c << 40) | (i << 2) | g, with
g = 0 for G, 1 for H and 2 for the per-pair size/density draws.

A graph is a dict {"n", "directed", "rows", "label"}: ``rows`` is a list of n
Python ints, bit j of rows[i] set iff the arc i -> j exists (symmetric when
undirected, no diagonal bits); ``label`` is None or a list of n ints.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """First ``count`` outputs of the splitmix64 stream that starts at ``seed``."""
    k = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + k * GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniforms(seed: int, count: int) -> np.ndarray:
    """``count`` doubles in [0, 1) from the stream at ``seed``."""
    return (splitmix64(seed, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def stream_seed(workload: int, pair: int, g: int) -> int:
    return (workload << 40) | (pair << 2) | g


def label_count(n: int) -> int:
    """ceil(0.33 n) label values, computed in integers (n=40 -> 14, 50 -> 17, 60 -> 20)."""
    return (33 * n + 99) // 100


def er_graph(n: int, p: float, seed: int, directed: bool = False,
             labelled: bool = False) -> dict:
    """G(n, p): undirected draws one uniform per pair i<j in row-major order;
    directed draws one per ordered pair i != j in row-major order (independent
    i->j and j->i).  Labels, if asked for, use the next n uniforms of the same
    stream: floor(u * ceil(0.33 n))."""
    if directed:
        pairs = [(i, j) for i in range(n) for j in range(n) if i != j]
    else:
        pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
    u = uniforms(seed, len(pairs) + (n if labelled else 0))
    rows = [0] * n
    for k, (i, j) in enumerate(pairs):
        if u[k] < p:
            rows[i] |= 1 << j
            if not directed:
                rows[j] |= 1 << i
    label = None
    if labelled:
        nl = label_count(n)
        label = [int(x * nl) for x in u[len(pairs):]]
    return {"n": n, "directed": bool(directed), "rows": rows, "label": label}


# ---------------------------------------------------------------------------
# The five workloads
# ---------------------------------------------------------------------------

def pair_c1() -> list:
    """One undirected unlabelled pair G(16, 0.3), H(16, 0.3)."""
    return [(er_graph(16, 0.3, stream_seed(1, 0, 0)),
             er_graph(16, 0.3, stream_seed(1, 0, 1)))]


C2_N = (30, 35, 40)
C2_P = (0.1, 0.3, 0.5)


def pairs_c2(ns=C2_N, ps=C2_P, seeds=range(20)) -> list:
    """Undirected unlabelled pairs, n in {30,35,40} x p in {0.1,0.3,0.5} x
    20 seeds; pair index ((n_idx * 3) + p_idx) * 20 + seed."""
    out = []
    for ni, n in enumerate(C2_N):
        if n not in ns:
            continue
        for pi, p in enumerate(C2_P):
            if p not in ps:
                continue
            for s in seeds:
                i = (ni * len(C2_P) + pi) * 20 + s
                out.append((er_graph(n, p, stream_seed(2, i, 0)),
                            er_graph(n, p, stream_seed(2, i, 1))))
    return out


C3_N = (40, 50, 60)


def pairs_c3(ns=C3_N, seeds=range(20)) -> list:
    """Directed vertex-labelled pairs, n in {40,50,60}, p = 0.1, labels over
    ceil(0.33 n) values, 20 seeds each; pair index n_idx * 20 + seed."""
    out = []
    for ni, n in enumerate(C3_N):
        if n not in ns:
            continue
        for s in seeds:
            i = ni * 20 + s
            out.append((er_graph(n, 0.1, stream_seed(3, i, 0), True, True),
                        er_graph(n, 0.1, stream_seed(3, i, 1), True, True)))
    return out


W_N = (80, 100)


def pairs_w(ns=W_N, seeds=range(20)) -> list:
    """The directed vertex-labelled recipe at 80 and 100 vertices (p = 0.1,
    labels over ceil(0.33 n) values, 20 seeds each): graphs beyond 64
    vertices; pair index n_idx * 20 + seed of workload 7."""
    out = []
    for ni, n in enumerate(W_N):
        if n not in ns:
            continue
        for s in seeds:
            i = ni * 20 + s
            out.append((er_graph(n, 0.1, stream_seed(7, i, 0), True, True),
                        er_graph(n, 0.1, stream_seed(7, i, 1), True, True)))
    return out


def c4_shape(i: int) -> tuple:
    u = uniforms(stream_seed(4, i, 2), 2)
    return 10 + int(u[0] * 26), 0.05 + float(u[1]) * 0.45


def pairs_c4(count: int = 4096, start: int = 0) -> list:
    """Batched workload: per pair n ~ U{10..35}, p ~ U[0.05, 0.5), shared by
    G and H of the pair."""
    out = []
    for i in range(start, start + count):
        n, p = c4_shape(i)
        out.append((er_graph(n, p, stream_seed(4, i, 0)),
                    er_graph(n, p, stream_seed(4, i, 1))))
    return out


def c5_shape(i: int, train: bool = False) -> tuple:
    """Learned-ordering workload: evaluation pairs n ~ U{35..50}, p = 0.2 for
    the first 512 and 0.4 for the rest; training pairs (workload id 6)
    n ~ U{20..30} with p alternating 0.2 / 0.4."""
    u = uniforms(stream_seed(6 if train else 5, i, 2), 1)
    if train:
        return 20 + int(u[0] * 11), (0.2 if i % 2 == 0 else 0.4)
    return 35 + int(u[0] * 16), (0.2 if i < 512 else 0.4)


def pairs_c5(count: int = 1024, start: int = 0, train: bool = False) -> list:
    wl = 6 if train else 5
    out = []
    for i in range(start, start + count):
        n, p = c5_shape(i, train)
        out.append((er_graph(n, p, stream_seed(wl, i, 0)),
                    er_graph(n, p, stream_seed(wl, i, 1))))
    return out


# ---------------------------------------------------------------------------
# Small helpers for tests (graph surgery, not search)
# ---------------------------------------------------------------------------

def to_matrix(g: dict) -> np.ndarray:
    n = g["n"]
    a = np.zeros((n, n), dtype=np.uint8)
    for i, r in enumerate(g["rows"]):
        for j in range(n):
            if (r >> j) & 1:
                a[i, j] = 1
    return a


def from_matrix(a, directed: bool, label=None) -> dict:
    a = np.asarray(a)
    n = a.shape[0]
    rows = [0] * n
    for i in range(n):
        for j in range(n):
            if a[i, j] and i != j:
                rows[i] |= 1 << j
    return {"n": n, "directed": bool(directed), "rows": rows,
            "label": None if label is None else [int(x) for x in label]}


def permute(g: dict, perm) -> dict:
    """Relabel vertex i as perm[i]."""
    n = g["n"]
    a = to_matrix(g)
    b = np.zeros_like(a)
    for i in range(n):
        for j in range(n):
            b[perm[i], perm[j]] = a[i, j]
    lab = None
    if g["label"] is not None:
        lab = [0] * n
        for i in range(n):
            lab[perm[i]] = g["label"][i]
    return from_matrix(b, g["directed"], lab)


def complement(g: dict) -> dict:
    n = g["n"]
    a = 1 - to_matrix(g)
    np.fill_diagonal(a, 0)
    return from_matrix(a, g["directed"], g["label"])


def induced(g: dict, verts) -> dict:
    a = to_matrix(g)[np.ix_(verts, verts)]
    lab = None if g["label"] is None else [g["label"][v] for v in verts]
    return from_matrix(a, g["directed"], lab)


def empty_graph(n: int) -> dict:
    return {"n": n, "directed": False, "rows": [0] * n, "label": None}


def complete_graph(n: int) -> dict:
    full = (1 << n) - 1
    return {"n": n, "directed": False,
            "rows": [full & ~(1 << i) for i in range(n)], "label": None}


def random_small(rng: np.random.Generator, n: int, p: float, directed=False,
                 nlabels=0) -> dict:
    """Ad-hoc small graph for property tests (numpy Generator, not splitmix)."""
    if directed:
        a = (rng.random((n, n)) < p).astype(np.uint8)
    else:
        t = np.triu((rng.random((n, n)) < p).astype(np.uint8), 1)
        a = t + t.T
    np.fill_diagonal(a, 0)
    lab = None if nlabels <= 0 else list(rng.integers(0, nlabels, n))
    return from_matrix(a, directed, lab)


def rows_u64(g: dict) -> np.ndarray:
    return np.array(g["rows"], dtype=np.uint64)


def workload_hash(pairs) -> str:
    """Short digest of a list of pairs, to name stored expected values."""
    import hashlib
    h = hashlib.sha256()
    for G, H in pairs:
        for g in (G, H):
            h.update(repr((g["n"], g["directed"], g["rows"], g["label"])).encode())
    return h.hexdigest()[:16]


__all__ = [n for n in dir() if not n.startswith("_")]
