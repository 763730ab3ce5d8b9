"""ORACLE (test infrastructure only): the learned branching policy's reference
arithmetic in float64 numpy -- features of a candidate vertex at a search
node, the 16 -> 64 -> 64 -> 1 ReLU network, its binary cross-entropy loss and
the gradients by the chain rule.  The GPU kernels (forward, backward, update,
and the in-search scorer) are checked against these.

The paper has no learned component; the policy only reorders which vertex is
branched on and in which order its partners are tried, so it cannot change
any answer (every child is still explored or soundly pruned by Eq. 1).

Features of candidate u (16 values, all in [0, 1] or exactly 1):
   0  degree of u in its own graph / n            (total degree if directed)
   1  |L| / n of the selected class
   2  |R| / n of the selected class
   3  |M| / n
   4  number of classes / n
   5  neighbours of u among its side's vertices in classes / n
 6-11 neighbours of u on its side in classes whose min(|L|,|R|) is
      1, 2, 3-4, 5-8, 9-16, >= 17   (each / n)
  12  side: 0 for a G candidate (choice of v), 1 for an H candidate (order of w)
  13  1 if u's degree is the largest among the candidates on its side, else 0
  14  0
  15  1 (bias input)
n is the vertex count of u's graph; "neighbour" uses out- or in-arcs.
"""
from __future__ import annotations

import numpy as np

F, H1, H2 = 16, 64, 64


def bucket(m: int) -> int:
    """Size bucket of a class by min(|L|, |R|): 1, 2, 3-4, 5-8, 9-16, >= 17."""
    if m <= 1:
        return 0
    if m == 2:
        return 1
    if m <= 4:
        return 2
    if m <= 8:
        return 3
    if m <= 16:
        return 4
    return 5


def _nbrs(g, u):
    s = set()
    for j in range(g["n"]):
        if (g["rows"][u] >> j) & 1 or (g["rows"][j] >> u) & 1:
            s.add(j)
    return s


def features(g: dict, u: int, side: int, classes, sel: int, depth: int,
             candidates) -> np.ndarray:
    """classes: list of (set_G, set_H); sel: index of the selected class;
    side 0: u in G (uses set_G of each class), 1: u in H."""
    n = g["n"]
    x = np.zeros(F)
    nb = _nbrs(g, u)
    deg = {c: len(_nbrs(g, c)) for c in candidates}
    x[0] = deg[u] / n
    x[1] = len(classes[sel][0]) / n
    x[2] = len(classes[sel][1]) / n
    x[3] = depth / n
    x[4] = len(classes) / n
    tot = 0
    for L, R in classes:
        mine = L if side == 0 else R
        k = len(nb & set(mine))
        tot += k
        x[6 + bucket(min(len(L), len(R)))] += k / n
    x[5] = tot / n
    x[12] = float(side)
    x[13] = 1.0 if deg[u] == max(deg.values()) else 0.0
    x[15] = 1.0
    return x


def init_params(seed: int = 0) -> dict:
    rng = np.random.default_rng(seed)
    return {"W1": rng.normal(0, np.sqrt(2.0 / F), (H1, F)), "b1": np.zeros(H1),
            "W2": rng.normal(0, np.sqrt(2.0 / H1), (H2, H1)), "b2": np.zeros(H2),
            "w3": rng.normal(0, np.sqrt(1.0 / H2), H2), "b3": np.zeros(1)}


def forward(p: dict, X: np.ndarray):
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["w3"] + p["b3"][0]
    return z, (X, a1, h1, a2, h2)


def bce_loss(z: np.ndarray, y: np.ndarray) -> float:
    """Mean binary cross-entropy of sigmoid(z) against y, in a stable form."""
    return float(np.mean(np.maximum(z, 0) - z * y + np.log1p(np.exp(-np.abs(z)))))


def loss_and_grads(p: dict, X: np.ndarray, y: np.ndarray):
    z, (X, a1, h1, a2, h2) = forward(p, X)
    B = X.shape[0]
    dz = (1.0 / (1.0 + np.exp(-z)) - y) / B
    g = {"w3": h2.T @ dz, "b3": np.array([dz.sum()])}
    dh2 = np.outer(dz, p["w3"]) * (a2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(0)
    dh1 = (dh2 @ p["W2"]) * (a1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(0)
    return bce_loss(z, y), g


def sgd(p: dict, g: dict, lr: float) -> dict:
    return {k: p[k] - lr * g[k] for k in p}


def flat(p: dict) -> np.ndarray:
    """Parameters in the packed order the GPU uses: W1, b1, W2, b2, w3, b3."""
    return np.concatenate([p["W1"].ravel(), p["b1"], p["W2"].ravel(), p["b2"],
                           p["w3"], p["b3"]])


def unflat(v: np.ndarray) -> dict:
    v = np.asarray(v, dtype=np.float64)
    o = 0
    out = {}
    for k, shape in (("W1", (H1, F)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)),
                     ("w3", (H2,)), ("b3", (1,))):
        size = int(np.prod(shape))
        out[k] = v[o:o + size].reshape(shape)
        o += size
    return out


N_PARAMS = H1 * F + H1 + H2 * H1 + H2 + H2 + 1
