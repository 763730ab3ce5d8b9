"""Pins the policy's float64 reference (oracle/policy.py): gradients against
central finite differences, closed forms, and hand-computed features."""
import math

import numpy as np

import mcs_instances as mi
from oracle import policy


def _data(seed, B=37):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0, 1, (B, policy.F))
    X[:, 15] = 1.0
    y = (rng.uniform(0, 1, B) < 0.3).astype(float)
    return X, y


def test_gradients_match_finite_differences():
    p = policy.init_params(1)
    X, y = _data(2)
    loss, g = policy.loss_and_grads(p, X, y)
    v = policy.flat(p)
    gv = policy.flat(g)
    rng = np.random.default_rng(3)
    idx = rng.choice(v.size, 80, replace=False)
    h = 1e-6
    for i in idx:
        vp = v.copy()
        vm = v.copy()
        vp[i] += h
        vm[i] -= h
        lp = policy.loss_and_grads(policy.unflat(vp), X, y)[0]
        lm = policy.loss_and_grads(policy.unflat(vm), X, y)[0]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gv[i]) <= 1e-6 + 1e-5 * abs(fd), (i, fd, gv[i])


def test_zero_network_closed_form():
    p = {k: np.zeros_like(v) for k, v in policy.init_params(0).items()}
    p["b3"] = np.array([0.7])
    X, y = _data(4)
    loss, g = policy.loss_and_grads(p, X, y)
    s = 1 / (1 + math.exp(-0.7))
    assert abs(loss - np.mean(-(y * math.log(s) + (1 - y) * math.log(1 - s)))) < 1e-12
    assert abs(g["b3"][0] - np.mean(s - y)) < 1e-12
    for k in ("W1", "b1", "W2", "b2", "w3"):
        assert not np.any(g[k])


def test_loss_is_stable_for_large_logits():
    z = np.array([800.0, -800.0, 0.0])
    y = np.array([1.0, 0.0, 1.0])
    assert abs(policy.bce_loss(z, y) - math.log(2) / 3) < 1e-12


def test_flat_round_trip():
    p = policy.init_params(5)
    v = policy.flat(p)
    assert v.size == policy.N_PARAMS == 5313
    q = policy.unflat(v)
    assert all(np.array_equal(p[k], q[k]) for k in p)


def test_features_by_hand():
    # path graph 0-1-2-3 plus isolated 4 (G side)
    rows = [0b00010, 0b00101, 0b01010, 0b00100, 0]
    g = {"n": 5, "directed": False, "rows": rows, "label": None}
    classes = [({1, 2}, {0, 1, 2}), ({3, 4}, {3})]
    x = policy.features(g, 2, 0, classes, 0, 1, candidates=[1, 2])
    assert x[0] == 2 / 5                        # deg(2) = 2
    assert x[1] == 2 / 5 and x[2] == 3 / 5      # selected class sizes
    assert x[3] == 1 / 5 and x[4] == 2 / 5      # depth, class count
    # neighbours of 2 on the G side in classes: 1 (class 0), 3 (class 1)
    assert x[5] == 2 / 5
    assert x[6 + policy.bucket(2)] == 1 / 5     # class 0: min(2,3) = 2
    assert x[6 + policy.bucket(1)] == 1 / 5     # class 1: min(2,1) = 1
    assert x[12] == 0 and x[15] == 1
    assert x[13] == 1.0                         # deg 2 is the max among {1, 2}
