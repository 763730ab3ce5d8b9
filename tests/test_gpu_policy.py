"""GPU tests of the learned branching policy: forward and gradient kernels
against the float64 reference (oracle/policy.py), training, exactness of the
search with the policy on, and what the trained policy gains."""
import json
import os

import numpy as np
import pytest
from _report import write_report

import mcs_instances as mi
import oracle
from oracle import policy as ref

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


def _half(a):
    return np.asarray(a, dtype=np.float16).astype(np.float64)


def _data(seed, rows):
    rng = np.random.default_rng(seed)
    X = _half(rng.uniform(0, 1, (rows, ref.F)))
    X[:, 15] = 1.0
    y = (rng.uniform(0, 1, rows) < 0.4).astype(np.float64)
    return X, y


def test_forward_matches_reference(gpu):
    import torch
    from paper_1908_06418_amd.policy import Policy
    P = Policy(seed=3)
    v = _half(P.numpy())
    X, _ = _data(1, 1000)
    got = P.forward(torch.from_numpy(X.astype(np.float16)).cuda()).cpu().numpy()
    want, _ = ref.forward(ref.unflat(v), X)
    assert np.allclose(got, want, rtol=1e-4, atol=1e-4), np.abs(got - want).max()


def test_gradients_match_reference(gpu):
    """fp32 accumulation over half-rounded weights and inputs against float64
    on the same rounded values: relative error well under 1e-4."""
    import torch
    from paper_1908_06418_amd.policy import Policy
    P = Policy(seed=4)
    v = _half(P.numpy())
    for rows in (1, 63, 64, 1000):
        X, y = _data(rows, rows)
        loss, g = P.grad(torch.from_numpy(X.astype(np.float16)).cuda(),
                         torch.from_numpy(y.astype(np.float32)).cuda())
        wl, wg = ref.loss_and_grads(ref.unflat(v), X, y)
        gv = g.cpu().numpy().astype(np.float64)
        ref_flat = ref.flat(wg)
        scale = np.abs(ref_flat).max()
        assert np.abs(gv - ref_flat).max() <= 1e-4 * scale + 1e-7, rows
        assert abs(float(loss.item()) - wl) <= 1e-4 * max(1.0, wl)


def test_sgd_and_pack(gpu):
    import torch
    from paper_1908_06418_amd.policy import Policy
    P = Policy(seed=5)
    before = P.numpy()
    X, y = _data(7, 256)
    loss, g = P.grad(torch.from_numpy(X.astype(np.float16)).cuda(),
                     torch.from_numpy(y.astype(np.float32)).cuda())
    P.sgd(g, 0.1)
    after = P.numpy()
    assert np.allclose(after, before - 0.1 * g.cpu().numpy(), atol=1e-6)
    P.pack()
    assert np.array_equal(P.half_params.cpu().numpy(), after.astype(np.float16))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _training_set():
    """Rows from the learned-ordering workload's training pairs (n ~ U{20..30},
    p 0.2 / 0.4), stored by tests/golden/make_policy_rows.py from the oracle
    alone: branching-vertex rows (proof-cost labels) and partner-order rows
    (reachability labels)."""
    d = np.load(os.path.join(GOLDEN, "policy_rows_c5_train.npz"))
    return (d["X"].astype(np.float64), d["y"].astype(np.float64),
            np.bincount(d["n"].astype(np.int64), minlength=31)[20:31].tolist())


_TRAINED = {}


def _trained_policy():
    if "p" not in _TRAINED:
        from paper_1908_06418_amd.policy import Policy
        X, y, by_n = _training_set()
        _say(f"policy: {len(y)} rows (per n = 20..30: {by_n}), mean label {y.mean():.2f}; "
             "training on the GPU")
        P = Policy(seed=0)
        curve = P.train(X, y, steps=600, lr=0.5)
        _TRAINED.update(p=P, curve=curve, rows=len(y), rows_by_n=by_n)
    return _TRAINED["p"], _TRAINED["curve"]


def test_training_reduces_loss(gpu):
    _, curve = _trained_policy()
    assert curve[-1] < curve[0] * 0.9, (curve[0], curve[-1])


@pytest.mark.parametrize("trained", [False, True])
def test_policy_search_is_exact(gpu, trained):
    """Ordering changes nothing but the order: sizes equal the oracle's."""
    from paper_1908_06418_amd import solve_batch
    from paper_1908_06418_amd.policy import Policy
    P = _trained_policy()[0] if trained else Policy(seed=9)
    rng = np.random.default_rng(77)
    pairs = [pq for pq in mi.pairs_c4(200, start=3000) if pq[0]["n"] <= 26][:60]
    pairs += mi.pairs_c3(ns=(40,), seeds=range(6))
    pairs += [(mi.random_small(rng, 14, 0.5, True, 2), mi.random_small(rng, 15, 0.5, True, 2))
              for _ in range(10)]
    want = [oracle.mcs(G, H)["size"] for G, H in pairs]
    for depth, mode in ((0, 3), (2, 1), (2, 2), (1, 3)):
        _say(f"policy search trained={trained} depth={depth} mode={mode}")
        res = solve_batch(pairs, time_limit_s=60, policy=P, policy_depth=depth,
                          policy_mode=mode)
        for (G, H), r, w in zip(pairs, res, want):
            assert r.optimal and r.size == w
            assert oracle.check.is_valid(G, H, r.mapping)
    _say("policy search single wave")
    res = solve_batch(pairs[:20], time_limit_s=60, policy=P, policy_depth=2, policy_mode=3,
                      tuning={"single_wave": 1})
    assert [r.size for r in res] == want[:20]


def _feature_net(k: int, sign: float) -> np.ndarray:
    """Parameters whose network output is sign * feature k: W1[0][k] = 1,
    W2[0][0] = 1, w3[0] = sign, everything else 0 (exact in half precision;
    every feature is non-negative, so the ReLUs pass it unchanged)."""
    p = ref.unflat(np.zeros(ref.N_PARAMS))
    p = {key: a.copy() for key, a in p.items()}
    p["W1"][0, k] = 1.0
    p["W2"][0, 0] = 1.0
    p["w3"][0] = sign
    return ref.flat(p)


def _scorer_pairs():
    rng = np.random.default_rng(11)
    pairs = []
    while len(pairs) < 16:
        n = int(rng.integers(10, 15))
        p = float(rng.uniform(0.25, 0.6))
        nl = int(rng.integers(0, 3)) if len(pairs) % 4 == 3 else 0
        pairs.append((mi.random_small(rng, n, p, False, nl), mi.random_small(rng, n, p, False, nl)))
    return pairs


def _python_nodes(pairs, k, sign, depth, mode):
    """Node counts of the plain Python recursion ordered by sign * feature k
    of oracle.policy.features at nodes with |M| <= depth.  Every feature is a
    count over n (or a 0/1 flag), so it is compared as the integer count:
    a float64 sum of fractions can differ in the last place between equal
    counts, which would break ties differently from the exact counts."""
    from _mcsplit_py import Counter, root
    out = []
    for G, H in pairs:
        def score(u, side, classes, sel, d, cand, G=G, H=H):
            g = G if side == 0 else H
            x = ref.features(g, u, side, classes, sel, d, cand)[k]
            return sign * round(x * g["n"])
        c = Counter(G, H, 0, score=score, depth_max=depth, mode=mode)
        c.rec(root(G, H), 0)
        out.append(c.nodes)
    return out


def test_in_search_scorer_features(gpu):
    """The in-search scorer computes the features the policy is trained on.
    For every feature k, a network whose score is +feature k (and, for the
    features that differ between candidates, -feature k) orders the search
    at |M| <= 3: choosing v (mode 1), the partners (mode 2) or both (3).
    One search alone, one child at a time and no re-pruning expands exactly
    the nodes of the plain Python recursion ordered by the float64 features
    of oracle.policy; sizes stay the oracle's."""
    from paper_1908_06418_amd import solve_batch
    from paper_1908_06418_amd.policy import Policy
    pairs = _scorer_pairs()
    want = [oracle.mcs(G, H) for G, H in pairs]
    tun = {"single_wave": 1, "children_per_wave": 1, "no_reprune": 1, "seg_lanes": 64}
    plain = solve_batch(pairs, time_limit_s=60, tuning=tun)
    assert [r.nodes for r in plain] == [o["nodes"] for o in want]
    varying = (0, 5, 6, 7, 8, 9, 13)
    changed = 0
    for k in range(ref.F):
        for sign in ((1.0, -1.0) if k in varying else (1.0,)):
            for mode in (1, 2, 3):
                _say(f"scorer feature {k} sign {sign:+.0f} mode {mode}")
                res = solve_batch(pairs, time_limit_s=60, tuning=tun,
                                  policy=Policy(params=_feature_net(k, sign)), policy_depth=3,
                                  policy_mode=mode)
                exp = _python_nodes(pairs, k, sign, 3, mode)
                assert [r.nodes for r in res] == exp, (k, sign, mode)
                assert [r.size for r in res] == [o["size"] for o in want]
                changed += exp != [o["nodes"] for o in want]
    # the orders really differ from the plain rule in many of these runs
    assert changed >= 10


def test_policy_gain_report(gpu):
    """What the trained policy gains over the plain rule (smallest vertex in
    descending-degree order, partners in index order) at |M| <= 1: node
    counts on held-out pairs of the training distribution (one wavefront, so
    counts are deterministic) for each policy mode, and time-to-proof on the
    60 pairs of G(30,p) (parallel search) for the best mode."""
    from paper_1908_06418_amd import Plan, solve_batch
    P, curve = _trained_policy()
    held = [pq for pq in mi.pairs_c5(200, start=5000, train=True) if pq[0]["n"] <= 24][:40]
    tun = {"single_wave": 1}
    _say("gain: held-out, plain rule")
    base = solve_batch(held, time_limit_s=100, tuning=tun)
    modes = {}
    for mode in (1, 2, 3):
        _say(f"gain: held-out, policy mode {mode}")
        lrn = solve_batch(held, time_limit_s=100, tuning=tun, policy=P, policy_depth=1,
                          policy_mode=mode)
        both = [(b, l) for b, l in zip(base, lrn) if b.optimal and l.optimal]
        assert len(both) >= 30
        assert all(b.size == l.size for b, l in both)
        modes[mode] = {"pairs": len(both),
                       "nodes_ratio_total": sum(l.nodes for _, l in both) /
                       sum(b.nodes for b, _ in both),
                       "nodes_ratio_median": float(np.median([l.nodes / b.nodes
                                                              for b, l in both]))}
    best = min(modes, key=lambda m: modes[m]["nodes_ratio_total"])
    _TRAINED["best_mode"] = best
    c2 = mi.pairs_c2(ns=(30,))
    times = {}
    for name, kw in (("plain", {}), ("learned", {"policy": P, "policy_depth": 1,
                                                 "policy_mode": best})):
        plan = Plan(c2, time_limit_s=60, **kw).upload()
        ms = []
        for rep in range(3):
            _say(f"gain: c2 n=30, {name}, run {rep}")
            plan.run()
            res = plan.results()
            assert all(r.optimal for r in res)
            ms.append(plan.stats().kernel_ms)
        times[name] = (min(ms), [r.size for r in res], sum(r.nodes for r in res))
        plan.close()
    assert times["plain"][1] == times["learned"][1]
    report = {"held_out_by_mode": modes, "best_mode": best,
              "c2_n30_kernel_ms_plain": times["plain"][0],
              "c2_n30_kernel_ms_learned": times["learned"][0],
              "c2_n30_nodes_plain": times["plain"][2],
              "c2_n30_nodes_learned": times["learned"][2],
              "train_rows": _TRAINED["rows"],
              "train_rows_by_n_20_to_30": _TRAINED["rows_by_n"],
              "train_loss_first_last": [curve[0], curve[-1]]}
    _say("policy gain: " + json.dumps(report))
    write_report("policy_gain.json", report)


def test_c5_learned_vs_degree_report(gpu):
    """The learned-ordering workload's evaluation pairs (n ~ U{35..50}, p
    0.2 for the first 512 and 0.4 for the rest): the 48 smallest of each
    half (the ones a launch can prove), one launch per way under the same
    40 s limit -- the plain degree rule and the trained policy, both one
    search per wavefront (the layout the scorer runs in), and the plain rule
    on the default segmented layout.  Proven count, nodes and median time to
    proof, and, on the pairs both one-search-per-wavefront ways proved, the
    policy's nodes and time to proof relative to the degree rule's.  Sizes
    agree wherever two ways both proved a pair, and every mapping is
    valid."""
    from paper_1908_06418_amd import solve_batch
    P, _ = _trained_policy()
    mode = _TRAINED.get("best_mode", 3)
    pairs = []
    for start in (0, 512):
        half = mi.pairs_c5(512, start=start)
        half.sort(key=lambda pq: (max(pq[0]["n"], pq[1]["n"]), pq[0]["n"] + pq[1]["n"]))
        pairs += half[:48]
    ways = {"degree_segmented": {},
            "degree_one_per_wave": {"tuning": {"seg_lanes": 64}},
            "learned_one_per_wave": {"policy": P, "policy_depth": 2, "policy_mode": mode}}
    out, res_by = {}, {}
    for name, kw in ways.items():
        _say(f"c5: {name}")
        res, st = solve_batch(pairs, time_limit_s=40, with_stats=True, **kw)
        for (G, H), r in zip(pairs, res):
            assert oracle.check.is_valid(G, H, r.mapping)
        proven = [r for r in res if r.optimal]
        out[name] = {"proven": len(proven), "pairs": len(pairs), "nodes": st.nodes,
                     "kernel_ms": st.kernel_ms,
                     "median_time_to_proof_s": float(np.median([r.t_proof_s for r in proven]))
                     if proven else None}
        res_by[name] = res
    names = list(ways)
    for i in range(len(pairs)):
        sizes = {res_by[n][i].size for n in names if res_by[n][i].optimal}
        assert len(sizes) <= 1, (i, sizes)
    both = [i for i in range(len(pairs)) if res_by["degree_one_per_wave"][i].optimal
            and res_by["learned_one_per_wave"][i].optimal]
    if both:
        d, l = res_by["degree_one_per_wave"], res_by["learned_one_per_wave"]
        out["both_proven"] = {
            "pairs": len(both),
            "nodes_ratio_median": float(np.median([l[i].nodes / max(1, d[i].nodes)
                                                   for i in both])),
            "time_to_proof_ratio_median": float(np.median(
                [l[i].t_proof_s / max(1e-9, d[i].t_proof_s) for i in both]))}
    out["policy_mode"] = mode
    _say("c5 report: " + json.dumps(out))
    write_report("c5_learned_vs_degree.json", out)


# Arithmetic of the 16 -> 64 -> 64 -> 1 network per row, in FLOPs (a
# multiply-add counts two): forward 2 (16*64 + 64*64 + 64); the gradient adds
# the backward products (64*64 and 16*64 weight gradients, the 64*64 input
# gradient of the middle layer, and the 64-wide output layer's).
FWD_FLOP = 2 * (16 * 64 + 64 * 64 + 64)
GRAD_FLOP = FWD_FLOP + 2 * (64 * 64 + 16 * 64 + 64 * 64 + 64 + 64)
PEAK_FP16_MFMA = 2.5e15   # dense, MI355X
PEAK_FP32_VECTOR = 157.3e12


def test_policy_kernel_timing_report(gpu):
    """The network's forward and gradient kernels timed on the stored
    training rows and on a large synthetic batch, against the FP16 MFMA roof
    (and the FP32 vector roof their FMAs actually run on).  Report only:
    training is a few hundred such steps on tens of thousands of rows, far
    below a second, so it is not what bounds the learned ordering."""
    import torch
    from paper_1908_06418_amd.policy import Policy
    X, y, _ = _training_set()
    rng = np.random.default_rng(3)
    big = rng.random((1 << 20, 16)).astype(np.float16)
    bigy = (rng.random(1 << 20) < 0.5).astype(np.float32)
    P = Policy(seed=1)
    out = {}
    for name, xs, ys in (("training_rows", X.astype(np.float16), y.astype(np.float32)),
                         ("synthetic_1M", big, bigy)):
        xh = torch.from_numpy(np.ascontiguousarray(xs)).cuda()
        yt = torch.from_numpy(np.ascontiguousarray(ys)).cuda()
        rows = int(xh.shape[0])
        for _ in range(3):
            P.forward(xh)
            P.grad(xh, yt)
        torch.cuda.synchronize()
        reps = 20
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record()
        for _ in range(reps):
            P.forward(xh)
        e[1].record()
        for _ in range(reps):
            P.grad(xh, yt)
        e[2].record()
        torch.cuda.synchronize()
        f_ms = e[0].elapsed_time(e[1]) / reps
        g_ms = e[1].elapsed_time(e[2]) / reps
        ftf = rows * FWD_FLOP / (f_ms * 1e-3) / 1e12
        gtf = rows * GRAD_FLOP / (g_ms * 1e-3) / 1e12
        out[name] = {"rows": rows, "forward_ms": f_ms, "grad_ms": g_ms,
                     "forward_tflops": ftf, "grad_tflops": gtf,
                     "forward_frac_fp16_mfma": ftf * 1e12 / PEAK_FP16_MFMA,
                     "grad_frac_fp16_mfma": gtf * 1e12 / PEAK_FP16_MFMA,
                     "forward_frac_fp32_vector": ftf * 1e12 / PEAK_FP32_VECTOR,
                     "grad_frac_fp32_vector": gtf * 1e12 / PEAK_FP32_VECTOR}
        assert f_ms > 0 and g_ms > 0
    _say("policy kernel timing: " + json.dumps(out))
    write_report("policy_kernel_timing.json", out)
