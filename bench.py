"""Benchmark: McSplit search throughput on one MI355X.

A step is one pass of the whole search over one batch of synthetic pairs: a
replay of the HIP graph that copies the packed inputs in, resets the search
state, runs the search kernel (class split, Eq. 1 bound, prune/spawn, work
queue, incumbent, termination) and copies the results back, followed by the
un-permuting of the mappings on the host.  Inputs were packed and uploaded
once before the timed region; the graph's input copy is part of every step.
Every step's sizes are checked against the oracle's stored results for the
workload: equal where the oracle finished (oracle_checked counts those
pairs), at least its lower bound where its node budget ran out, and every
pair proven optimal by the search itself; anything else marks the line
"exact": false.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--budget-s S]
                    [--workload c4|c4_1024|c2|c2_n30|c3|c1|c5|w]

The default workload is the batched one (4096 pairs).  Warmup and timed
steps are cut to fit the wall-clock budget (default 420 s, the oracle leg
included); "steps" and "warmup" in the output are the numbers actually run,
beside "steps_requested" and "warmup_requested".  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "search nodes/sec + MCS instances/sec (batched) at exact size match"
PEAK_INT32_OPS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: int32 lane-ops/s
PEAK_LDS_BYTES = 256 * 128 * 2.4e9     # CUs x 128 bytes per clock x clock: LDS bytes/s
PEAK_HBM_BYTES = 8e12

# HBM bytes per launch of the search kernel, from the copy-calibrated
# FETCH_SIZE / WRITE_SIZE runs recorded in profiles/; reported only while the
# kernel code (comments aside, code_hash) is the one those counters were
# taken on.
TRAFFIC = {
    # profiles/mcs_seg_kernel_c4.md: FETCH_SIZE 11,588,817.8 KiB x 1.9997 plus
    # WRITE_SIZE 401,781,246.1 KiB x 1.000
    "c4": {"source": "mcs_seg.hip", "kernel_code_hash": "4e05206b255fb045",
           "bytes": 435_154_020_482},
    # profiles/mcs_search_kernel_w.md: FETCH_SIZE 192,689.2 KiB x 1.9997 plus
    # WRITE_SIZE 19,447,989.8 KiB x 1.000
    "w": {"source": "mcs_search.hip", "kernel_code_hash": "31a3f47dc12d01c3",
          "bytes": 20_309_302_811},
}

# Algorithmic 32-bit lane operations of one matched child (v, w), per class
# it splits.  Word-wise steps (each one lane-op per 32-bit word of a row):
# remove v and w (2), split both sides by the adjacency letters (4; directed
# 16), popcount every part (4; 8), test each part for emptiness (4; 8) and
# store the surviving parts (2; 4).  Per-class scalar steps: min() per letter
# (2; 4), add into Eq. 1 (2; 4), and both sides non-empty (2; 4).  Undirected
# 16 word-wise + 6 = 22 at 32 bits, directed 38 + 12 = 50.  Each child also
# costs a fixed 30 for the segment reduction of Eq. 1, the compare with the
# incumbent and the ballot.
WORD_OPS = {False: 16, True: 38}
CLASS_OPS = {False: 6, True: 12}
CHILD_OPS = 30


def ops_per_class(word_bytes: int, directed: bool) -> int:
    return WORD_OPS[directed] * (word_bytes // 4) + CLASS_OPS[directed]


def workloads():
    import mcs_instances as mi
    return {
        "c2": ("180 undirected unlabelled pairs G(n,p), n in {30,35,40}, p in {0.1,0.3,0.5}, "
               "20 seeds each, one batched launch", lambda: mi.pairs_c2(), "expected_c2.json"),
        "c2_n30": ("60 undirected unlabelled pairs G(30,p), p in {0.1,0.3,0.5}, 20 seeds each, "
                   "one batched launch", lambda: mi.pairs_c2(ns=(30,)), "expected_c2_n30.json"),
        "c3": ("60 directed vertex-labelled pairs n in {40,50,60}, p=0.1, ceil(0.33n) labels, "
               "one batched launch", lambda: mi.pairs_c3(), "expected_c3.json"),
        "c4_1024": ("first 1024 pairs of the batched workload, n ~ U{10..35}, p ~ U[0.05,0.5)",
                    lambda: mi.pairs_c4(1024), "expected_c4_1024.json"),
        "c4": ("the batched workload: 4096 undirected pairs, n ~ U{10..35}, p ~ U[0.05,0.5), "
               "one persistent launch", lambda: mi.pairs_c4(4096), "expected_c4.json"),
        "c1": ("one undirected unlabelled pair G(16,0.3)", lambda: mi.pair_c1(), None),
        "c5": ("the learned-ordering workload: 1024 undirected pairs, n ~ U{35..50}, "
               "p 0.2 (first 512) / 0.4, one launch", lambda: mi.pairs_c5(1024), None),
        "w": ("40 directed vertex-labelled pairs n in {80,100}, p=0.1, ceil(0.33n) labels "
              "(128-bit rows), one batched launch", lambda: mi.pairs_w(), "expected_w.json"),
    }


def code_hash(text: str) -> str:
    """sha256 (first 16 hex) of source text with // comments, trailing
    blanks and empty lines removed: edits to comments keep it, edits to
    code do not."""
    import hashlib
    import re
    lines = []
    for line in text.splitlines():
        line = re.sub(r"//.*$", "", line).rstrip()
        if line:
            lines.append(line)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def kernel_hash(source: str) -> str:
    """code_hash of a kernel source file together with the device headers
    it includes."""
    text = ""
    for name in (source, "mcs_device.h", "mcs_layout.h"):
        with open(os.path.join(ROOT, "paper_1908_06418_amd", "csrc", name)) as f:
            text += f.read() + "\n"
    return code_hash(text)


def traffic_for(workload: str, source: str, launches: int):
    t = TRAFFIC.get(workload)
    if not t or t.get("source") != source or t["kernel_code_hash"] != kernel_hash(source):
        return None
    return t["bytes"] * launches


def expected_sizes(fname):
    path = os.path.join(ROOT, "tests", "golden", fname) if fname else None
    if path is None or not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def host_cpu() -> str:
    """The host CPU model as lscpu names it (else /proc/cpuinfo)."""
    import subprocess
    try:
        out = subprocess.run(["lscpu"], stdout=subprocess.PIPE, stderr=subprocess.DEVNULL,
                             text=True, timeout=10).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                return line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def usable_cores() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline(pairs, exp, wall_s=15.0, seed=20260, pair_cap_s=30.0):
    """The oracle, as it stands, on a bounded random sample of the workload.

    Pairs are drawn in a seeded random order from those the stored oracle run
    finished (the others cannot be timed to completion) in at most
    pair_cap_s seconds of one core (so that no single pair sets the leg's
    wall time: the stored run finished some pairs only after minutes),
    and taken until their stored one-core times add up to about
    wall_s x cores seconds; the sample is then solved one process per pair on
    that many host cores."""
    import random
    from concurrent.futures import ProcessPoolExecutor

    import oracle
    oracle._load()
    cores = usable_cores()
    idx = list(range(len(pairs)))
    finished = len(idx)
    eligible = len(idx)
    if exp is not None:
        idx = [i for i in idx if exp["pairs"][i]["complete"]]
        finished = len(idx)
        idx = [i for i in idx if exp["pairs"][i]["seconds"] <= pair_cap_s]
        eligible = len(idx)
        random.Random(seed).shuffle(idx)
        acc, keep = 0.0, []
        for i in idx:
            if acc >= wall_s * cores:
                break
            acc += exp["pairs"][i]["seconds"]
            keep.append(i)
        idx = keep
    sample = [pairs[i] for i in idx]
    t0 = time.time()
    with ProcessPoolExecutor(cores) as ex:
        out = list(ex.map(_oracle_one, [G for G, _ in sample], [H for _, H in sample]))
    dt = time.time() - t0
    nodes = sum(n for n, _ in out)
    return {"value": nodes / dt, "unit": "nodes/s", "cores": cores, "kind": "oracle",
            "instances_per_s": len(sample) / dt, "cpu": host_cpu(),
            "sample": f"{len(sample)} pairs drawn at random (seed {seed}) from the {eligible} "
                      f"of the {finished} (of {len(pairs)}) pairs of the same workload the oracle "
                      f"finishes within its stored node budget that took it at most {pair_cap_s:.0f} s "
                      f"of one core, until their one-core times sum to about "
                      f"{wall_s:.0f} s x {cores} cores; solved to optimality by the plain "
                      f"recursive C oracle, one process per pair on {cores} host cores "
                      f"({host_cpu()}), {dt:.1f} s wall"}


def _spread(xs):
    """Median and maximum over instances (and steps), in seconds of kernel time."""
    if not xs:
        return None
    xs = sorted(xs)
    return {"median": xs[len(xs) // 2], "max": xs[-1]}


def _oracle_one(G, H):
    import oracle
    r = oracle.mcs(G, H)
    return r["nodes"], r["complete"]


def main():
    t_start = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--time-limit", type=float, default=300.0,
                    help="per-launch search time limit, seconds")
    ap.add_argument("--budget-s", type=float, default=420.0,
                    help="wall-clock budget of the whole run: warmup and timed steps are cut "
                         "to fit it (at least one warmup step, if any was asked for, and 3 "
                         "timed steps, or all asked for if fewer, are always run), "
                         "leaving room for the cpu_baseline leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the kernels directly instead of replaying the HIP graph")
    ap.add_argument("--tuning", default="", help="JSON dict of mcs_tuning fields")
    ap.add_argument("--ordering", default="degree", choices=("degree", "btf", "portfolio"),
                    help="static vertex order (portfolio: both orders racing on one "
                         "incumbent per pair)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain 256 MiB device copy (outside the timed region), "
                         "so HBM byte counters can be scaled against a known size")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this search runs on one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1908_06418_amd import Plan, _abi, build
    if not os.path.exists(_abi.LIB_PATH):
        build.build()
    assert torch.cuda.is_available(), "bench.py needs the GPU"
    torch.cuda.set_device(0)

    if args.calibrate_copy:
        src = torch.ones(256 << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    desc, factory, exp_file = workloads()[args.workload]
    pairs = factory()
    exp = expected_sizes(exp_file)
    if args.tuning:
        tuning, tuning_src = json.loads(args.tuning), "command line"
    else:
        from paper_1908_06418_amd import autotune
        tuning = autotune.tuned(pairs)
        tuning_src = "autotuner table" if tuning else "library defaults"
    tuning = dict(tuning or {})
    if not args.no_graph:
        tuning["use_graph"] = 1
    plan = Plan(pairs, time_limit_s=args.time_limit, tuning=tuning,
                ordering=args.ordering).upload()
    print(f"bench: {args.workload}, {len(pairs)} pairs, tuning {tuning} ({tuning_src})",
          file=sys.stderr, flush=True)

    def step():
        plan.run()
        return plan.results()

    # The reserve kept for the oracle leg and for printing.
    reserve = 5.0 if args.no_cpu_baseline else 40.0

    def left():
        return args.budget_s - (time.perf_counter() - t_start) - reserve

    warm_done = 0
    step_s = None
    for _ in range(max(0, args.warmup)):
        if warm_done >= 1 and step_s is not None and left() < step_s * (3 + 1):
            break
        t1 = time.perf_counter()
        step()
        torch.cuda.synchronize()
        step_s = time.perf_counter() - t1
        warm_done += 1
        print(f"bench: warmup step {warm_done} took {step_s:.2f} s", file=sys.stderr, flush=True)
    K = args.steps
    if step_s is not None and step_s > 0:
        K = max(min(3, args.steps), min(args.steps, int(left() / step_s)))
    exact = True
    nodes = 0
    kernel_ms = 0.0
    lane_slots = batches = children = node_classes = 0
    lds_bytes = pops = donations = hbm_frames = 0
    proven = 0
    busy = []
    t_best, t_proof = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        res = step()
        st = plan.stats()
        nodes += st.nodes
        kernel_ms += st.kernel_ms
        lane_slots += st.lane_slots
        node_classes += st.node_classes
        lds_bytes += st.lds_bytes
        batches += st.batches
        children += st.children
        pops += st.pops
        donations += st.donations
        hbm_frames += st.hbm_frames
        proven += sum(r.optimal for r in res)
        busy.append(st.busy_frac)
        t_best += [r.t_best_s for r in res]
        t_proof += [r.t_proof_s for r in res if r.optimal]
        if exp is not None:
            for r, e in zip(res, exp["pairs"]):
                if (e["complete"] and r.size != e["size"]) or r.size < e["size"]:
                    exact = False
        if not all(r.optimal for r in res):
            exact = False
        print(f"bench: timed step {k + 1}/{K}: kernel {st.kernel_ms:.1f} ms, "
              f"{st.nodes:.3e} nodes", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    nmax = max(max(G["n"], H["n"]) for G, H in pairs)
    word = 4 if nmax <= 32 else 8 if nmax <= 64 else 16
    directed = any(G["directed"] for G, _ in pairs)
    seg_lanes = int(tuning.get("seg_lanes", 0) or 8)
    segmented = word <= 8 and seg_lanes != 64
    kernel_src = "mcs_seg.hip" if segmented else "mcs_search.hip"
    kernel_name = (f"mcs_seg_kernel ({seg_lanes}-lane searches)" if segmented
                   else "mcs_search_kernel")
    opc = ops_per_class(word, directed)
    ops = node_classes * opc + nodes * CHILD_OPS
    kern_s = kernel_ms / 1e3
    achieved = ops / kern_s / 1e12 if kern_s > 0 else 0.0
    peak = PEAK_INT32_OPS / 1e12
    line = {
        "metric": METRIC,
        "value": nodes / elapsed,
        "unit": "nodes/s",
        "n_gpus": 1,
        "steps": K,
        "steps_requested": args.steps,
        "warmup": warm_done,
        "warmup_requested": args.warmup,
        "ms_per_step": elapsed / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {4: "u32", 8: "u64", 16: "u128", 32: "u256"}[word],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {desc}", "pairs": len(pairs),
                   "word_bits": 8 * word, "directed": directed, "hip_graph": not args.no_graph,
                   "ordering": args.ordering,
                   "tuning": tuning, "tuning_source": tuning_src},
        "instances_per_s": len(pairs) * K / elapsed,
        "exact": exact,
        "oracle_checked": sum(e["complete"] for e in exp["pairs"]) if exp else 0,
        "proven_per_step": proven / K,
        "kernel_ms_per_step": kernel_ms / K,
        "nodes_per_step": nodes / K,
        "time_to_best_s": _spread(t_best),
        "time_to_proof_s": _spread(t_proof),
        "busy_frac": sum(busy) / len(busy) if busy else 0.0,
        "active_lane_frac": lane_slots / (64.0 * batches) if batches else 0.0,
        "children_per_batch": children / batches if batches else 0.0,
        "search_stats": {"steps_per_node": batches / nodes if nodes else 0.0,
                         "children_per_node": children / nodes if nodes else 0.0,
                         "queue_takes_per_node": pops / nodes if nodes else 0.0,
                         "donations_per_node": donations / nodes if nodes else 0.0,
                         "hbm_frames_per_node": hbm_frames / nodes if nodes else 0.0},
        "waves": st.waves,
        "lds_per_wave": st.lds_per_wave,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "Tops/s",
                     "frac": achieved / peak if peak else 0.0,
                     "traffic": traffic_for(args.workload, kernel_src, 1),
                     "kernel": kernel_name,
                     "per_unit": f"{opc} int32 lane-ops per class of each matched child "
                                 f"counted as a node, plus {CHILD_OPS} per node; "
                                 "re-evaluated siblings are not counted"},
    }
    traffic = line["roofline"]["traffic"]
    line["bandwidth"] = {
        "lds": {"achieved_GBps": lds_bytes / kern_s / 1e9 if kern_s else 0.0,
                "peak_GBps": PEAK_LDS_BYTES / 1e9,
                "frac": lds_bytes / kern_s / PEAK_LDS_BYTES if kern_s else 0.0,
                "bytes": "algorithmic: adjacency rows of v and the partners per child batch, "
                         "and each pushed frame's classes written once and read twice "
                         "(mcs_stats.lds_bytes, from the kernel's counters)"
                         + ("; with 128- and 256-bit rows the classes and v's G row live in "
                            "the workspace (L1/L2), not LDS" if word >= 16 else "")},
        "hbm": {"achieved_GBps": traffic * K / kern_s / 1e9 if traffic and kern_s else None,
                "peak_GBps": PEAK_HBM_BYTES / 1e9,
                "frac": traffic * K / kern_s / PEAK_HBM_BYTES if traffic and kern_s else None,
                "bytes": "FETCH_SIZE + WRITE_SIZE per launch, copy-calibrated (profiles/)"},
    }
    plan.close()
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(pairs, exp)
    line["wall_s"] = time.perf_counter() - t_start
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
