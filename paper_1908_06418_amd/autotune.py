"""Autotuner for the search kernel's launch and scheduling knobs.

The knobs (mcs_tuning in include/mcs.h) change only speed, never answers:
the search layout (searches of 4, 8 or 16 lanes, or one per wavefront, and then
how many sibling children a wavefront evaluates at once), resident
wavefronts per CU, the LDS part of each search's class stack, the node
queue's depth, how many records each XCD's queue ring is kept stocked with,
and how often a busy search looks at the queue.
The tuner times candidate settings on a sample of the workload through the C
ABI, rejects any setting whose sizes differ from the others (they must agree:
the search is exact), and caches the fastest per workload class in a JSON
file ($MCS_TUNING_FILE, else ~/.cache/mcs_tuning.json).  tune() times a
given list; tune_staged() walks the axes one at a time (coordinate descent:
every value of one axis with the others at their best so far).
"""
from __future__ import annotations

import json
import math
import os
import time

DEFAULT_CANDIDATES = [
    {"seg_lanes": sl, "waves_per_cu": w, "donate_low": lo}
    for sl in (8, 16)
    for w in (8, 12, 16)
    for lo in (1, 2)
]

# Axes of the staged search, in the order they are walked.  Zero is the
# library's own choice.  children_per_wave applies to one search per
# wavefront (seg_lanes 64) only.
AXES = [
    ("seg_lanes", (0, 16, 4, 64)),
    ("waves_per_cu", (0, 8, 12, 16, 20)),
    ("children_per_wave", (8, 4, 2)),
    ("stack_classes", (0, 1)),
    ("ring_slots", (0, 4096, 32768)),
    ("donate_low", (0, 1, 4)),
    ("check_interval", (0, 64, 256)),
]


def cache_path() -> str:
    return os.environ.get("MCS_TUNING_FILE",
                          os.path.join(os.path.expanduser("~"), ".cache", "mcs_tuning.json"))


def workload_key(pairs) -> str:
    """Workload class: row word size, directed, largest n (to 8), mean
    density (to 0.1), labelled, batch size (to a power of two)."""
    nmax = max(max(G["n"], H["n"]) for G, H in pairs)
    directed = any(G["directed"] for G, _ in pairs)
    labelled = any(G.get("label") is not None for G, _ in pairs)
    dens = []
    for G, H in pairs:
        for g in (G, H):
            n = g["n"]
            if n > 1:
                e = sum(bin(r).count("1") for r in g["rows"])
                dens.append(e / (n * (n - 1)))
    p = sum(dens) / len(dens) if dens else 0.0
    bits = 32 if nmax <= 32 else 64 if nmax <= 64 else 128 if nmax <= 128 else 256
    nb = 8 * math.ceil(max(nmax, 1) / 8)
    batch = 1 << max(0, math.ceil(math.log2(len(pairs))))
    return (f"w{bits}-{'d' if directed else 'u'}{'l' if labelled else ''}-n{nb}"
            f"-p{round(p, 1):.1f}-b{batch}")


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def pick(measurements: list) -> dict:
    """Fastest candidate among those that proved every pair with the common
    sizes.  measurements: dicts {tuning, kernel_ms, sizes, proven}."""
    ok = [m for m in measurements if m["proven"]]
    if not ok:
        raise RuntimeError("no candidate proved every sample pair within the time limit")
    ref = ok[0]["sizes"]
    for m in ok:
        if m["sizes"] != ref:
            raise RuntimeError(f"tunings disagree on sizes: {m['tuning']}")
    return min(ok, key=lambda m: m["kernel_ms"])


def measure(pairs, cand: dict, time_limit_s: float = 30.0, reps: int = 1) -> dict:
    """Kernel time (best of reps launches) of one candidate on pairs."""
    from . import Plan
    plan = Plan(pairs, time_limit_s=time_limit_s, tuning=cand).upload()
    try:
        best_ms = None
        for _ in range(reps):
            plan.run()
            res = plan.results()
            st = plan.stats()
            best_ms = st.kernel_ms if best_ms is None else min(best_ms, st.kernel_ms)
    finally:
        plan.close()
    return {"tuning": dict(cand), "kernel_ms": best_ms, "sizes": [r.size for r in res],
            "proven": all(r.optimal for r in res), "nodes": st.nodes}


def tune(pairs, candidates=None, time_limit_s: float = 30.0, reps: int = 1, log=None) -> dict:
    """Time every candidate on pairs (GPU); returns the winning measurement
    with the whole table under 'table'."""
    table = []
    for cand in candidates or DEFAULT_CANDIDATES:
        m = measure(pairs, cand, time_limit_s, reps)
        table.append(m)
        if log:
            log(m)
    best = dict(pick(table))
    best["table"] = table
    return best


def staged_candidates(best: dict, axis: str, values) -> list:
    """The candidates of one stage: best with axis set to each value (values
    that cannot apply to best's layout are left out)."""
    out = []
    for v in values:
        if axis == "children_per_wave" and best.get("seg_lanes", 16) != 64:
            continue
        c = dict(best)
        if v:
            c[axis] = v
        else:
            c.pop(axis, None)
        if c not in out:
            out.append(c)
    return out


def tune_staged(pairs, axes=None, base=None, time_limit_s: float = 30.0, reps: int = 1,
                log=None) -> dict:
    """Coordinate descent over the axes: each stage times every value of one
    axis with the others at the best found so far, and keeps the fastest
    (sizes must agree across every candidate of every stage).  Returns the
    winning measurement with every measurement under 'table'."""
    best_t = dict(base or {})
    table = []
    seen = {}
    best = None
    for axis, values in axes or AXES:
        stage = []
        for cand in staged_candidates(best_t, axis, values):
            key = json.dumps(cand, sort_keys=True)
            if key not in seen:
                seen[key] = measure(pairs, cand, time_limit_s, reps)
                seen[key]["stage"] = axis
                table.append(seen[key])
                if log:
                    log(seen[key])
            stage.append(seen[key])
        if stage:
            best = pick(stage)
            best_t = dict(best["tuning"])
    pick(table)  # every candidate of every stage agrees on sizes
    best = dict(best)
    best["table"] = table
    return best


SHIPPED = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuning_table.json")


def tuned(pairs, path: str | None = None) -> dict | None:
    """Tuning for this workload class: the user's cache first, then the table
    shipped with the package (measured with tune_and_store on an MI355X),
    else None (library defaults)."""
    key = workload_key(pairs)
    entry = load_cache(path).get(key)
    if entry is None and path is None:
        entry = load_cache(SHIPPED).get(key)
    return dict(entry["tuning"]) if entry else None


def tune_and_store(pairs, sample=None, path: str | None = None, staged: bool = False,
                   note: str = "", **kw) -> dict:
    """Tune on sample (default: pairs) and store the winner under pairs'
    workload class."""
    best = (tune_staged if staged else tune)(sample or pairs, **kw)
    data = load_cache(path)
    entry = {"tuning": best["tuning"], "kernel_ms": best["kernel_ms"],
             "when": time.strftime("%Y-%m-%d %H:%M:%S")}
    if note:
        entry["measured_on"] = note
    data[workload_key(pairs)] = entry
    save_cache(data, path)
    return best


# Named synthetic workloads the command line below can tune (the generators
# of mcs_instances, at the shapes bench.py measures).
def _named_workload(name: str):
    import mcs_instances as mi
    return {
        "c2_n30": (lambda: mi.pairs_c2(ns=(30,)),
                   "60 undirected pairs G(30,p), p in {0.1,0.3,0.5}"),
        "c3": (lambda: mi.pairs_c3(), "60 directed labelled pairs n in {40,50,60}, p=0.1"),
        "c4": (lambda: mi.pairs_c4(4096),
               "the 4096 batched pairs, n ~ U{10..35}, p ~ U[0.05,0.5)"),
    }[name]


def main(argv=None) -> int:
    """python -m paper_1908_06418_amd.autotune WORKLOAD [--out PATH]:
    staged tuning of a named workload on the GPU, stored under its workload
    class (in the shipped table unless --out names another file)."""
    import argparse
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("workload", choices=("c2_n30", "c3", "c4"))
    ap.add_argument("--out", default=SHIPPED)
    ap.add_argument("--time-limit", type=float, default=120.0)
    args = ap.parse_args(argv)
    factory, desc = _named_workload(args.workload)
    pairs = factory()

    def log(m):
        print(json.dumps({"tuning": m["tuning"], "kernel_ms": round(m["kernel_ms"], 3),
                          "proven": m["proven"]}), flush=True)

    stages = sum(len(staged_candidates({}, a, v)) for a, v in AXES)
    best = tune_and_store(pairs, path=args.out, staged=True, time_limit_s=args.time_limit,
                          log=log, note=f"MI355X, {desc}; staged tuning, about {stages} "
                                        "candidates, one launch each")
    print(json.dumps({"workload": args.workload, "key": workload_key(pairs),
                      "tuning": best["tuning"], "kernel_ms": best["kernel_ms"]}), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
