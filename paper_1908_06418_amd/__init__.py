"""MI355X (gfx950) maximum common induced subgraph search -- Python binding.

The search (McSplit branch and bound: class split by adjacency, Eq. 1 bound,
device work queue, atomic incumbents) runs in the HIP library libmcs.so behind
the C ABI of include/mcs.h.  This module only marshals arguments; PyTorch
supplies the device workspace and the stream.

Graphs are dicts {"n", "directed", "rows", "label"}: rows[i] is an int whose
bit j is set iff the arc i -> j exists; label is None or a list of n ints.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import numpy as np

from . import _abi

__all__ = ["McsError", "Plan", "solve", "solve_batch", "solve_goals", "workspace_size",
           "Tuning", "status_string"]


class McsError(RuntimeError):
    def __init__(self, status: int, detail: str):
        self.status = status
        super().__init__(f"{status_string(status)} ({status}): {detail}")


def status_string(s: int) -> str:
    return _abi.load().mcs_status_string(s).decode()


def _last_error() -> str:
    return _abi.load().mcs_last_error().decode()


@dataclass
class Tuning:
    waves_per_cu: int = 0
    children_per_wave: int = 0
    ring_slots: int = 0
    donate_low: int = 0
    donate_depth: int = 0
    check_interval: int = 0
    no_reprune: int = 0
    single_wave: int = 0
    use_graph: int = 0
    stack_classes: int = 0
    backoff_max: int = 0
    seg_lanes: int = 0

    def to_c(self) -> _abi.mcs_tuning:
        return _abi.mcs_tuning(self.waves_per_cu, self.children_per_wave, self.ring_slots,
                               self.donate_low, self.donate_depth, self.check_interval,
                               self.no_reprune, self.single_wave, self.use_graph,
                               self.stack_classes, self.backoff_max, self.seg_lanes)


class _Marshal:
    """Keeps the numpy buffers behind mcs_graph arrays alive."""

    def __init__(self, pairs):
        self.keep = []
        n = len(pairs)
        self.G = (_abi.mcs_graph * max(n, 1))()
        self.H = (_abi.mcs_graph * max(n, 1))()
        for i, (g, h) in enumerate(pairs):
            self.G[i] = self._graph(g)
            self.H[i] = self._graph(h)

    def _graph(self, g) -> _abi.mcs_graph:
        n = int(g["n"])
        # rw 64-bit words per row: one up to 64 vertices, ceil(n / 64) above
        rw = 1 if n <= 64 else (n + 63) // 64
        rows = np.zeros(max(n, 1) * rw, dtype=np.uint64)
        for i, r in enumerate(g["rows"][:max(n, 0)]):
            for k in range(rw):
                rows[i * rw + k] = np.uint64((int(r) >> (64 * k)) & 0xFFFFFFFFFFFFFFFF)
        self.keep.append(rows)
        lab = None
        if g.get("label") is not None:
            la = np.array(list(g["label"]) or [0], dtype=np.int32)
            self.keep.append(la)
            lab = la.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        return _abi.mcs_graph(n, 1 if g.get("directed") else 0,
                              rows.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), lab)


ORDERINGS = {"degree": 0, "btf": 1, "portfolio": 2}


def _opts(node_limit, time_limit_s, tuning, policy=None, policy_depth=0, policy_mode=0,
          ordering="degree", deadend_nodes=0, deadend_ratio=0):
    """policy: a torch half tensor of packed parameters on the device (or an
    object with .half_params, see policy.Policy).  ordering: "degree",
    "btf" or "portfolio" (both orders racing on one incumbent;
    mcs_opts.ordering)."""
    t = None
    tc = None
    if tuning is not None:
        tc = tuning.to_c() if isinstance(tuning, Tuning) else Tuning(**tuning).to_c()
        t = ctypes.pointer(tc)
    ptr = None
    if policy is not None:
        hp = getattr(policy, "half_params", policy)
        ptr = ctypes.c_void_p(hp.data_ptr())
    o = _abi.mcs_opts(int(node_limit or 0), float(time_limit_s or 0.0), t, ptr,
                      int(policy_depth), int(policy_mode), ORDERINGS[ordering],
                      int(deadend_ratio), int(deadend_nodes))
    return o, tc


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no GPU visible: the search runs only on the HIP device")
    return torch


@dataclass
class Result:
    size: int
    optimal: bool
    mapping: list
    nodes: int
    t_best_s: float
    t_proof_s: float


@dataclass
class Stats:
    nodes: int = 0
    batches: int = 0
    children: int = 0
    lane_slots: int = 0
    donations: int = 0
    pops: int = 0
    waves: int = 0
    blocks: int = 0
    lds_per_wave: int = 0
    stopped: int = 0
    kernel_ms: float = 0.0
    busy_wave_s: float = 0.0
    hbm_frames: int = 0
    stack_classes: int = 0
    max_stack_used: int = 0
    sleep_wave_s: float = 0.0
    lds_bytes: int = 0
    node_classes: int = 0
    extra: dict = field(default_factory=dict)

    @property
    def busy_frac(self) -> float:
        """Share of the launch's wavefront-time spent searching."""
        span = self.waves * self.kernel_ms * 1e-3
        return self.busy_wave_s / span if span > 0 else 0.0


class Plan:
    """A batch of pairs prepared once (mcs_plan_create), uploaded once into a
    torch-allocated workspace (mcs_plan_upload), then run any number of times
    (mcs_plan_run) -- inputs stay resident in HBM between runs."""

    def __init__(self, pairs, node_limit=0, time_limit_s=0.0, tuning=None, policy=None,
                 policy_depth=1, policy_mode=0, ordering="degree", deadend_nodes=0,
                 deadend_ratio=0):
        self.lib = _abi.load()
        self.pairs = list(pairs)
        self._m = _Marshal(self.pairs)
        self._policy = policy  # keeps the device parameters alive
        self._o, self._t = _opts(node_limit, time_limit_s, tuning, policy, policy_depth,
                                 policy_mode, ordering, deadend_nodes, deadend_ratio)
        h = ctypes.c_void_p()
        st = self.lib.mcs_plan_create(len(self.pairs), self._m.G, self._m.H,
                                      ctypes.byref(self._o), ctypes.byref(h))
        if st < 0:
            raise McsError(st, _last_error())
        self.handle = h
        self.ws = None
        self.stream = None

    @property
    def workspace_bytes(self) -> int:
        return int(self.lib.mcs_plan_workspace_size(self.handle))

    def upload(self, stream=None):
        torch = _torch()
        nbytes = self.workspace_bytes
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
        base = self.ws.data_ptr()
        base = (base + 255) & ~255
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        st = self.lib.mcs_plan_upload(self.handle, ctypes.c_void_p(base), nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream))
        if st < 0:
            raise McsError(st, _last_error())
        return self

    def run(self):
        st = self.lib.mcs_plan_run(self.handle, ctypes.c_void_p(self.stream.cuda_stream))
        if st < 0:
            raise McsError(st, _last_error())

    def set_goals(self, goals):
        """mcs_plan_set_goals: goal[i] > 0 asks the next runs only whether
        instance i has a common induced subgraph of at least goal[i]
        vertices; 0 is a plain search, < 0 skips the instance."""
        if len(goals) != len(self.pairs):
            raise ValueError("one goal per instance")
        g = (ctypes.c_int32 * len(goals))(*[int(x) for x in goals])
        st = self.lib.mcs_plan_set_goals(self.handle, g, ctypes.c_void_p(self.stream.cuda_stream))
        if st < 0:
            raise McsError(st, _last_error())

    def results(self):
        n = len(self.pairs)
        res = (_abi.mcs_result * n)()
        bufs = []
        for i, (g, h) in enumerate(self.pairs):
            cap = max(1, min(int(g["n"]), int(h["n"])))
            mg = (ctypes.c_int32 * cap)()
            mh = (ctypes.c_int32 * cap)()
            bufs.append((mg, mh))
            res[i].map_g = mg
            res[i].map_h = mh
        st = self.lib.mcs_plan_results(self.handle, res,
                                       ctypes.c_void_p(self.stream.cuda_stream))
        if st < 0:
            raise McsError(st, _last_error())
        out = []
        for i in range(n):
            r = res[i]
            mg, mh = bufs[i]
            out.append(Result(int(r.size), bool(r.optimal),
                              [(int(mg[j]), int(mh[j])) for j in range(max(r.size, 0))],
                              int(r.nodes), float(r.t_best_s), float(r.t_proof_s)))
        self.status = st
        return out

    def stats(self) -> Stats:
        s = _abi.mcs_stats()
        st = self.lib.mcs_plan_stats(self.handle, ctypes.byref(s))
        if st < 0:
            raise McsError(st, _last_error())
        return Stats(int(s.nodes), int(s.batches), int(s.children), int(s.lane_slots),
                     int(s.donations), int(s.pops), int(s.waves), int(s.blocks),
                     int(s.lds_per_wave), int(s.stopped), float(s.kernel_ms),
                     float(s.busy_wave_s), int(s.hbm_frames), int(s.stack_classes),
                     int(s.max_stack_used), float(s.sleep_wave_s), int(s.lds_bytes),
                     int(s.node_classes))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.mcs_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(pairs, node_limit=0, time_limit_s=0.0, tuning=None, with_stats=False,
                policy=None, policy_depth=1, policy_mode=0, ordering="degree",
                deadend_nodes=0, deadend_ratio=0):
    """MCS of every pair in one launch.  Returns a list of Result (and Stats)."""
    p = Plan(pairs, node_limit, time_limit_s, tuning, policy, policy_depth, policy_mode,
             ordering, deadend_nodes, deadend_ratio).upload()
    p.run()
    res = p.results()
    st = p.stats() if with_stats else None
    p.close()
    return (res, st) if with_stats else res


def solve_batch_static(pairs, node_limit=0, time_limit_s=0.0, tuning=None, ordering="degree",
                       deadend_nodes=0, deadend_ratio=0):
    """MCS of every pair in one launch on the library's static device scratch
    (mcs_solve_batch_static): no device memory is allocated.  Returns a list
    of Result."""
    lib = _abi.load()
    torch = _torch()
    pairs = list(pairs)
    m = _Marshal(pairs)
    o, _t = _opts(node_limit, time_limit_s, tuning, ordering=ordering,
                  deadend_nodes=deadend_nodes, deadend_ratio=deadend_ratio)
    n = len(pairs)
    res = (_abi.mcs_result * max(n, 1))()
    bufs = []
    for i, (g, h) in enumerate(pairs):
        cap = max(1, min(int(g["n"]), int(h["n"])))
        mg, mh = (ctypes.c_int32 * cap)(), (ctypes.c_int32 * cap)()
        bufs.append((mg, mh))
        res[i].map_g, res[i].map_h = mg, mh
    stream = torch.cuda.current_stream()
    st = lib.mcs_solve_batch_static(n, m.G, m.H, ctypes.byref(o),
                                    ctypes.c_void_p(stream.cuda_stream), res)
    if st < 0:
        raise McsError(st, _last_error())
    return [Result(int(r.size), bool(r.optimal),
                   [(int(bufs[i][0][j]), int(bufs[i][1][j])) for j in range(max(r.size, 0))],
                   int(r.nodes), float(r.t_best_s), float(r.t_proof_s))
            for i, r in enumerate(res[:n])]


GOAL_STRATEGIES = {"top-down": 0, "bisect": 1, "dead-end+1": 2, "dead-end*2": 3}


def solve_goals(pairs, strategy="top-down", node_limit=0, time_limit_s=0.0, tuning=None,
                with_launches=False, ordering="degree", deadend_nodes=0, deadend_ratio=0):
    """Goal-directed search (mcs_solve_goals): strategy "top-down" asks for
    the root bound, then one less, ...; "bisect" takes a node-limited plain
    run's size as a lower bound and binary-searches the goal; "dead-end+1"
    and "dead-end*2" run the plain search with the dead-end forecast
    (deadend_nodes, deadend_ratio) and answer each forecast by raising the
    incumbent by 1, or by an increment that doubles at each forecast, then
    binary-search once a raised bound proves unreachable."""
    import torch
    lib = _abi.load()
    _torch()
    pairs = list(pairs)
    m = _Marshal(pairs)
    o, _t = _opts(node_limit, time_limit_s, tuning, ordering=ordering,
                  deadend_nodes=deadend_nodes, deadend_ratio=deadend_ratio)
    nbytes = int(lib.mcs_workspace_size(len(pairs), m.G, m.H, ctypes.byref(o)))
    if nbytes == 0:
        raise McsError(-1, _last_error())
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
    base = (ws.data_ptr() + 255) & ~255
    stream = torch.cuda.current_stream()
    n = len(pairs)
    res = (_abi.mcs_result * n)()
    bufs = []
    for i, (g, h) in enumerate(pairs):
        cap = max(1, min(int(g["n"]), int(h["n"])))
        mg, mh = (ctypes.c_int32 * cap)(), (ctypes.c_int32 * cap)()
        bufs.append((mg, mh))
        res[i].map_g, res[i].map_h = mg, mh
    launches = ctypes.c_int32(0)
    strat = GOAL_STRATEGIES[strategy]
    st = lib.mcs_solve_goals(n, m.G, m.H, ctypes.byref(o), strat, ctypes.c_void_p(base), nbytes,
                             ctypes.c_void_p(stream.cuda_stream), res, ctypes.byref(launches))
    if st < 0:
        raise McsError(st, _last_error())
    out = [Result(int(r.size), bool(r.optimal),
                  [(int(bufs[i][0][j]), int(bufs[i][1][j])) for j in range(max(r.size, 0))],
                  int(r.nodes), float(r.t_best_s), float(r.t_proof_s))
           for i, r in enumerate(res)]
    return (out, int(launches.value)) if with_launches else out


def solve(G, H, **kw):
    """MCS of one pair."""
    out = solve_batch([(G, H)], **kw)
    return out[0] if not kw.get("with_stats") else (out[0][0], out[1])


def workspace_size(pairs, node_limit=0, time_limit_s=0.0, tuning=None) -> int:
    lib = _abi.load()
    m = _Marshal(pairs)
    o, _t = _opts(node_limit, time_limit_s, tuning)
    return int(lib.mcs_workspace_size(len(pairs), m.G, m.H, ctypes.byref(o)))
