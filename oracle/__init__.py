"""ORACLE -- test infrastructure only.

Plain CPU implementations of what the GPU search computes, used to prove it
right.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
``cpu_baseline`` leg may import this package; the product package
``paper_1908_06418_amd`` never does, and shares no code with it.

Contents
  - ``mcs``:        plain recursive McSplit in C (``mcsplit_oracle.c``), called
                    through ctypes (paper Sec. II.B, Eq. 1, Algorithm 1).
  - ``path``:       the same C code's class split replayed along a given path.
  - ``brute``:      exhaustive search over injective partial maps (definition,
                    Sec. II.A).
  - ``clique``:     maximum clique of the modular product graph (the
                    Barrow-Burstall reduction the paper cites in Sec. I and
                    Sec. IV).
  - ``labels``:     label strings and classes computed from their definition
                    (Sec. II.B, Table 1).
  - ``check``:      validity of a returned mapping.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mcsplit_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


class _Graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("directed", ctypes.c_int32),
                ("adj", ctypes.POINTER(ctypes.c_uint8)),
                ("label", ctypes.POINTER(ctypes.c_int32))]


def build() -> str:
    """Compile the C oracle with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-shared", "-fPIC",
                           "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def build_planted(plant: int, out_path: str) -> str:
    """Test-only: compile a deliberately wrong variant (see ORACLE_PLANT in
    mcsplit_oracle.c) to out_path."""
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC",
                           f"-DORACLE_PLANT={int(plant)}", "-o", out_path, _SRC])
    return out_path


def _bind(lib):
    lib.oracle_mcs_ordered.restype = ctypes.c_int32
    lib.oracle_mcs_ordered.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Graph),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32)]
    lib.oracle_mcs.restype = ctypes.c_int32
    lib.oracle_mcs.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Graph),
                               ctypes.c_int64, ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_int32),
                               ctypes.POINTER(ctypes.c_int32)]
    return lib


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = _bind(ctypes.CDLL(_LIB))
        lib.oracle_extend.restype = ctypes.c_int32
        lib.oracle_extend.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Graph),
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                      ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]
        lib.oracle_branch_cost.restype = ctypes.c_int64
        lib.oracle_branch_cost.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Graph),
                                           ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                           ctypes.c_int32, ctypes.c_int64]
        lib.oracle_path.restype = ctypes.c_int32
        lib.oracle_path.argtypes = [ctypes.POINTER(_Graph), ctypes.POINTER(_Graph),
                                    ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_int32)]
        _lib = lib
    return _lib


def _matrix(g: dict) -> np.ndarray:
    n = g["n"]
    a = np.zeros((max(n, 1), max(n, 1)), dtype=np.uint8)
    for i, r in enumerate(g["rows"]):
        for j in range(n):
            a[i, j] = (r >> j) & 1
    return np.ascontiguousarray(a)


def _cgraph(g: dict, keep: list) -> _Graph:
    a = _matrix(g)
    keep.append(a)
    lab_p = None
    if g.get("label") is not None:
        lab = np.ascontiguousarray(np.array(g["label"], dtype=np.int32).reshape(-1))
        if lab.size == 0:
            lab = np.zeros(1, np.int32)
        keep.append(lab)
        lab_p = lab.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    return _Graph(g["n"], 1 if g["directed"] else 0,
                  a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), lab_p)


def _p32(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def mcs(G: dict, H: dict, node_limit: int = 0, lib=None, order: str = "degree") -> dict:
    """Maximum common induced subgraph by the plain recursive McSplit.

    Returns {"size", "map" (list of (g, h) original ids), "nodes", "complete",
    "root_bound"}.  ``complete`` is False when ``node_limit`` stopped it.
    ``order``: "degree" (descending degree, Sec. IV.A's default) or "btf"
    (components and the bordered block-triangular order of Sec. IV.A,
    oracle.ordering)."""
    if bool(G["directed"]) != bool(H["directed"]):
        raise ValueError("G and H must both be directed or both undirected")
    if (G.get("label") is None) != (H.get("label") is None):
        raise ValueError("G and H must both be labelled or both unlabelled")
    lib = lib or _load()
    keep: list = []
    cg, ch = _cgraph(G, keep), _cgraph(H, keep)
    cap = max(1, min(G["n"], H["n"]))
    mg = np.zeros(cap, np.int32)
    mh = np.zeros(cap, np.int32)
    nodes = ctypes.c_int64(0)
    complete = ctypes.c_int32(0)
    rb = ctypes.c_int32(0)
    if order == "degree":
        size = lib.oracle_mcs(ctypes.byref(cg), ctypes.byref(ch), int(node_limit), _p32(mg),
                              _p32(mh), ctypes.byref(nodes), ctypes.byref(complete),
                              ctypes.byref(rb))
    elif order == "btf":
        from .ordering import btf_order
        og = np.array(btf_order(G) or [0], np.int32)
        oh = np.array(btf_order(H) or [0], np.int32)
        size = lib.oracle_mcs_ordered(ctypes.byref(cg), ctypes.byref(ch), _p32(og), _p32(oh),
                                      int(node_limit), _p32(mg), _p32(mh),
                                      ctypes.byref(nodes), ctypes.byref(complete),
                                      ctypes.byref(rb))
    else:
        raise ValueError(f"unknown order {order!r}")
    return {"size": int(size), "map": [(int(mg[i]), int(mh[i])) for i in range(size)],
            "nodes": int(nodes.value), "complete": bool(complete.value),
            "root_bound": int(rb.value)}


def path(G: dict, H: dict, steps) -> dict:
    """Replay the C oracle's class split along ``steps`` = [(v, w) or (v, None)]
    in original ids.  Returns {"bounds": [...] (k+1 values), "classes":
    [(set_g, set_h), ...]} or None if a step is not allowed."""
    lib = _load()
    keep: list = []
    cg, ch = _cgraph(G, keep), _cgraph(H, keep)
    k = len(steps)
    pg = np.array([s[0] for s in steps] or [0], np.int32)
    ph = np.array([(-1 if s[1] is None else s[1]) for s in steps] or [0], np.int32)
    bounds = np.zeros(k + 1, np.int32)
    clg = np.zeros(max(1, G["n"]), np.int32)
    clh = np.zeros(max(1, H["n"]), np.int32)
    K = lib.oracle_path(ctypes.byref(cg), ctypes.byref(ch), k, _p32(pg), _p32(ph),
                        _p32(bounds), _p32(clg), _p32(clh))
    if K < 0:
        return None
    classes = []
    for c in range(K):
        classes.append((frozenset(i for i in range(G["n"]) if clg[i] == c),
                        frozenset(i for i in range(H["n"]) if clh[i] == c)))
    return {"bounds": [int(b) for b in bounds], "classes": classes}


def extend(G: dict, H: dict, steps, target: int, node_limit: int = 0, with_nodes: bool = False):
    """True/False: does a common induced subgraph of size >= target contain
    the pairs in steps (original ids, a legal sequence of McSplit steps)?
    None if node_limit stopped the search; raises on an illegal path.  With
    with_nodes, returns (answer, nodes the search entered)."""
    lib = _load()
    keep: list = []
    cg, ch = _cgraph(G, keep), _cgraph(H, keep)
    k = len(steps)
    pg = np.array([s[0] for s in steps] or [0], np.int32)
    ph = np.array([s[1] for s in steps] or [0], np.int32)
    nodes = ctypes.c_int64(0)
    r = lib.oracle_extend(ctypes.byref(cg), ctypes.byref(ch), k, _p32(pg), _p32(ph),
                          int(target), int(node_limit), ctypes.byref(nodes))
    if r == -1:
        raise ValueError("illegal path")
    ans = None if r == -2 else bool(r)
    return (ans, int(nodes.value)) if with_nodes else ans


def branch_cost(G: dict, H: dict, steps, v_first: int, incumbent: int,
                node_limit: int = 0):
    """Nodes the search spends below the node reached by steps when it
    branches on v_first there (incumbent fixed): None if node_limit was hit;
    raises if steps or v_first are not legal there."""
    lib = _load()
    keep: list = []
    cg, ch = _cgraph(G, keep), _cgraph(H, keep)
    k = len(steps)
    pg = np.array([s[0] for s in steps] or [0], np.int32)
    ph = np.array([s[1] for s in steps] or [0], np.int32)
    r = lib.oracle_branch_cost(ctypes.byref(cg), ctypes.byref(ch), k, _p32(pg), _p32(ph),
                               int(v_first), int(incumbent), int(node_limit))
    if r == -1:
        raise ValueError("illegal path or branching vertex")
    return None if r == -2 else int(r)


from . import brute, check, clique, labels  # noqa: E402,F401
