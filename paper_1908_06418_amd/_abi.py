"""ctypes mirror of include/mcs.h.  Argument marshalling only: every step of
the search runs in libmcs.so."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmcs.so")

MCS_OK = 0
MCS_LIMIT = 1
MCS_E_INVALID = -1
MCS_E_TOO_LARGE = -2
MCS_E_DEVICE = -3
MCS_E_WORKSPACE = -4
MCS_E_INTERNAL = -5
MCS_MAX_N = 254
MCS_STATIC_SCRATCH_BYTES = 64 << 20


class mcs_graph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("directed", ctypes.c_int32),
                ("adj", ctypes.POINTER(ctypes.c_uint64)),
                ("label", ctypes.POINTER(ctypes.c_int32))]


class mcs_tuning(ctypes.Structure):
    _fields_ = [("waves_per_cu", ctypes.c_int32), ("children_per_wave", ctypes.c_int32),
                ("ring_slots", ctypes.c_int32), ("donate_low", ctypes.c_int32),
                ("donate_depth", ctypes.c_int32),
                ("check_interval", ctypes.c_int32), ("no_reprune", ctypes.c_int32),
                ("single_wave", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("stack_classes", ctypes.c_int32), ("backoff_max", ctypes.c_int32),
                ("seg_lanes", ctypes.c_int32)]


class mcs_opts(ctypes.Structure):
    _fields_ = [("node_limit", ctypes.c_int64), ("time_limit_s", ctypes.c_double),
                ("tuning", ctypes.POINTER(mcs_tuning)),
                ("policy", ctypes.c_void_p), ("policy_depth", ctypes.c_int32),
                ("policy_mode", ctypes.c_int32), ("ordering", ctypes.c_int32),
                ("deadend_ratio", ctypes.c_int32), ("deadend_nodes", ctypes.c_int64)]


class mcs_result(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("optimal", ctypes.c_int32),
                ("map_g", ctypes.POINTER(ctypes.c_int32)),
                ("map_h", ctypes.POINTER(ctypes.c_int32)),
                ("nodes", ctypes.c_int64), ("t_best_s", ctypes.c_double),
                ("t_proof_s", ctypes.c_double)]


class mcs_stats(ctypes.Structure):
    _fields_ = [("nodes", ctypes.c_int64), ("batches", ctypes.c_int64),
                ("children", ctypes.c_int64), ("lane_slots", ctypes.c_int64),
                ("donations", ctypes.c_int64), ("pops", ctypes.c_int64),
                ("waves", ctypes.c_int32), ("blocks", ctypes.c_int32),
                ("lds_per_wave", ctypes.c_int32), ("stopped", ctypes.c_int32),
                ("kernel_ms", ctypes.c_double), ("busy_wave_s", ctypes.c_double),
                ("hbm_frames", ctypes.c_int64), ("stack_classes", ctypes.c_int32),
                ("max_stack_used", ctypes.c_int32), ("sleep_wave_s", ctypes.c_double),
                ("lds_bytes", ctypes.c_int64), ("node_classes", ctypes.c_int64)]


# (name, restype, argtypes) of every entry point declared in include/mcs.h
_P = ctypes.c_void_p
SIGNATURES = [
    ("mcs_plan_create", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(mcs_graph),
                                       ctypes.POINTER(mcs_graph), ctypes.POINTER(mcs_opts),
                                       ctypes.POINTER(_P)]),
    ("mcs_plan_workspace_size", ctypes.c_size_t, [_P]),
    ("mcs_plan_upload", ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    ("mcs_plan_run", ctypes.c_int, [_P, _P]),
    ("mcs_plan_results", ctypes.c_int, [_P, ctypes.POINTER(mcs_result), _P]),
    ("mcs_plan_stats", ctypes.c_int, [_P, ctypes.POINTER(mcs_stats)]),
    ("mcs_plan_set_goals", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32), _P]),
    ("mcs_plan_root_bounds", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32)]),
    ("mcs_plan_destroy", None, [_P]),
    ("mcs_solve_goals", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(mcs_graph),
                                       ctypes.POINTER(mcs_graph), ctypes.POINTER(mcs_opts),
                                       ctypes.c_int32, _P, ctypes.c_size_t, _P,
                                       ctypes.POINTER(mcs_result),
                                       ctypes.POINTER(ctypes.c_int32)]),
    ("mcs_workspace_size", ctypes.c_size_t, [ctypes.c_int32, ctypes.POINTER(mcs_graph),
                                             ctypes.POINTER(mcs_graph), ctypes.POINTER(mcs_opts)]),
    ("mcs_solve_batch", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(mcs_graph),
                                       ctypes.POINTER(mcs_graph), ctypes.POINTER(mcs_opts), _P,
                                       ctypes.c_size_t, _P, ctypes.POINTER(mcs_result)]),
    ("mcs_solve_batch_static", ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(mcs_graph),
                                              ctypes.POINTER(mcs_graph),
                                              ctypes.POINTER(mcs_opts), _P,
                                              ctypes.POINTER(mcs_result)]),
    ("mcs_solve", ctypes.c_int, [ctypes.POINTER(mcs_graph), ctypes.POINTER(mcs_graph),
                                 ctypes.POINTER(mcs_opts), _P, ctypes.c_size_t, _P,
                                 ctypes.POINTER(mcs_result)]),
    ("mcs_policy_param_count", ctypes.c_int32, []),
    ("mcs_policy_workspace_size", ctypes.c_size_t, [ctypes.c_int32]),
    ("mcs_policy_forward", ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P]),
    ("mcs_policy_grad", ctypes.c_int, [_P, _P, ctypes.c_int32, _P, _P, _P, _P,
                                       ctypes.c_size_t, _P]),
    ("mcs_policy_sgd", ctypes.c_int, [_P, _P, ctypes.c_float, _P]),
    ("mcs_policy_pack_half", ctypes.c_int, [_P, _P, _P]),
    ("mcs_status_string", ctypes.c_char_p, [ctypes.c_int]),
    ("mcs_last_error", ctypes.c_char_p, []),
]

_lib = None
_runtime = None


def hip_runtime():
    """Make the process's HIP runtime visible to libmcs.so, which links none of
    its own: torch's bundled libamdhip64 when torch is importable (so device
    memory, streams and kernels share one runtime), else the system one."""
    global _runtime
    if _runtime is None:
        path = None
        try:
            import torch
            cand = os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so")
            if os.path.exists(cand):
                path = cand
        except ImportError:
            pass
        if path is None:
            path = "libamdhip64.so.7"
        _runtime = ctypes.CDLL(path, mode=ctypes.RTLD_GLOBAL)
    return _runtime


def load():
    """Load libmcs.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1908_06418_amd.build.build() "
                "(hipcc, gfx950); the search has no CPU fallback")
        hip_runtime()
        lib = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib
