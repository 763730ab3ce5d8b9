"""The C ABI library without a GPU: it loads, exports every entry point that
include/mcs.h declares, and rejects malformed input before any device work."""
import ctypes
import os
import re

import pytest

import mcs_instances as mi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(mcs_\w+)\s*\(", src))
    return names


def test_exports_every_declared_symbol(mcs_lib):
    declared = _declared()
    assert {"mcs_solve", "mcs_solve_batch", "mcs_plan_create", "mcs_plan_run",
            "mcs_workspace_size", "mcs_status_string"} <= declared
    for name in sorted(declared):
        assert hasattr(mcs_lib, name), name


def test_binding_covers_header(mcs_lib):
    from paper_1908_06418_amd import _abi
    assert {n for n, _, _ in _abi.SIGNATURES} == _declared()


def test_struct_sizes_match_header():
    """ctypes mirrors have the C layout (compiled probe of include/mcs.h)."""
    import subprocess
    import tempfile
    from paper_1908_06418_amd import _abi
    src = r'''
#include <stdio.h>
#include "mcs.h"
int main(void) { printf("%zu %zu %zu %zu %zu\n", sizeof(mcs_graph), sizeof(mcs_tuning),
  sizeof(mcs_opts), sizeof(mcs_result), sizeof(mcs_stats)); return 0; }
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "p.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "p")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    assert sizes == [ctypes.sizeof(_abi.mcs_graph), ctypes.sizeof(_abi.mcs_tuning),
                     ctypes.sizeof(_abi.mcs_opts), ctypes.sizeof(_abi.mcs_result),
                     ctypes.sizeof(_abi.mcs_stats)]


def _create(pairs):
    from paper_1908_06418_amd import Plan
    return Plan(pairs)


def _status(exc):
    return exc.value.status


def test_status_strings(mcs_lib):
    for s in (0, 1, -1, -2, -3, -4, -5, -6):
        assert mcs_lib.mcs_status_string(s)
    assert b"unknown" in mcs_lib.mcs_status_string(42)


@pytest.mark.parametrize("mutate,status", [
    (lambda G, H: (dict(G, n=255, rows=[0] * 255), H), -2),
    (lambda G, H: (dict(G, n=-1), H), -1),
    (lambda G, H: (dict(G, rows=[G["rows"][0] | 1] + G["rows"][1:]), H), -1),   # self loop
    (lambda G, H: (dict(G, rows=[G["rows"][0] | (1 << 20)] + G["rows"][1:]), H), -1),  # bit >= n
    (lambda G, H: (dict(G, rows=[G["rows"][0] ^ 2] + G["rows"][1:]), H), -1),   # asymmetric
    (lambda G, H: (dict(G, directed=True), H), -1),                             # mixed directed
    (lambda G, H: (dict(G, label=[0] * G["n"]), H), -1),                        # label on one side
])
def test_validation_errors(mcs_lib, mutate, status):
    from paper_1908_06418_amd import McsError
    G = mi.er_graph(12, 0.4, 1)
    H = mi.er_graph(12, 0.4, 2)
    G, H = mutate(G, H)
    with pytest.raises(McsError) as e:
        _create([(G, H)])
    assert _status(e) == status
    assert mcs_lib.mcs_last_error()


def _flip(g, i, j):
    rows = list(g["rows"])
    rows[i] ^= 1 << j
    return dict(g, rows=rows)


@pytest.mark.parametrize("mutate", [
    lambda G: _flip(G, 0, 110),    # a bit at or above n, in the second word of a row
    lambda G: _flip(G, 90, 90),    # a self loop in the second word
    lambda G: _flip(G, 3, 80),     # asymmetric in the second word
    lambda G: _flip(G, 80, 3),     # asymmetric in the first word of a wide row
])
def test_validation_errors_two_word_rows(mcs_lib, mutate):
    """Graphs of 65..128 vertices have two 64-bit words per row."""
    from paper_1908_06418_amd import McsError
    G = mi.er_graph(100, 0.1, 1)
    H = mi.er_graph(100, 0.1, 2)
    _create([(G, H)]).close()
    with pytest.raises(McsError) as e:
        _create([(mutate(G), H)])
    assert _status(e) == -1
    assert mcs_lib.mcs_last_error()


@pytest.mark.parametrize("mutate", [
    lambda G: _flip(G, 0, 230),     # a bit at or above n, in the fourth word of a row
    lambda G: _flip(G, 150, 150),   # a self loop in the third word
    lambda G: _flip(G, 199, 199),   # a self loop in the fourth word
    lambda G: _flip(G, 3, 190),     # asymmetric in the third word
    lambda G: _flip(G, 195, 3),     # asymmetric in the first word of a four-word row
])
def test_validation_errors_four_word_rows(mcs_lib, mutate):
    """Graphs of 193..254 vertices have four 64-bit words per row."""
    from paper_1908_06418_amd import McsError
    G = mi.er_graph(200, 0.05, 1)
    H = mi.er_graph(200, 0.05, 2)
    _create([(G, H)]).close()
    with pytest.raises(McsError) as e:
        _create([(mutate(G), H)])
    assert _status(e) == -1
    assert mcs_lib.mcs_last_error()


def test_largest_graphs_accepted(mcs_lib):
    """254 vertices, the paper's limit, make a plan (with 3- and 4-word rows
    in one batch); 255 do not."""
    from paper_1908_06418_amd import McsError
    _create([(mi.er_graph(254, 0.05, 1), mi.er_graph(150, 0.05, 2)),
             (mi.empty_graph(254), mi.complete_graph(254))]).close()
    with pytest.raises(McsError) as e:
        _create([(mi.empty_graph(255), mi.empty_graph(3))])
    assert _status(e) == -2


def test_two_word_rows_marshalled_low_word_first():
    from paper_1908_06418_amd import _Marshal
    g = mi.er_graph(100, 0.2, 3)
    m = _Marshal([(g, g)])
    words = m.keep[0]
    assert words.size == 2 * 100
    for i, r in enumerate(g["rows"]):
        assert int(words[2 * i]) | (int(words[2 * i + 1]) << 64) == r
    small = _Marshal([(mi.er_graph(64, 0.2, 3), mi.er_graph(64, 0.2, 4))])
    assert small.keep[0].size == 64
    for n, rw in ((150, 3), (254, 4)):
        g = mi.er_graph(n, 0.2, 3)
        words = _Marshal([(g, g)]).keep[0]
        assert words.size == rw * n
        for i, r in enumerate(g["rows"]):
            assert sum(int(words[rw * i + k]) << (64 * k) for k in range(rw)) == r


def test_wide_plan_sizes(mcs_lib):
    """128-bit rows: the plan keeps a capped class stack and larger records."""
    from paper_1908_06418_amd import Plan, workspace_size
    pairs = [(mi.er_graph(128, 0.3, 5), mi.er_graph(120, 0.3, 6))]
    narrow = [(mi.er_graph(64, 0.3, 5), mi.er_graph(60, 0.3, 6))]
    assert workspace_size(pairs) > workspace_size(narrow) > 0
    widest = [(mi.er_graph(254, 0.3, 5), mi.er_graph(200, 0.3, 6))]
    assert workspace_size(widest) > workspace_size(pairs)
    Plan(pairs).close()


def test_policy_rejected_above_64_vertices(mcs_lib):
    from paper_1908_06418_amd import _abi, _Marshal
    m = _Marshal([(mi.er_graph(70, 0.3, 1), mi.er_graph(70, 0.3, 2))])
    o = _abi.mcs_opts()
    o.policy = 4096  # (never dereferenced: the plan is refused first)
    o.policy_depth = 2
    h = ctypes.c_void_p()
    assert mcs_lib.mcs_plan_create(1, m.G, m.H, ctypes.byref(o), ctypes.byref(h)) == \
        _abi.MCS_E_INVALID
    assert b"64" in mcs_lib.mcs_last_error()


def test_single_wave_plan_at_128_vertices(mcs_lib):
    """With 128-bit rows every wavefront's class stack lives in HBM, so one
    wavefront can hold the whole worst case (8256 classes at 128 vertices)."""
    from paper_1908_06418_amd import Plan
    pairs = [(mi.er_graph(128, 0.3, 5), mi.er_graph(128, 0.3, 6))]
    Plan(pairs, tuning={"single_wave": 1}).close()


def test_null_and_count_errors(mcs_lib):
    from paper_1908_06418_amd import _abi
    h = ctypes.c_void_p()
    assert mcs_lib.mcs_plan_create(0, None, None, None, ctypes.byref(h)) == _abi.MCS_E_INVALID
    assert mcs_lib.mcs_plan_create(1, None, None, None, ctypes.byref(h)) == _abi.MCS_E_INVALID
    res = (_abi.mcs_result * 1)()
    res[0].size = 7
    assert mcs_lib.mcs_solve(None, None, None, None, 0, None, res) == _abi.MCS_E_INVALID
    assert res[0].size == -1


def test_upload_rejects_small_workspace(mcs_lib):
    from paper_1908_06418_amd import _abi
    from paper_1908_06418_amd import _Marshal
    m = _Marshal([(mi.er_graph(10, 0.3, 1), mi.er_graph(10, 0.3, 2))])
    h = ctypes.c_void_p()
    assert mcs_lib.mcs_plan_create(1, m.G, m.H, None, ctypes.byref(h)) == 0
    need = mcs_lib.mcs_plan_workspace_size(h)
    assert need > 0
    assert mcs_lib.mcs_plan_upload(h, None, need, None) == _abi.MCS_E_WORKSPACE
    assert mcs_lib.mcs_plan_upload(h, ctypes.c_void_p(256), need - 1, None) == _abi.MCS_E_WORKSPACE
    assert mcs_lib.mcs_plan_upload(h, ctypes.c_void_p(257), need, None) == _abi.MCS_E_WORKSPACE
    assert mcs_lib.mcs_plan_run(h, None) == _abi.MCS_E_WORKSPACE
    mcs_lib.mcs_plan_destroy(h)


def test_workspace_size_grows_with_batch(mcs_lib):
    from paper_1908_06418_amd import workspace_size
    one = workspace_size(mi.pairs_c4(1))
    many = workspace_size(mi.pairs_c4(64))
    assert 0 < one < many


def test_product_package_never_imports_oracle():
    pkg = os.path.join(ROOT, "paper_1908_06418_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in src and "from oracle" not in src, fn
                assert "mcsplit_oracle" not in src and "liboracle" not in src, fn


def test_mixed_batch_accepted(mcs_lib):
    """Directed and undirected, labelled and unlabelled pairs share one call."""
    pairs = [(mi.er_graph(12, 0.3, 1), mi.er_graph(12, 0.3, 2)),
             (mi.er_graph(12, 0.3, 3, directed=True), mi.er_graph(12, 0.3, 4, directed=True)),
             (mi.er_graph(12, 0.3, 5, labelled=True), mi.er_graph(12, 0.3, 6, labelled=True))]
    p = _create(pairs)
    assert p.workspace_bytes > 0
    p.close()


def test_root_bounds_host(mcs_lib):
    """Eq. 1 at the root: min(nG, nH) unlabelled; sum over shared labels of
    min(counts) labelled."""
    from paper_1908_06418_amd import _Marshal
    G = mi.er_graph(10, 0.3, 1)
    H = mi.er_graph(7, 0.3, 2)
    Gl = dict(G, label=[0, 0, 0, 1, 1, 2, 2, 2, 2, 3])
    Hl = dict(H, label=[0, 1, 1, 1, 2, 5, 5])
    m = _Marshal([(G, H), (Gl, Hl), (mi.empty_graph(0), H)])
    h = ctypes.c_void_p()
    assert mcs_lib.mcs_plan_create(3, m.G, m.H, None, ctypes.byref(h)) == 0
    out = (ctypes.c_int32 * 3)()
    assert mcs_lib.mcs_plan_root_bounds(h, out) == 0
    assert list(out) == [7, 1 + 2 + 1, 0]
    mcs_lib.mcs_plan_destroy(h)


def test_ordering_option_validated(mcs_lib):
    """mcs_opts.ordering takes 0 (degree), 1 (block-triangular) or 2 (both,
    as a portfolio: two search instances per pair, so a larger workspace);
    anything else is rejected before any device work."""
    from paper_1908_06418_amd import _Marshal, _abi, _opts
    m = _Marshal([(mi.er_graph(10, 0.3, 1), mi.er_graph(10, 0.3, 2))] * 3)
    h = ctypes.c_void_p()
    sizes = {}
    for ordering, status in ((0, _abi.MCS_OK), (1, _abi.MCS_OK), (2, _abi.MCS_OK),
                             (3, _abi.MCS_E_INVALID), (-1, _abi.MCS_E_INVALID)):
        o, _t = _opts(0, 0.0, None)
        o.ordering = ordering
        st = mcs_lib.mcs_plan_create(3, m.G, m.H, ctypes.byref(o), ctypes.byref(h))
        assert st == status, (ordering, st)
        if st == _abi.MCS_OK:
            sizes[ordering] = mcs_lib.mcs_plan_workspace_size(h)
            mcs_lib.mcs_plan_destroy(h)
    assert sizes[0] == sizes[1] < sizes[2]


def test_deadend_and_goal_options_validated(mcs_lib):
    """Negative dead-end thresholds are rejected; goal strategies 2 and 3
    need deadend_nodes > 0; strategies outside 0..3 are rejected (all before
    any device work, with every result size set to -1)."""
    from paper_1908_06418_amd import _Marshal, _abi, _opts
    m = _Marshal([(mi.er_graph(10, 0.3, 1), mi.er_graph(10, 0.3, 2))])
    h = ctypes.c_void_p()
    for nodes, ratio, status in ((0, 0, _abi.MCS_OK), (100, 2, _abi.MCS_OK),
                                 (-1, 0, _abi.MCS_E_INVALID), (100, -2, _abi.MCS_E_INVALID)):
        o, _t = _opts(0, 0.0, None, deadend_nodes=nodes, deadend_ratio=ratio)
        st = mcs_lib.mcs_plan_create(1, m.G, m.H, ctypes.byref(o), ctypes.byref(h))
        assert st == status, (nodes, ratio, st)
        if st == _abi.MCS_OK:
            mcs_lib.mcs_plan_destroy(h)
    res = (_abi.mcs_result * 1)()
    for strategy, nodes in ((2, 0), (3, 0), (4, 100), (-1, 100)):
        o, _t = _opts(0, 0.0, None, deadend_nodes=nodes)
        res[0].size = 7
        st = mcs_lib.mcs_solve_goals(1, m.G, m.H, ctypes.byref(o), strategy, None, 0, None, res,
                                     None)
        assert st == _abi.MCS_E_INVALID, (strategy, st)
        assert res[0].size == -1


def test_root_bounds_host_beyond_64(mcs_lib):
    """Eq. 1 at the root on graphs with two-word rows: min(nG, nH)
    unlabelled; with labels, the sum over shared labels of min(counts),
    including labels whose vertices sit only above vertex 64."""
    from paper_1908_06418_amd import _Marshal
    G = mi.er_graph(128, 0.2, 11)
    H = mi.er_graph(90, 0.2, 12)
    Gl = dict(G, label=[0] * 64 + [1] * 60 + [2] * 4)
    Hl = dict(H, label=[1] * 10 + [2] * 70 + [3] * 10)
    m = _Marshal([(G, H), (Gl, Hl), (mi.empty_graph(70), mi.empty_graph(100))])
    h = ctypes.c_void_p()
    assert mcs_lib.mcs_plan_create(3, m.G, m.H, None, ctypes.byref(h)) == 0
    out = (ctypes.c_int32 * 3)()
    assert mcs_lib.mcs_plan_root_bounds(h, out) == 0
    assert list(out) == [90, min(60, 10) + min(4, 70), 70]
    mcs_lib.mcs_plan_destroy(h)
