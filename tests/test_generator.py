"""The seeded instance generator (shared input module, no search arithmetic)."""
import numpy as np

import mcs_instances as mi


def test_splitmix64_published_vector():
    # splitmix64 seeded with 0 (Steele, Lea and Flood; Vigna's reference code)
    z = mi.splitmix64(0, 3)
    assert [int(x) for x in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_uniforms_in_unit_interval():
    u = mi.uniforms(12345, 10000)
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.02


def test_deterministic_and_seed_sensitive():
    a = mi.er_graph(30, 0.3, mi.stream_seed(2, 5, 0))
    b = mi.er_graph(30, 0.3, mi.stream_seed(2, 5, 0))
    c = mi.er_graph(30, 0.3, mi.stream_seed(2, 5, 1))
    assert a == b and a != c


def test_undirected_simple_and_density():
    edges = 0
    for i in range(20):
        g = mi.er_graph(40, 0.3, mi.stream_seed(9, i, 0))
        m = mi.to_matrix(g)
        assert (m == m.T).all() and m.diagonal().sum() == 0
        edges += m.sum() // 2
    p_hat = edges / (20 * 40 * 39 / 2)
    assert abs(p_hat - 0.3) < 0.02


def test_directed_independent_arcs():
    arcs = recip = 0
    for i in range(20):
        g = mi.er_graph(50, 0.1, mi.stream_seed(9, i, 0), directed=True)
        m = mi.to_matrix(g)
        assert m.diagonal().sum() == 0
        arcs += m.sum()
        recip += (m & m.T).sum() // 2
    pairs = 20 * 50 * 49
    assert abs(arcs / pairs - 0.1) < 0.01
    # independent draws: P(both arcs) = p^2
    assert abs(recip / (pairs / 2) - 0.01) < 0.005


def test_labels_range():
    assert [mi.label_count(n) for n in (40, 50, 60)] == [14, 17, 20]
    g = mi.er_graph(60, 0.1, 77, directed=True, labelled=True)
    assert len(g["label"]) == 60 and min(g["label"]) >= 0 and max(g["label"]) < 20


def test_workload_shapes():
    c2 = mi.pairs_c2()
    assert len(c2) == 180
    assert {G["n"] for G, _ in c2} == {30, 35, 40}
    assert all(G["n"] == H["n"] for G, H in c2)
    c3 = mi.pairs_c3(seeds=range(2))
    assert len(c3) == 6 and all(G["directed"] and G["label"] for G, _ in c3)
    shapes = [mi.c4_shape(i) for i in range(4096)]
    ns = [n for n, _ in shapes]
    ps = [p for _, p in shapes]
    assert min(ns) == 10 and max(ns) == 35
    assert min(ps) >= 0.05 and max(ps) < 0.5
    c5 = [mi.c5_shape(i) for i in range(1024)]
    assert all(35 <= n <= 50 for n, _ in c5)
    assert sum(1 for _, p in c5 if p == 0.2) == 512
    tr = [mi.c5_shape(i, train=True) for i in range(100)]
    assert all(20 <= n <= 30 for n, _ in tr)


def test_workload_w_shape():
    """The workload beyond 64 vertices: 40 directed labelled pairs, 20 of 80
    and 20 of 100 vertices, labels over ceil(0.33 n) values, rows as Python
    ints with bits above 63 in use."""
    w = mi.pairs_w()
    assert len(w) == 40
    assert [G["n"] for G, _ in w] == [80] * 20 + [100] * 20
    assert all(G["n"] == H["n"] and G["directed"] and H["directed"] for G, H in w)
    for G, H in w:
        for g in (G, H):
            assert max(g["label"]) < mi.label_count(g["n"])
            assert all(r >> g["n"] == 0 for r in g["rows"])
            assert all(not (r >> i) & 1 for i, r in enumerate(g["rows"]))
    assert any(r >> 64 for G, _ in w for r in G["rows"])
    assert mi.pairs_w(ns=(100,), seeds=range(1)) == [w[20]]


def test_bench_accounting_covers_every_word_size():
    """bench.py prices every row width and direction it can meet, and every
    workload it names resolves to pairs of the width it says."""
    import bench
    # the per-class counts written out in bench.py: 22 / 50 lane-ops at 32
    # bits (undirected / directed), the word-wise part scaling with the word
    assert bench.ops_per_class(4, False) == 22 and bench.ops_per_class(4, True) == 50
    assert bench.ops_per_class(8, False) == 38 and bench.ops_per_class(8, True) == 88
    assert bench.ops_per_class(16, False) == 70 and bench.ops_per_class(16, True) == 164
    wl = bench.workloads()
    assert {"c1", "c2", "c2_n30", "c3", "c4", "c4_1024", "w"} <= set(wl)
    assert "128-bit" in wl["w"][0]
    for name, t in bench.TRAFFIC.items():
        assert name in wl and t["bytes"] > 0 and len(t["kernel_code_hash"]) == 16


def test_report_helper_writes_only_where_asked(tmp_path, monkeypatch):
    from _report import write_report
    monkeypatch.delenv("MCS_REPORT_DIR", raising=False)
    write_report("r.json", {"a": 1})
    assert not (tmp_path / "r.json").exists()
    monkeypatch.setenv("MCS_REPORT_DIR", str(tmp_path / "out"))
    write_report("r.json", {"a": 1})
    import json
    assert json.loads((tmp_path / "out" / "r.json").read_text()) == {"a": 1}
