"""Input generators and the CSR builder (host only)."""
import os

import numpy as np
import pytest

import graphgen as gg


def test_c1_shape():
    g = gg.workload_c1()
    s = g.stats()
    assert s["N"] == 10000 and s["E"] == 80000 and s["dangling"] >= 500
    src, dst = g.edges()
    assert not np.any(src == dst)
    assert len(set(zip(src.tolist(), dst.tolist()))) == 80000


def test_deterministic_and_thread_independent(monkeypatch):
    a = gg.rmat(14, seed=3)
    monkeypatch.setenv("OMP_NUM_THREADS", "1")
    b = gg.rmat(14, seed=3)
    assert np.array_equal(a.off, b.off) and np.array_equal(a.idx, b.idx)
    c = gg.rmat(14, seed=4)
    assert not np.array_equal(a.idx[:1000], c.idx[:1000])


def test_csr_invariants():
    g = gg.rmat(13, seed=2)
    assert g.off[0] == 0 and np.all(np.diff(g.off) >= 0) and g.off[-1] == g.E
    for v in range(0, g.N, 97):
        row = g.idx[g.off[v]:g.off[v + 1]]
        assert np.all(np.diff(row) > 0)  # sorted, no duplicates
        assert not np.any(row == v)
    assert np.array_equal(np.bincount(g.idx, minlength=g.N), g.outdeg)


def test_rmat_skew_and_dangling():
    g = gg.rmat(16, seed=1)
    s = g.stats()
    assert 0.88 < s["E"] / (16 * 65536) < 0.95
    assert 0.3 < s["dangling"] / s["N"] < 0.5
    assert s["max_indeg"] > 2000


def test_non_power_of_two_rmat():
    g = gg.rmat(N=3000, edge_factor=8, seed=7)
    assert g.N == 3000 and g.idx.max() < 3000


def test_multigraph_kept_when_asked():
    g = gg.from_edges(3, [0, 0, 1, 2, 2], [1, 1, 1, 0, 0], dedupe=False, drop_self_loops=False)
    assert list(g.off) == [0, 2, 5, 5] and list(g.outdeg) == [2, 1, 2]


def test_relabel_roundtrip():
    g = gg.rmat(10, seed=1)
    p = gg.permutation(g.N, 5)
    h = gg.relabel(g, p)
    assert h.E == g.E and np.array_equal(np.sort(h.outdeg), np.sort(g.outdeg))
    assert np.array_equal(h.outdeg[p], g.outdeg)


def test_bad_ids_rejected():
    with pytest.raises(ValueError):
        gg.from_edges(3, [0, 5], [1, 1])


def test_specs_cover_the_ranges():
    specs = gg.many_graph_specs()
    assert len(specs) == 64
    Ns = [s["N"] for s in specs]
    assert min(Ns) >= 1000 and max(Ns) <= 1000000
    assert {s["alpha"] for s in specs} == {0.75, 0.85, 0.95}
    assert {s["norm"] for s in specs} == {1, 2, 3}
    assert gg.ALPHA_SWEEP[0] == 0.5 and gg.ALPHA_SWEEP[7] == 0.85 and gg.ALPHA_SWEEP[-1] == 1.0
    assert len(gg.tau_sweep_21()) == 21


def test_load_mtx_general_and_symmetric(tmp_path):
    gen = tmp_path / "g.mtx"
    gen.write_text("%%MatrixMarket matrix coordinate pattern general\n% a comment\n4 4 5\n"
                   "1 2\n2 3\n3 1\n3 4\n3 4\n")          # one duplicate entry
    g = gg.load_mtx(str(gen))
    assert g.N == 4 and g.E == 4
    src, dst = g.edges()
    assert sorted(zip(src.tolist(), dst.tolist())) == [(0, 1), (1, 2), (2, 0), (2, 3)]
    assert g.outdeg.tolist() == [1, 1, 2, 0]
    sym = tmp_path / "s.mtx"
    sym.write_text("%%MatrixMarket matrix coordinate real symmetric\n3 3 3\n2 1 1.5\n3 2 -1\n3 3 7\n")
    h = gg.load_mtx(str(sym))                             # both directions; the diagonal is a self-loop
    src, dst = h.edges()
    assert sorted(zip(src.tolist(), dst.tolist())) == [(0, 1), (1, 0), (1, 2), (2, 1)]
    bad = tmp_path / "b.mtx"
    bad.write_text("%%MatrixMarket matrix array real general\n2 2\n1\n2\n3\n4\n")
    with pytest.raises(ValueError):
        gg.load_mtx(str(bad))
    out = tmp_path / "o.mtx"
    out.write_text("%%MatrixMarket matrix coordinate pattern general\n2 2 1\n3 1\n")
    with pytest.raises(ValueError):
        gg.load_mtx(str(out))


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def test_committed_mtx_fixtures():
    # the two hand-written MatrixMarket files the GPU test solves: structure read off by hand
    g = gg.load_mtx(os.path.join(GOLDEN, "small_general.mtx"))
    assert g.N == 12 and g.E == 19                        # 21 entries - 1 duplicate - 1 self-loop
    assert g.outdeg.tolist() == [2, 2, 2, 2, 0, 2, 2, 2, 0, 2, 3, 0]
    assert [v for v in range(12) if g.outdeg[v] == 0] == [4, 8, 11]   # 5, 9, 12 in the file
    assert g.indeg[11] == 0 and g.indeg[6] == 1           # 12 isolated; 7 only from 6
    src, dst = g.edges()
    assert (2, 3) in set(zip(src.tolist(), dst.tolist())) and (6, 6) not in set(zip(src.tolist(), dst.tolist()))
    h = gg.load_mtx(os.path.join(GOLDEN, "small_symmetric.mtx"))
    assert h.N == 8 and h.E == 16                         # 8 undirected edges, both ways
    assert np.array_equal(h.outdeg, h.indeg) and h.outdeg.tolist() == [3, 2, 3, 3, 2, 2, 1, 0]


def test_degree_order_is_a_permutation_by_decreasing_out_degree():
    g = gg.rmat(10, seed=4)
    p = gg.degree_order(g)
    assert sorted(p.tolist()) == list(range(g.N))
    inv = np.empty(g.N, dtype=np.int64)
    inv[p] = np.arange(g.N)
    d = g.outdeg[inv]                      # out-degree of new id 0, 1, ...
    assert np.all(np.diff(d.astype(np.int64)) <= 0)
    # ties keep the original order
    for k in range(g.N - 1):
        if d[k] == d[k + 1]:
            assert inv[k] < inv[k + 1]
    h = gg.relabel(g, p)
    assert np.array_equal(h.outdeg[p], g.outdeg)
