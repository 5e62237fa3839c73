"""Parity of the HIP pull PageRank (pr_pull through the C ABI) with the CPU oracle.

FP64 bar (tests/parity.py): ranks within 1e-12 in L1 of the oracle's after the same number of
updates, traces row by row, and the same iteration count except at a tie that the measured
distance of the two sides explains; on such a tie the oracle is run again for exactly the GPU's
number of updates and the ranks are still compared.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
from parity import TRACE_ATOL, check_fp64_result, check_mixed_result  # noqa: F401

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pr():
    import paper_2108_02997_amd as pr
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return pr


@pytest.fixture(scope="module")
def ctx(pr):
    c = pr.Context(0)
    yield c
    c.close()


def dev(pr, g):
    return pr.DeviceGraph.from_host(g)


def oracle_run(g, **kw):
    return oracle.pagerank_graph(g, trace=True, **kw)


def check_fp64(pr, ctx, g, alpha=0.85, tau=1e-6, norm=1, max_iter=500, init=None, dg=None):
    dg = dg or dev(pr, g)
    init_t = None if init is None else torch.from_numpy(np.asarray(init, dtype=np.float64)).cuda()
    res = pr.pull(ctx, dg, alpha=alpha, tau=tau, norm=norm, max_iter=max_iter, init=init_t, trace=True)
    ref = check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], alpha, tau, norm,
                            max_iter, init=init, gpu_trace=res["trace"].cpu().numpy())
    return res, ref


# ------------------------------------------------------------------ the small configuration

def test_c1_parity_all_norms(pr, ctx):
    g = gg.workload_c1()
    dg = dev(pr, g)
    for norm in (1, 2, 3):
        for tau in (1e-3, 1e-6, 1e-10):
            check_fp64(pr, ctx, g, tau=tau, norm=norm, dg=dg)


def test_c1_headline_setting(pr, ctx):
    g = gg.workload_c1()
    res, ref = check_fp64(pr, ctx, g, alpha=0.85, tau=1e-6, norm=1)
    assert res["status"] == 0 and res["iterations"] == ref["iterations"]


@pytest.mark.parametrize("alpha", [0.0, 0.5, 0.95, 1.0])
def test_alpha_range(pr, ctx, alpha):
    check_fp64(pr, ctx, gg.rmat(13, seed=3), alpha=alpha, tau=1e-10, norm=3)


# ------------------------------------------------------------------ tiny graphs and edge cases

@pytest.mark.parametrize("make", [lambda: gg.cycle(7), lambda: gg.complete(40), lambda: gg.edgeless(9),
                                  lambda: gg.edgeless(1), lambda: gg.in_star(3), lambda: gg.out_star(6),
                                  lambda: gg.in_star(1), lambda: gg.cycle(2)])
def test_tiny_zoo(pr, ctx, make):
    g = make()
    for norm in (1, 2, 3):
        check_fp64(pr, ctx, g, tau=1e-12, norm=norm)


def test_two_triangles_from_given_start(pr, ctx):
    g = gg.two_triangles()
    init = [1 / 3, 1 / 3, 1 / 3, 0, 0, 0]
    res, ref = check_fp64(pr, ctx, g, alpha=0.85, tau=1e-6, norm=1, init=init)
    assert res["iterations"] == 75


@pytest.mark.parametrize("seed", range(8))
def test_random_multigraphs(pr, ctx, seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(1, 300))
    g = gg.random_small(N, int(rng.integers(0, 6 * N)), seed, dedupe=False, self_loops=True)
    check_fp64(pr, ctx, g, alpha=float(rng.uniform(0, 1)), tau=1e-11, norm=int(rng.integers(1, 4)))


def test_hub_segments_and_mid_rows(pr, ctx):
    # in-degrees spanning lane rows (<=32), wave rows (33..1024), one-segment long rows
    # (1025..8192) and hubs of several 8192-entry segments, with ragged ends
    rng = np.random.default_rng(5)
    N = 40000
    src, dst = [], []
    for v, deg in ((0, 5000), (17, 1025), (18, 1024), (19, 2049), (300, 40), (301, 33), (302, 32), (9999, 4097),
                   (20000, 8192), (20001, 8193), (20002, 30001), (39999, 16384)):
        s = rng.choice(N, size=deg, replace=False)
        src.extend(s.tolist())
        dst.extend([v] * deg)
    s = rng.integers(0, N, 60000)
    d = rng.integers(0, N, 60000)
    src.extend(s.tolist())
    dst.extend(d.tolist())
    g = gg.from_edges(N, src, dst)
    for norm in (1, 3):
        check_fp64(pr, ctx, g, tau=1e-11, norm=norm)


def test_rmat_several_tiles(pr, ctx):
    g = gg.rmat(16, seed=11)
    for norm in (1, 2, 3):
        check_fp64(pr, ctx, g, tau=1e-10, norm=norm)


def test_relabelled_rmat(pr, ctx):
    g = gg.relabel(gg.rmat(15, seed=2), gg.permutation(1 << 15, 3))
    check_fp64(pr, ctx, g, tau=1e-9, norm=2)


@pytest.mark.parametrize("make", [lambda: gg.rmat(14, seed=5), gg.workload_c1, lambda: gg.edgeless(3),
                                  lambda: gg.out_star(6), gg.two_triangles, lambda: gg.complete(100)])
def test_degree_relabel_on_the_device(pr, ctx, make):
    # pr_relabel: the permutation is the host's definition (decreasing out-degree, ties by id), the
    # relabelled CSR the host's relabelling, and ranks solved on it map back to the oracle's on the
    # original graph
    g = make()
    dg = dev(pr, g)
    h, perm = dg.relabelled(ctx)
    p_ref = gg.degree_order(g)
    assert np.array_equal(perm.cpu().numpy(), p_ref)
    ref = gg.relabel(g, p_ref)
    assert np.array_equal(h.off.cpu().numpy(), ref.off) and np.array_equal(h.outdeg.cpu().numpy(), ref.outdeg)
    # rows in ascending source order on both sides: the same arrays
    assert np.array_equal(h.idx.cpu().numpy(), ref.idx)
    res = pr.pull(ctx, h, alpha=0.85, tau=1e-10, norm=1)
    back = pr.unpermute(ctx, perm, res["ranks"])
    check_fp64_result(g, back.cpu().numpy(), res["iterations"], res["converged"], 0.85, 1e-10, 1, 500)


@pytest.mark.parametrize("name", ["small_general.mtx", "small_symmetric.mtx"])
def test_matrix_market_input(pr, ctx, name):
    # a MatrixMarket file (the paper's input format) loaded by graphgen.load_mtx and solved on the
    # GPU: every norm, tight tolerances, against the oracle on the same loaded graph
    import os
    g = gg.load_mtx(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name))
    dg = dev(pr, g)
    for norm in (1, 2, 3):
        for alpha in (0.5, 0.85, 1.0):
            res, ref = check_fp64(pr, ctx, g, alpha=alpha, tau=1e-12, norm=norm, dg=dg)
            assert res["iterations"] == ref["iterations"]


def test_max_iter_halt(pr, ctx):
    g = gg.workload_c1()
    dg = dev(pr, g)
    res = pr.pull(ctx, dg, alpha=0.85, tau=0.0, norm=1, max_iter=9)
    ref = oracle.pagerank_graph(g, alpha=0.85, tau=0.0, norm=1, max_iter=9)
    assert res["status"] == pr.PR_NOT_CONVERGED and not res["converged"] and res["iterations"] == 9
    assert np.abs(res["ranks"].cpu().numpy() - ref["ranks"]).sum() <= 1e-12


def test_resume_continues_the_sequence(pr, ctx):
    g = gg.rmat(14, seed=4)
    dg = dev(pr, g)
    part = oracle.pagerank_graph(g, alpha=0.85, tau=0.0, norm=1, max_iter=5)
    full = oracle.pagerank_graph(g, alpha=0.85, tau=0.0, norm=1, max_iter=12)
    init = torch.from_numpy(part["ranks"]).cuda()
    res = pr.pull(ctx, dg, alpha=0.85, tau=0.0, norm=1, max_iter=7, init=init)
    assert np.abs(res["ranks"].cpu().numpy() - full["ranks"]).sum() <= 1e-12


def test_ranks_may_alias_init(pr, ctx):
    g = gg.rmat(12, seed=8)
    dg = dev(pr, g)
    ref = oracle.pagerank_graph(g, alpha=0.85, tau=1e-9, norm=1)
    buf = torch.full((g.N,), 1.0 / g.N, dtype=torch.float64, device="cuda")
    res = pr.pull(ctx, dg, alpha=0.85, tau=1e-9, norm=1, init=buf, ranks=buf)
    assert res["iterations"] == ref["iterations"]
    assert np.abs(buf.cpu().numpy() - ref["ranks"]).sum() <= 1e-12


def test_bitwise_repeatable(pr, ctx):
    g = gg.rmat(15, seed=6)
    dg = dev(pr, g)
    a = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1)["ranks"].clone()
    b = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1)["ranks"].clone()
    assert torch.equal(a, b)


def test_loop_modes_and_grids_agree(pr, ctx):
    g = gg.rmat(14, seed=12)
    dg = dev(pr, g)
    ref = oracle.pagerank_graph(g, alpha=0.85, tau=1e-10, norm=2)
    try:
        for loop, grid, chunk in ((1, 2048, 8), (0, 7, 4), (0, 64, 16), (1, 1, 2), (0, 16384, 8)):
            ctx.set_option("loop", loop)
            ctx.set_option("grid", grid)
            ctx.set_option("chunk", chunk)
            res = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=2)
            assert res["iterations"] == ref["iterations"]
            assert np.abs(res["ranks"].cpu().numpy() - ref["ranks"]).sum() <= 1e-12
    finally:
        ctx.set_option("loop", 0)
        ctx.set_option("grid", 0)
        ctx.set_option("chunk", 16)


def test_prepare_inside_workspace(pr, ctx):
    g = gg.rmat(13, seed=1)
    dg = dev(pr, g)
    ranks = torch.empty(g.N, dtype=torch.float64, device="cuda")
    ws = torch.empty(ctx.lib.pr_workspace_bytes(g.N, g.E, 0, 1), dtype=torch.uint8, device="cuda")
    st, res = pr.pr_pull(ctx, dg, 0.85, 1e-8, 1, 500, 0, None, ranks, None, ws, use_prep=False)
    ref = oracle.pagerank_graph(g, alpha=0.85, tau=1e-8, norm=1)
    assert res["iterations"] == ref["iterations"]
    assert np.abs(ranks.cpu().numpy() - ref["ranks"]).sum() <= 1e-12


# ------------------------------------------------------------------ errors

def test_argument_errors(pr, ctx):
    g = gg.cycle(5)
    dg = dev(pr, g)
    for kw in (dict(alpha=1.5), dict(alpha=-0.5), dict(tau=-1.0), dict(tau=float("nan")), dict(norm=0),
               dict(norm=4), dict(max_iter=0), dict(precision=7)):
        args = dict(alpha=0.85, tau=1e-6, norm=1, max_iter=10, precision=0)
        args.update(kw)
        with pytest.raises(pr.PrError) as ei:
            pr.pull(ctx, dg, **args)
        assert ei.value.status == -1
    ranks = torch.empty(5, dtype=torch.float64, device="cuda")
    tiny = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(pr.PrError) as ei:
        pr.pr_pull(ctx, dg, 0.85, 1e-6, 1, 10, 0, None, ranks, None, tiny)
    assert ei.value.status == -2


def test_validate_graph(pr, ctx):
    g = gg.rmat(12, seed=2)
    dev(pr, g).validate(ctx)
    bad_deg = gg.Graph(g.N, g.off.copy(), g.idx.copy(), g.outdeg.copy())
    bad_deg.outdeg[5] += 1
    bad_idx = gg.Graph(g.N, g.off.copy(), g.idx.copy(), g.outdeg.copy())
    bad_idx.idx[10] = g.N + 3
    bad_off = gg.Graph(g.N, g.off.copy(), g.idx.copy(), g.outdeg.copy())
    bad_off.off[100] = bad_off.off[101] + 1
    for b in (bad_deg, bad_idx, bad_off):
        with pytest.raises(pr.PrError) as ei:
            dev(pr, b).validate(ctx)
        assert ei.value.status == -4


def test_prep_mismatch_rejected(pr, ctx):
    a = dev(pr, gg.rmat(10, seed=1)).prepare(ctx)
    b = dev(pr, gg.rmat(11, seed=1))
    b.prep = a.prep
    with pytest.raises(pr.PrError):
        pr.pull(ctx, b)


def test_autotune_then_parity(pr, ctx):
    g = gg.rmat(15, seed=31)
    dg = dev(pr, g)
    t = dg.autotune(ctx)
    assert t["candidates"] == 45 + 12 and t["mid_deg"] in (8, 16, 32, 64, 128) and t["grid"] >= 1
    assert (t["tile"], t["rows"]) in ((1024, 512), (512, 256), (256, 128))
    assert (t["tile_batch"], t["rows_batch"]) in ((256, 128), (128, 64))
    assert t["mid_deg_batch"] in (16, 32, 64) and t["grid_batch_factor"] in (1, 2)
    assert t["best_us"] <= t["default_us"] and t["best_batch_us"] <= t["default_batch_us"]
    print("autotune:", t)
    # the single-vector solve, the many-graph launch and the K-column batch on the tuned settings
    res, ref = check_fp64(pr, ctx, g, alpha=0.9, tau=1e-10, norm=1, dg=dg)
    assert res["iterations"] == ref["iterations"]
    m = pr.pull_multi(ctx, [dg, dev(pr, gg.workload_c1())],
                      [dict(alpha=0.9, tau=1e-10, norm=1, max_iter=500), dict(alpha=0.85, tau=1e-6, norm=1,
                                                                              max_iter=500)])
    assert m[0]["iterations"] == ref["iterations"]
    assert np.abs(m[0]["ranks"].cpu().numpy() - ref["ranks"]).sum() <= 1e-12
    probs = [dict(alpha=a, tau=1e-10, norm=n, max_iter=500) for a, n in ((0.5, 1), (0.9, 1), (0.99, 3))]
    for r, p in zip(pr.pull_batch(ctx, dg, probs, precision=pr.PR_FP64, trace=True), probs):
        check_fp64_result(g, r["ranks"].cpu().numpy(), r["iterations"], r["converged"], p["alpha"], p["tau"],
                          p["norm"], 500, gpu_trace=r["trace"].cpu().numpy())
    for r, p in zip(pr.pull_batch(ctx, dg, probs, precision=pr.PR_MIXED), probs):
        check_mixed_result(g, r["ranks"].cpu().numpy(), r["err"], p["alpha"], p["tau"], p["norm"])


@pytest.mark.parametrize("tile", [512, 256])
def test_smaller_tile_windows(pr, ctx, tile):
    # partitions written with the autotuner's smaller windows run through the same kernels
    g = gg.rmat(14, seed=33)
    ctx.set_option("tile", tile)
    ctx.set_option("tile_b", 128)
    try:
        dg = dev(pr, g)
        dg.prepare(ctx)
    finally:
        ctx.set_option("tile", 1024)
        ctx.set_option("tile_b", 256)
    for norm in (1, 3):
        check_fp64(pr, ctx, g, alpha=0.85, tau=1e-10, norm=norm, dg=dg)
    probs = [dict(alpha=a, tau=1e-10, norm=1, max_iter=500) for a in (0.6, 0.85, 0.95)]
    for r, p in zip(pr.pull_batch(ctx, dg, probs, precision=pr.PR_FP64, trace=True), probs):
        check_fp64_result(g, r["ranks"].cpu().numpy(), r["iterations"], r["converged"], p["alpha"], p["tau"],
                          p["norm"], 500, gpu_trace=r["trace"].cpu().numpy())
    with pytest.raises(pr.PrError):
        ctx.set_option("tile", 300)


@pytest.mark.parametrize("mid", [0, 1, 1024])
def test_row_threshold_extremes(pr, ctx, mid):
    # mid_deg 0: every non-empty row of a tile by a wave; 1024: every row by one lane
    g = gg.rmat(14, seed=32)
    try:
        ctx.set_option("mid_deg", mid)
        check_fp64(pr, ctx, g, tau=1e-10, norm=3)
    finally:
        ctx.set_option("mid_deg", 32)


def test_road_like_lattice_single_iteration(pr, ctx):
    # 1000 x 1000 lattice: the first update changes no rank by more than alpha/(3N) = 2.8e-7, so
    # L-infinity at tau = 1e-6 stops after one update (the paper's road networks); L1 and L2 run on
    g = gg.grid2d(1000, 1000)
    dg = dev(pr, g)
    res, ref = check_fp64(pr, ctx, g, alpha=0.85, tau=1e-6, norm=3, dg=dg)
    assert res["iterations"] == 1 == ref["iterations"]
    for norm in (1, 2):
        res, ref = check_fp64(pr, ctx, g, alpha=0.85, tau=1e-6, norm=norm, dg=dg)
        assert res["iterations"] > 1


def test_fp32_only_ablation(pr, ctx):
    # float32 iterate with no float64 update: its stops are its own; where it converges, the
    # ranks sit within the L1 fixed-point bound of the oracle's plus float32 rounding of the
    # iterate (2^-24 relative per vertex, amplified at most 1/(1-alpha) by the map)
    g = gg.rmat(15, seed=41)
    dg = dev(pr, g)
    for norm, tau in ((3, 1e-9), (2, 1e-8), (1, 1e-6)):
        res = pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm, precision=pr.PR_FP32)
        ref = oracle.pagerank_graph(g, alpha=0.85, tau=tau, norm=norm)
        assert res["fp64_iters"] == 0 and res["fp32_iters"] == res["iterations"]
        assert res["converged"] and res["err"][norm - 1] < tau
        r = res["ranks"].cpu().numpy()
        d = np.abs(r - ref["ranks"]).sum()
        assert d <= 0.85 / 0.15 * (res["err"][0] + ref["err"][0]) + 2.0 ** -24 / 0.15 * 4, d
        # the stated L-infinity tolerance, with the float32 map's own fixed-point offset
        check_mixed_result(g, r, res["err"], 0.85, tau, norm, ref=ref, fp32_only=True)
    # the batch and many-graph paths refuse it
    with pytest.raises(pr.PrError):
        pr.pull_batch(ctx, dg, [dict(alpha=0.85, tau=1e-6, norm=1, max_iter=10)], precision=pr.PR_FP32)
