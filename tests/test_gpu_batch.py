"""Parity of the K-column path (pr_pull_batch) and of mixed precision with the CPU oracle.

Every column of a batch must match its own single-problem oracle run (tests/parity.py): in
FP64, ranks within 1e-12 in L1 after the same number of updates and the same iteration count up
to an explained tie.  Mixed-precision results are held to the L1 fixed-point bound of the
section-2 map (for alpha < 1, ||r_k - r*||_1 <= alpha/(1-alpha) * ||r_k - r_{k-1}||_1, so two
solves whose last L1 changes are e_a and e_b differ by at most alpha/(1-alpha) * (e_a + e_b),
plus float64 rounding) and to the stated per-vertex tolerance
max_v |r - r_oracle| <= 2 (e_inf + e_inf_oracle)/(1 - alpha) (10 tau at alpha = 1).
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from parity import TRACE_ATOL, check_fp64_result, check_mixed_result, mixed_bound  # noqa: E402,F401


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


def sweep_problems(tau=1e-10, norm=3, max_iter=500):
    return [dict(alpha=a, tau=tau, norm=norm, max_iter=max_iter) for a in gg.ALPHA_SWEEP]


def check_column(res, g, p, init=None, l1_tol=1e-12):
    tr = res.get("trace")
    return check_fp64_result(g, res["ranks"].cpu().numpy(), res["iterations"], res["converged"], p["alpha"],
                             p["tau"], p["norm"], p["max_iter"], init=init,
                             gpu_trace=None if tr is None else tr.cpu().numpy(), l1_tol=l1_tol)


@pytest.mark.parametrize("make", [gg.workload_c1, lambda: gg.rmat(15, seed=7)])
def test_alpha_sweep_fp64(pr, ctx, make):
    g = make()
    dg = pr.DeviceGraph.from_host(g)
    probs = sweep_problems()
    res = pr.pull_batch(ctx, dg, probs, precision=pr.PR_FP64, trace=True)
    for r, p in zip(res, probs):
        check_column(r, g, p)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5, 8, 9, 12, 13, 16])
def test_column_counts_and_mixed_settings(pr, ctx, K):
    g = gg.rmat(13, seed=K)
    dg = pr.DeviceGraph.from_host(g)
    rng = np.random.default_rng(K)
    probs = [dict(alpha=float(rng.choice([0.5, 0.85, 0.95, 1.0])), tau=float(rng.choice([1e-4, 1e-8, 1e-11])),
                  norm=int(rng.integers(1, 4)), max_iter=int(rng.choice([3, 500]))) for _ in range(K)]
    res = pr.pull_batch(ctx, dg, probs, precision=pr.PR_FP64)
    for r, p in zip(res, probs):
        check_column(r, g, p)


def test_more_than_sixteen_problems_are_grouped(pr, ctx):
    g = gg.workload_c1()
    dg = pr.DeviceGraph.from_host(g)
    probs = [dict(alpha=a, tau=t, norm=n, max_iter=500) for a in gg.ALPHA_SWEEP for t, n in ((1e-6, 1), (1e-9, 3))]
    res = pr.pull_batch(ctx, dg, probs)
    assert len(res) == 22
    for r, p in zip(res, probs):
        check_column(r, g, p)


def test_per_column_starts(pr, ctx):
    g = gg.rmat(12, seed=3)
    dg = pr.DeviceGraph.from_host(g)
    rng = np.random.default_rng(0)
    starts = []
    for _ in range(3):
        x = rng.random(g.N)
        starts.append(x / x.sum())
    inits = [torch.from_numpy(starts[0]).cuda(), None, torch.from_numpy(starts[2]).cuda()]
    probs = [dict(alpha=0.85, tau=1e-9, norm=1, max_iter=500)] * 3
    res = pr.pull_batch(ctx, dg, probs, inits=inits)
    for r, p, s0 in zip(res, probs, (starts[0], None, starts[2])):
        check_column(r, g, p, init=s0)


@pytest.mark.parametrize("K", [1, 2, 7, 11])
def test_hubs_in_batch(pr, ctx, K):
    rng = np.random.default_rng(9)
    N = 40000
    src, dst = [], []
    for v, deg in ((0, 30001), (5, 8193), (6, 5000), (7, 1025), (8, 40)):
        src.extend(rng.choice(N, size=deg, replace=False).tolist())
        dst.extend([v] * deg)
    src.extend(rng.integers(0, N, 80000).tolist())
    dst.extend(rng.integers(0, N, 80000).tolist())
    g = gg.from_edges(N, src, dst)
    dg = pr.DeviceGraph.from_host(g)
    probs = sweep_problems(tau=1e-11, norm=1)[:K]
    for r, p in zip(pr.pull_batch(ctx, dg, probs), probs):
        check_column(r, g, p)
    for r, p in zip(pr.pull_batch(ctx, dg, probs, precision=pr.PR_MIXED), probs):
        assert r["converged"], p
        check_mixed_result(g, r["ranks"].cpu().numpy(), r["err"], p["alpha"], p["tau"], p["norm"])


def test_batch_repeatable(pr, ctx):
    g = gg.rmat(14, seed=2)
    dg = pr.DeviceGraph.from_host(g)
    a = [r["ranks"].clone() for r in pr.pull_batch(ctx, dg, sweep_problems())]
    b = [r["ranks"].clone() for r in pr.pull_batch(ctx, dg, sweep_problems())]
    assert all(torch.equal(x, y) for x, y in zip(a, b))


@pytest.mark.parametrize("K", [9, 12, 16])
def test_mixed_settings_on_wide_rows(pr, ctx, K):
    # 9 to 12 float32 columns share rows of 12 values (three per lane of a four-lane group), 13
    # to 16 rows of 16; random settings, some columns halted by max_iter inside the float32 phase
    g = gg.rmat(13, seed=100 + K)
    dg = pr.DeviceGraph.from_host(g)
    rng = np.random.default_rng(100 + K)
    probs = [dict(alpha=float(rng.choice([0.5, 0.85, 0.95])), tau=float(rng.choice([1e-6, 1e-9, 1e-11])),
                  norm=int(rng.integers(1, 4)), max_iter=int(rng.choice([3, 500]))) for _ in range(K)]
    ctx.reset_stats()
    ctx.set_option("timing", 1)
    try:
        res = pr.pull_batch(ctx, dg, probs, precision=pr.PR_MIXED)
    finally:
        ctx.set_option("timing", 0)
    width = 12 if K <= 12 else 16
    assert ctx.stats(pr._lib.batch_kind(True, width))[0] > 0
    assert all(ctx.stats(pr._lib.batch_kind(True, w))[0] == 0 for w in pr._lib.BATCH_ROW_WIDTHS if w > width)
    for r, p in zip(res, probs):
        ref = oracle.pagerank_graph(g, alpha=p["alpha"], tau=p["tau"], norm=p["norm"], max_iter=p["max_iter"])
        d = np.abs(r["ranks"].cpu().numpy() - ref["ranks"]).sum()
        assert r["fp32_iters"] + r["fp64_iters"] == r["iterations"]
        if p["max_iter"] == 3:
            # stopped by max_iter in the float32 phase: three float32 updates of the oracle's map
            assert r["iterations"] == 3 and r["fp32_iters"] == 3 and not r["converged"], (p, r)
            assert d <= 5e-5, (p, d)
        else:
            assert r["converged"] and r["err"][p["norm"] - 1] < p["tau"], (p, r)
            check_mixed_result(g, r["ranks"].cpu().numpy(), r["err"], p["alpha"], p["tau"], p["norm"], ref=ref)


@pytest.mark.parametrize("norm,tau", [(1, 1e-10), (3, 1e-10), (2, 1e-8), (1, 1e-4)])
def test_mixed_single_against_oracle(pr, ctx, norm, tau):
    g = gg.rmat(15, seed=5)
    dg = pr.DeviceGraph.from_host(g)
    res = pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm, precision=pr.PR_MIXED)
    assert res["converged"] and res["fp64_iters"] >= 1 and res["fp32_iters"] >= 1
    assert res["err"][norm - 1] < tau  # the deciding update is a float64 one
    check_mixed_result(g, res["ranks"].cpu().numpy(), res["err"], 0.85, tau, norm)


def test_mixed_batch_sweep(pr, ctx):
    g = gg.rmat(15, seed=6)
    dg = pr.DeviceGraph.from_host(g)
    probs = sweep_problems(tau=1e-10, norm=3)[:-1]  # alpha < 1 for the bound
    res = pr.pull_batch(ctx, dg, probs, precision=pr.PR_MIXED)
    for r, p in zip(res, probs):
        assert r["converged"] and r["fp64_iters"] >= 1
        assert r["err"][2] < p["tau"]
        check_mixed_result(g, r["ranks"].cpu().numpy(), r["err"], p["alpha"], p["tau"], p["norm"])


def test_batch_errors(pr, ctx):
    g = gg.cycle(5)
    dg = pr.DeviceGraph.from_host(g)
    with pytest.raises(pr.PrError) as ei:
        pr.pull_batch(ctx, dg, [dict(alpha=1.2, tau=1e-6, norm=1, max_iter=10)])
    assert ei.value.status == -1
    with pytest.raises(ValueError):
        pr.pr_pull_batch(ctx, dg, [], 0, None, [], None, torch.empty(8, dtype=torch.uint8, device="cuda"))


@pytest.mark.parametrize("precision", [0, 1])
def test_compaction_changes_nothing(pr, ctx, precision):
    # Repacking the still-active columns into narrower rows keeps every per-column sum in the
    # same order; with the grid pinned (same block partials) the results are bitwise equal.
    g = gg.rmat(14, seed=21)
    dg = pr.DeviceGraph.from_host(g)
    probs = sweep_problems(tau=1e-10, norm=3)
    # rows of one or two values (one lane per row fetch) sum in another order: kept out here
    out = {}
    try:
        ctx.set_option("grid", 300)
        ctx.set_option("narrow", 0)
        for compact in (0, 1):
            ctx.set_option("compact", compact)
            out[compact] = pr.pull_batch(ctx, dg, probs, precision=precision)
            out[compact] = [(r["iterations"], r["fp32_iters"], r["ranks"].clone()) for r in out[compact]]
    finally:
        ctx.set_option("compact", 1)
        ctx.set_option("narrow", 1)
        ctx.set_option("grid", 0)
    for (i0, f0, r0), (i1, f1, r1) in zip(out[0], out[1]):
        assert i0 == i1 and f0 == f1
        assert torch.equal(r0, r1)


def test_batch_chunk_sizes_agree(pr, ctx):
    # The host looks at the columns every batch_chunk updates (the compaction points).  Any even
    # chunk gives the same result (grid pinned, rows of four or more values, as above); an odd
    # one is rejected, since the updates of a chunk alternate the two row buffers from the first.
    g = gg.rmat(13, seed=41)
    dg = pr.DeviceGraph.from_host(g)
    probs = sweep_problems(tau=1e-10, norm=1)[:-1]
    out = []
    try:
        ctx.set_option("grid", 300)
        ctx.set_option("narrow", 0)
        for bc in (2, 4, 6, 64):
            ctx.set_option("batch_chunk", bc)
            res = pr.pull_batch(ctx, dg, probs, precision=pr.PR_MIXED)
            out.append([(r["iterations"], r["fp32_iters"], r["ranks"].clone()) for r in res])
        for bad in (0, 1, 3, 65, 66):
            with pytest.raises(pr.PrError):
                ctx.set_option("batch_chunk", bad)
    finally:
        ctx.set_option("batch_chunk", 2)
        ctx.set_option("narrow", 1)
        ctx.set_option("grid", 0)
    for o in out[1:]:
        for (i0, f0, r0), (i1, f1, r1) in zip(out[0], o):
            assert i0 == i1 and f0 == f1 and torch.equal(r0, r1)


def test_float32_row_handover_is_the_float64_update(pr, ctx):
    # The first float64 update of a mixed batch reads the handover's float32 rows (exact in
    # float64) instead of float64 copies and sums in float64: with the grid pinned (the same
    # block partials) every result is bitwise the one of the float64 rows, on rows of 12, 8, 1,
    # 2 and 16 values.  A column stopped by max_iter in the float32 phase keeps the float64-row
    # path (last case).
    g = gg.rmat(14, seed=51)
    dg = pr.DeviceGraph.from_host(g)
    cases = [sweep_problems(tau=1e-10, norm=3), sweep_problems(tau=1e-9, norm=1)[:5],
             sweep_problems(tau=1e-10, norm=3)[7:8], sweep_problems(tau=1e-10, norm=1)[8:10],
             [dict(alpha=a, tau=1e-10, norm=2, max_iter=500) for a in np.linspace(0.5, 0.97, 16)],
             [dict(alpha=0.85, tau=1e-10, norm=2, max_iter=500), dict(alpha=0.9, tau=1e-10, norm=1, max_iter=4)]]
    try:
        ctx.set_option("grid", 300)
        for probs in cases:
            out = {}
            for h in (0, 1):
                ctx.set_option("handover32", h)
                res = pr.pull_batch(ctx, dg, probs, precision=pr.PR_MIXED, trace=True)
                out[h] = [(r["iterations"], r["fp32_iters"], r["converged"], r["ranks"].clone(), r["trace"].clone())
                          for r in res]
            for a, b in zip(out[0], out[1]):
                assert a[:3] == b[:3] and torch.equal(a[3], b[3]) and torch.equal(a[4], b[4]), a[:3]
        with pytest.raises(pr.PrError):
            ctx.set_option("handover32", 2)
    finally:
        ctx.set_option("handover32", 1)
        ctx.set_option("grid", 0)


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_on_the_relabelled_graph(pr, ctx, precision):
    # the sweep solved on the out-degree-ordered graph (pr_relabel), each column mapped back with
    # pr_unpermute, against the oracle on the graph as generated
    g = gg.rmat(14, seed=61)
    dg = pr.DeviceGraph.from_host(g)
    h, perm = dg.relabelled(ctx)
    probs = sweep_problems(tau=1e-10, norm=3)[:-1]
    res = pr.pull_batch(ctx, h, probs, precision=precision)
    for r, p in zip(res, probs):
        back = pr.unpermute(ctx, perm, r["ranks"]).cpu().numpy()
        if precision == pr.PR_FP64:
            check_fp64_result(g, back, r["iterations"], r["converged"], p["alpha"], p["tau"], p["norm"], p["max_iter"])
        else:
            assert r["converged"], p
            check_mixed_result(g, back, r["err"], p["alpha"], p["tau"], p["norm"])


def test_compaction_with_traces_and_max_iter(pr, ctx):
    g = gg.rmat(13, seed=22)
    dg = pr.DeviceGraph.from_host(g)
    probs = [dict(alpha=a, tau=1e-10, norm=1, max_iter=m) for a, m in
             ((0.5, 500), (0.6, 4), (0.7, 500), (0.8, 7), (0.85, 500), (0.9, 500), (0.95, 2), (1.0, 500),
              (0.55, 500), (0.65, 500), (0.99, 500))]
    res = pr.pull_batch(ctx, dg, probs, trace=True)
    for r, p in zip(res, probs):
        check_column(r, g, p)


@pytest.mark.parametrize("make", [lambda: gg.edgeless(1), lambda: gg.cycle(2), lambda: gg.in_star(1),
                                  lambda: gg.out_star(5), gg.two_triangles])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_on_tiny_graphs(pr, ctx, make, precision):
    g = make()
    dg = pr.DeviceGraph.from_host(g)
    probs = [dict(alpha=0.85, tau=1e-12, norm=1, max_iter=500), dict(alpha=0.5, tau=1e-10, norm=3, max_iter=500),
             dict(alpha=1.0, tau=1e-12, norm=2, max_iter=50)]
    res = pr.pull_batch(ctx, dg, probs, precision=precision)
    for r, p in zip(res, probs):
        ref = oracle.pagerank_graph(g, trace=True, **p)
        d = np.abs(r["ranks"].cpu().numpy() - ref["ranks"]).sum()
        if precision == 0:
            check_column(r, g, p)
        else:
            assert r["err"][p["norm"] - 1] < p["tau"] or not r["converged"]
            if r["converged"]:
                check_mixed_result(g, r["ranks"].cpu().numpy(), r["err"], p["alpha"], p["tau"], p["norm"],
                                   max_iter=p["max_iter"], ref=ref)
            else:
                # stopped by max_iter at alpha = 1: float32 rounding of the iterate only
                assert d <= 1e-6, (p, d)


@pytest.mark.parametrize("precision", [0, 1])
def test_narrow_rows_against_oracle(pr, ctx, precision):
    # one and two columns run on rows of one and two values, from the start (K = 1, 2) and after
    # compaction of a sweep; every update is counted under the width it ran on
    g = gg.rmat(14, seed=31)
    dg = pr.DeviceGraph.from_host(g)
    fp32 = precision == pr.PR_MIXED
    sweeps = [sweep_problems(tau=1e-10, norm=3)[7:8], sweep_problems(tau=1e-10, norm=1)[8:10],
              sweep_problems(tau=1e-10, norm=3)[:-1]]
    for probs in sweeps:
        ctx.reset_stats()
        ctx.set_option("timing", 1)
        try:
            res = pr.pull_batch(ctx, dg, probs, precision=precision)
        finally:
            ctx.set_option("timing", 0)
        for r, p in zip(res, probs):
            if precision == pr.PR_FP64:
                check_column(r, g, p)
            else:
                assert r["converged"], p
                check_mixed_result(g, r["ranks"].cpu().numpy(), r["err"], p["alpha"], p["tau"], p["norm"])
        first = ctx.stats(pr._lib.PR_KERNEL_BATCH_F32 if fp32 else pr._lib.PR_KERNEL_BATCH_F64)[0]
        by_width = {w: ctx.stats(pr._lib.batch_kind(fp32, w))[0] for w in pr._lib.BATCH_ROW_WIDTHS}
        assert first > 0 and sum(by_width.values()) == first, by_width
        K = len(probs)
        if K <= 2:
            # starts at width K; a column that stops leaves the other on width 1
            assert by_width[K] > 0 and all(n == 0 for w, n in by_width.items() if w > K), by_width
        else:
            # ten columns start on rows of 12 values (4 * ceil(K / 4), never padded to 16) and the
            # sweep ends with its slowest one or two columns
            assert by_width[12] > 0 and by_width[16] == 0, by_width
            assert by_width[1] + by_width[2] > 0, by_width
