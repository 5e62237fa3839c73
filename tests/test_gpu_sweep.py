"""pr_pull_sweep (the damping-factor sweep as one power series, float64) against the oracle, through
the C ABI.

Every column is held to the float64 bar of tests/parity.py against the oracle's own power
iteration at that column's settings: ranks within 1e-12 in L1 after the same number of updates,
the norm trace row by row, and the same iteration count (tie rule).  The identity the path rests
on is pinned on the oracle alone in tests/test_oracle_pins.py.
"""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle
from parity import check_fp64_result

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


def check_sweep(pr, ctx, g, probs, dg=None):
    dg = dg or pr.DeviceGraph.from_host(g)
    res = pr.pull_sweep(ctx, dg, probs, trace=True)
    for r, p in zip(res, probs):
        check_fp64_result(g, r["ranks"].cpu().numpy(), r["iterations"], r["converged"], p["alpha"], p["tau"],
                          p["norm"], p["max_iter"], gpu_trace=r["trace"].cpu().numpy())
        assert r["fp32_iters"] == 0 and r["fp64_iters"] == r["iterations"]
    return res


def sweep_problems(tau=1e-10, norm=3, max_iter=500):
    return [dict(alpha=a, tau=tau, norm=norm, max_iter=max_iter) for a in gg.ALPHA_SWEEP]


def test_c1_alpha_sweep(pr, ctx):
    res = check_sweep(pr, ctx, gg.workload_c1(), sweep_problems())
    its = [r["iterations"] for r in res]
    assert its == sorted(its)  # larger damping factors need at least as many updates


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_rmat_sweep_every_norm(pr, ctx, norm):
    check_sweep(pr, ctx, gg.rmat(13, seed=61), sweep_problems(tau=1e-9, norm=norm))


def test_mixed_settings_and_max_iter(pr, ctx):
    g = gg.rmat(12, seed=62)
    rng = np.random.default_rng(62)
    probs = [dict(alpha=float(rng.choice([0.0, 0.3, 0.5, 0.85, 0.95, 0.99, 1.0])),
                  tau=float(rng.choice([0.0, 1e-3, 1e-7, 1e-11])), norm=int(rng.integers(1, 4)),
                  max_iter=int(rng.choice([1, 5, 40, 300]))) for _ in range(24)]
    res = check_sweep(pr, ctx, g, probs)
    for r, p in zip(res, probs):
        if p["tau"] == 0.0 and p["alpha"] > 0.0:
            assert r["iterations"] == p["max_iter"] and not r["converged"]


def test_one_and_sixty_four_columns_and_hubs(pr, ctx):
    rng = np.random.default_rng(5)
    N = 30000
    src, dst = [], []
    for v, deg in ((0, 20000), (3, 9000), (4, 1500)):
        src.extend(rng.choice(N, size=deg, replace=False).tolist())
        dst.extend([v] * deg)
    src.extend(rng.integers(0, N, 60000).tolist())
    dst.extend(rng.integers(0, N, 60000).tolist())
    g = gg.from_edges(N, src, dst)
    dg = pr.DeviceGraph.from_host(g)
    check_sweep(pr, ctx, g, [dict(alpha=0.85, tau=1e-10, norm=1, max_iter=500)], dg=dg)
    probs = [dict(alpha=float(a), tau=[1e-6, 1e-9, 1e-12][i % 3], norm=1 + i % 3, max_iter=500)
             for i, a in enumerate(np.linspace(0.0, 1.0, 64))]
    check_sweep(pr, ctx, g, probs, dg=dg)


def test_segmented_prep_and_repeatable(pr, ctx):
    g = gg.rmat(14, seed=63)
    dg = pr.DeviceGraph.from_host(g)
    dg.prepare_segmented(ctx, seg_len=1 << 10)
    a = check_sweep(pr, ctx, g, sweep_problems(), dg=dg)
    b = pr.pull_sweep(ctx, dg, sweep_problems())
    assert all(torch.equal(x["ranks"], y["ranks"]) and x["iterations"] == y["iterations"] for x, y in zip(a, b))


def test_agrees_with_the_batch(pr, ctx):
    g = gg.rmat(14, seed=64)
    dg = pr.DeviceGraph.from_host(g)
    s = pr.pull_sweep(ctx, dg, sweep_problems())
    b = pr.pull_batch(ctx, dg, sweep_problems(), precision=pr.PR_FP64)
    for x, y in zip(s, b):
        assert abs(x["iterations"] - y["iterations"]) <= 1
        assert pr.l1_distance(ctx, x["ranks"], y["ranks"]) <= 1e-12 or x["iterations"] != y["iterations"]


def test_argument_errors(pr, ctx):
    g = gg.rmat(8, seed=1)
    dg = pr.DeviceGraph.from_host(g).prepare(ctx)
    with pytest.raises(ValueError):
        pr.pull_sweep(ctx, dg, [])
    with pytest.raises(pr.PrError):
        pr.pull_sweep(ctx, dg, [dict(alpha=1.5, tau=1e-6, norm=1, max_iter=10)])
    with pytest.raises(pr.PrError):
        pr.pull_sweep(ctx, dg, [dict(alpha=0.5, tau=1e-6, norm=4, max_iter=10)])
    r = torch.empty(g.N, dtype=torch.float64, device="cuda")
    with pytest.raises(pr.PrError):  # two problems writing one buffer
        pr.pull_sweep(ctx, dg, sweep_problems()[:2], ranks=[r, r])
    lib = ctx.lib
    res = (pr._lib.pr_result * 1)()
    probs = (pr._lib.pr_problem * 1)(pr._lib.pr_problem(0.85, 1e-6, 1, 10))
    arr = (ctypes.c_void_p * 1)(r.data_ptr())
    ws = torch.empty(lib.pr_sweep_workspace_bytes(g.N, g.E, 1), dtype=torch.uint8, device="cuda")
    assert lib.pr_pull_sweep(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), dg.outdeg.data_ptr(), g.N,
                             g.E, None, 65, probs, arr, None, ws.data_ptr(), ws.numel(), res) == pr._lib.PR_EINVAL
    assert lib.pr_pull_sweep(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), dg.outdeg.data_ptr(), g.N,
                             g.E, None, 1, probs, arr, None, ws.data_ptr(), 100, res) == pr._lib.PR_ENOMEM
    # prepared inside the workspace
    assert lib.pr_pull_sweep(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), dg.outdeg.data_ptr(), g.N,
                             g.E, None, 1, probs, arr, None, ws.data_ptr(), ws.numel(), res) in (0, 1)
    ref = oracle.pagerank_graph(g, alpha=0.85, tau=1e-6, norm=1, max_iter=10)
    assert res[0].iterations == ref["iterations"]
    assert np.abs(r.cpu().numpy() - ref["ranks"]).sum() <= 1e-12


def test_scale22_sweep_against_oracle(pr, ctx):
    g = gg.rmat(22, edge_factor=16, seed=22)
    dg = pr.DeviceGraph.from_host(g)
    dg.prepare_segmented(ctx, seg_len=1 << 19)
    res = check_sweep(pr, ctx, g, sweep_problems(), dg=dg)
    print("scale 22 sweep iterations:", [r["iterations"] for r in res])
