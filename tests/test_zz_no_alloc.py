"""pr_pull_noalloc (the solve that allocates nothing: its workspace is the library's fixed device
array) against pr_pull with a caller's workspace, through the C ABI: two calls in a row, the
second on a smaller graph, each with the float64 parity bar of tests/parity.py (here the two
entry points run the same kernels on the same grid, so their results are also bitwise equal),
and the size limit refused with PR_ENOMEM before any launch.
"""
import ctypes

import numpy as np
import pytest

import graphgen as gg

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


def noalloc(pr, ctx, dg, alpha, tau, norm, max_iter, precision, trace=False):
    ranks = torch.full((dg.N,), float("nan"), dtype=torch.float64, device="cuda")
    tr = torch.zeros(3 * max_iter, dtype=torch.float64, device="cuda") if trace else None
    res = pr._lib.pr_result()
    st = ctx.lib.pr_pull_noalloc(ctx.handle, ctx.stream, dg.off.data_ptr(), pr._lib.ptr(dg.idx) if dg.E else None,
                                 dg.outdeg.data_ptr(), dg.N, dg.E, float(alpha), float(tau), int(norm),
                                 int(max_iter), int(precision), None, ranks.data_ptr(), pr._lib.ptr(tr),
                                 ctypes.byref(res))
    return st, res.as_dict(), ranks, tr


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_pull_twice_second_smaller(pr, ctx, precision):
    from parity import check_fp64_result, check_mixed_result
    graphs = [gg.rmat(17, seed=41), gg.rmat(12, seed=42)]  # the second call on a smaller graph
    for g in graphs:
        dg = pr.DeviceGraph.from_host(g)
        st, res, ranks, tr = noalloc(pr, ctx, dg, 0.85, 1e-10, 1, 500, precision, trace=True)
        assert st == pr._lib.PR_OK, pr._lib.last_error()
        ref = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1, max_iter=500, precision=precision, trace=True)
        assert res["iterations"] == ref["iterations"] and res["fp32_iters"] == ref["fp32_iters"]
        assert torch.equal(ranks, ref["ranks"]), float((ranks - ref["ranks"]).abs().max())
        it = res["iterations"]
        assert torch.equal(tr[:3 * it], ref["trace"].reshape(-1)[:3 * it])
        if precision == 0:
            check_fp64_result(g, ranks.cpu().numpy(), it, res["converged"], 0.85, 1e-10, 1, 500,
                              gpu_trace=tr[:3 * it].reshape(it, 3).cpu().numpy())
        else:
            check_mixed_result(g, ranks.cpu().numpy(), res["err"], 0.85, 1e-10, 1)


def test_noalloc_limit_and_arguments(pr, ctx):
    cap = ctx.lib.pr_noalloc_max_bytes()
    assert cap == 64 << 20
    # a graph whose workspace exceeds the fixed scratch is refused before anything runs
    N = 5_000_000
    assert ctx.lib.pr_workspace_bytes(N, 0, 0, 1) > cap
    off = torch.zeros(N + 1, dtype=torch.int32, device="cuda")
    outdeg = torch.zeros(N, dtype=torch.int32, device="cuda")
    ranks = torch.zeros(N, dtype=torch.float64, device="cuda")
    res = pr._lib.pr_result()
    st = ctx.lib.pr_pull_noalloc(ctx.handle, ctx.stream, off.data_ptr(), None, outdeg.data_ptr(), N, 0, 0.85, 1e-6,
                                 1, 10, 0, None, ranks.data_ptr(), None, ctypes.byref(res))
    assert st == pr._lib.PR_ENOMEM and "fixed scratch" in pr._lib.last_error()
    g = gg.rmat(10, seed=1)
    dg = pr.DeviceGraph.from_host(g)
    st = ctx.lib.pr_pull_noalloc(ctx.handle, ctx.stream, dg.off.data_ptr(), dg.idx.data_ptr(), dg.outdeg.data_ptr(),
                                 g.N, g.E, 1.5, 1e-6, 1, 10, 0, None, ranks.data_ptr(), None, ctypes.byref(res))
    assert st == pr._lib.PR_EINVAL
    # still correct after the refused calls
    st, out, r, _ = noalloc(pr, ctx, dg, 0.85, 1e-8, 3, 100, 0)
    ref = pr.pull(ctx, dg, alpha=0.85, tau=1e-8, norm=3, max_iter=100)
    assert st == pr._lib.PR_OK and out["iterations"] == ref["iterations"] and torch.equal(r, ref["ranks"])
