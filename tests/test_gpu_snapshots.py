"""pr_pull_snapshots (rank snapshots at (tau, norm) stopping points, from one solve) through the
C ABI.

A snapshot is defined as the ranks a solve with that (tau, norm) returns (the tolerance study of
sections 3 and 4 stops one power iteration at many (tau, norm) pairs): every snapshot is held
bit for bit to a separate pr_pull with that pair, and, in float64, to the oracle at the bar of
tests/parity.py (ranks within 1e-12 in L1 after the same number of updates, tie rule on the
count).
"""
import numpy as np
import pytest

import graphgen as gg
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


# every tolerance of the grid in every norm: the L1 change is the largest of the three, so the
# solve's own stop (L1, 1e-11) comes after all of them
PAIRS = [(t, n) for t in (1e-3, 1e-5, 1e-7, 1e-9) for n in (1, 2, 3)]


def check_against_separate_solves(pr, ctx, dg, res, pairs, alpha, max_iter, precision):
    for i, (t, n) in enumerate(pairs):
        one = pr.pull(ctx, dg, alpha=alpha, tau=t, norm=n, max_iter=max_iter, precision=precision)
        assert res["snap_iter"][i] == one["iterations"], (t, n, res["snap_iter"][i], one["iterations"])
        assert torch.equal(res["snapshots"][i], one["ranks"]), (t, n)


@pytest.mark.parametrize("layout", ["plain", "segmented"])
def test_snapshots_are_the_separate_solves(pr, ctx, layout):
    g = gg.rmat(13, seed=71)
    dg = pr.DeviceGraph.from_host(g)
    if layout == "segmented":
        dg.prepare_segmented(ctx, seg_len=1024)
    res = pr.pull_snapshots(ctx, dg, PAIRS, alpha=0.85, tau=1e-11, norm=1, max_iter=500)
    assert res["converged"] and all(k > 0 for k in res["snap_iter"])
    # stricter tolerances are met no earlier; in one norm they are met in order
    for n in (1, 2, 3):
        its = [res["snap_iter"][i] for i, (t, m) in enumerate(PAIRS) if m == n]
        assert its == sorted(its)
    check_against_separate_solves(pr, ctx, dg, res, PAIRS, 0.85, 500, pr.PR_FP64)
    for i, (t, n) in enumerate(PAIRS):
        check_fp64_result(g, res["snapshots"][i].cpu().numpy(), res["snap_iter"][i], True, 0.85, t, n, 500)


def test_float32_snapshots(pr, ctx):
    g = gg.rmat(12, seed=72)
    dg = pr.DeviceGraph.from_host(g)
    pairs = [(t, n) for t in (1e-3, 1e-4, 1e-5) for n in (1, 3)]
    res = pr.pull_snapshots(ctx, dg, pairs, alpha=0.85, tau=1e-6, norm=1, max_iter=300, precision=pr.PR_FP32)
    assert all(k > 0 for k in res["snap_iter"])
    check_against_separate_solves(pr, ctx, dg, res, pairs, 0.85, 300, pr.PR_FP32)


def test_unmet_repeated_and_max_iter(pr, ctx):
    g = gg.workload_c1()
    dg = pr.DeviceGraph.from_host(g)
    # a pair met after the solve's own stop is not taken; a repeated pair is taken twice
    pairs = [(1e-4, 1), (1e-4, 1), (1e-14, 3), (1e-6, 2)]
    res = pr.pull_snapshots(ctx, dg, pairs, alpha=0.85, tau=1e-8, norm=1, max_iter=500)
    assert res["snap_iter"][0] == res["snap_iter"][1] > 0 and res["snap_iter"][2] == 0
    assert torch.equal(res["snapshots"][0], res["snapshots"][1])
    assert bool(torch.isnan(res["snapshots"][2]).all())
    check_against_separate_solves(pr, ctx, dg, res, [pairs[0], pairs[3]], 0.85, 500, pr.PR_FP64)
    # the solve stopped by max_iter: snapshots met before it are taken, the rest are not
    res = pr.pull_snapshots(ctx, dg, [(1e-3, 3), (1e-12, 1)], alpha=0.85, tau=1e-12, norm=1, max_iter=7)
    assert not res["converged"] and res["iterations"] == 7
    assert 0 < res["snap_iter"][0] <= 7 and res["snap_iter"][1] == 0
    one = pr.pull(ctx, dg, alpha=0.85, tau=1e-3, norm=3, max_iter=7)
    assert one["iterations"] == res["snap_iter"][0] and torch.equal(res["snapshots"][0], one["ranks"])


def test_long_solve_across_chunks(pr, ctx):
    # a lattice converges slowly (99 updates to 1e-10 in L1 at alpha = 0.85, where the R-MAT and
    # random graphs above take 18-31): snapshots fall in several chunks of the captured loop
    g = gg.grid2d(48, 48)
    dg = pr.DeviceGraph.from_host(g)
    pairs = [(t, 2) for t in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10)]
    res = pr.pull_snapshots(ctx, dg, pairs, alpha=0.85, tau=1e-10, norm=1, max_iter=1000)
    assert res["converged"] and res["iterations"] > 64
    assert len(set(res["snap_iter"])) == len(pairs) and max(res["snap_iter"]) > 48
    check_against_separate_solves(pr, ctx, dg, res, pairs, 0.85, 1000, pr.PR_FP64)
    for i, (t, n) in enumerate(pairs):
        check_fp64_result(g, res["snapshots"][i].cpu().numpy(), res["snap_iter"][i], True, 0.85, t, n, 1000)


def test_argument_errors(pr, ctx):
    g = gg.rmat(10, seed=74)
    dg = pr.DeviceGraph.from_host(g)
    with pytest.raises(pr.PrError):
        pr.pull_snapshots(ctx, dg, [(1e-6, 1)], precision=pr.PR_MIXED)
    with pytest.raises(pr.PrError):
        pr.pull_snapshots(ctx, dg, [])
    with pytest.raises(pr.PrError):
        pr.pull_snapshots(ctx, dg, [(1e-6, 1)] * 65)
    with pytest.raises(pr.PrError):
        pr.pull_snapshots(ctx, dg, [(1e-6, 4)])
    with pytest.raises(pr.PrError):
        pr.pull_snapshots(ctx, dg, [(-1.0, 1)])
    with pytest.raises(pr.PrError):
        pr.pull_snapshots(ctx, dg, [(float("nan"), 1)])
    # a solve with snapshots, then one without, on the same context: the plain solve is unchanged
    a = pr.pull(ctx, dg, alpha=0.85, tau=1e-9, norm=1)
    pr.pull_snapshots(ctx, dg, [(1e-5, 1)], alpha=0.85, tau=1e-9, norm=1)
    b = pr.pull(ctx, dg, alpha=0.85, tau=1e-9, norm=1)
    assert torch.equal(a["ranks"], b["ranks"]) and a["iterations"] == b["iterations"]
    assert np.isfinite(b["ranks"].cpu().numpy()).all()


def test_sweep_columns_agree_with_snapshots(pr, ctx):
    # two independent routes to the same readout: the power-series sweep with one column per
    # (tau, norm) pair at one alpha (ranks formed from the alpha = 1 iterates) and the snapshots
    # of one alpha = 0.85 solve (the iterates themselves); equal stops, ranks within 1e-12 in L1
    g = gg.rmat(13, seed=75)
    dg = pr.DeviceGraph.from_host(g)
    pairs = [(t, n) for t in (1e-4, 1e-6, 1e-8) for n in (1, 2, 3)]
    snap = pr.pull_snapshots(ctx, dg, pairs, alpha=0.85, tau=1e-10, norm=1, max_iter=500)
    cols = pr.pull_sweep(ctx, dg, [dict(alpha=0.85, tau=t, norm=n, max_iter=500) for t, n in pairs])
    for i, c in enumerate(cols):
        # the two decide a stop from the same change computed along different routes: a tie may
        # move it by one update
        assert abs(c["iterations"] - snap["snap_iter"][i]) <= 1, (pairs[i], c["iterations"], snap["snap_iter"][i])
        if c["iterations"] == snap["snap_iter"][i]:
            assert pr.l1_distance(ctx, c["ranks"], snap["snapshots"][i].contiguous()) <= 1e-12, pairs[i]


def test_given_start_and_edgeless(pr, ctx):
    # from a given start vector the snapshots are the separate solves from that start
    g = gg.rmat(12, seed=76)
    dg = pr.DeviceGraph.from_host(g)
    init = torch.rand(g.N, dtype=torch.float64, device="cuda")
    init /= init.sum()
    pairs = [(1e-5, 1), (1e-7, 3)]
    res = pr.pull_snapshots(ctx, dg, pairs, alpha=0.9, tau=1e-10, norm=1, init=init)
    for i, (t, n) in enumerate(pairs):
        one = pr.pull(ctx, dg, alpha=0.9, tau=t, norm=n, init=init)
        assert res["snap_iter"][i] == one["iterations"] and torch.equal(res["snapshots"][i], one["ranks"])
    # no edges: every vertex dangling, the uniform start is the fixed point, the first update
    # changes nothing and takes every snapshot
    e = gg.edgeless(7)
    de = pr.DeviceGraph.from_host(e)
    res = pr.pull_snapshots(ctx, de, [(1e-3, 1), (0.5, 3)], alpha=0.85, tau=1e-12, norm=1)
    assert res["iterations"] == 1 and res["snap_iter"] == [1, 1]
    np.testing.assert_allclose(res["snapshots"].cpu().numpy(), np.full((2, 7), 1 / 7), rtol=1e-15)
