"""Parity at the full workload sizes, in the launch configuration the benchmark times.

* R-MAT scale 22 (4,194,304 vertices, ~65 M edges), alpha = 0.85: the float64 solve to
  tau = 1e-10 with its norm trace against the oracle's full trace; the tau x norm readout of
  section 3 taken from both traces; mixed precision per norm against the oracle.
* R-MAT scale 24 (16,777,216 vertices, ~263 M edges): the eleven-column damping sweep,
  tau = 1e-10 in L-infinity, float32 gather with float64 norms and refinement (the benchmark's
  step, default launch settings).  Every column against its own full oracle solve: within the L1
  fixed-point bound alpha/(1-alpha) * (e_gpu + e_oracle) for alpha < 1 (section 2 map, an
  alpha-contraction in L1) and within the stated per-vertex tolerance
  2 (e_inf + e_inf_oracle)/(1 - alpha) (10 tau at alpha = 1); the same column solved alone in
  float64 (the benchmark's baseline) within 1e-12 in L1 after the same number of updates.
* The uneven batch of 64 graphs (vertex counts log-uniform in [1e3, 1e6]) in one persistent
  launch, every graph against its own oracle solve.
"""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from parity import TRACE_ATOL, check_fp64_result, check_mixed_result  # noqa: E402
from test_gpu_batch import check_column  # noqa: E402

TAUS = [10.0 ** -k for k in range(3, 11)]


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


# ------------------------------------------------------------------ scale 22: traces and readout

@pytest.fixture(scope="module")
def rmat22():
    return gg.rmat(22, edge_factor=16, seed=22)


def test_scale22_fp64_trace_and_readout(pr, ctx, rmat22):
    g = rmat22
    dg = pr.DeviceGraph.from_host(g)
    res = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=1, max_iter=500, trace=True)
    ref = oracle.pagerank_graph(g, alpha=0.85, tau=1e-10, norm=1, max_iter=500, trace=True)
    tr = res["trace"].cpu().numpy()
    ranks = res["ranks"].cpu().numpy()
    check_fp64_result(g, ranks, res["iterations"], res["converged"], 0.85, 1e-10, 1, 500, gpu_trace=tr, ref=ref)
    k = min(len(tr), len(ref["trace"]))
    d1 = np.abs(ranks - ref["ranks"]).sum()
    print("scale-22 fp64: iterations %d / oracle %d, ranks L1 %.3e, largest trace difference %.3e"
          % (res["iterations"], ref["iterations"], d1, np.abs(tr[:k] - ref["trace"][:k]).max()))
    # every (tau, norm) stop read off the two traces; a stop decided by a near-tie may move by one
    readout = {}
    for norm in (1, 2, 3):
        for tau in TAUS:
            a = oracle.iterations_from_trace(tr, tau, norm)
            b = oracle.iterations_from_trace(ref["trace"], tau, norm)
            readout[(tau, norm)] = b
            if a != b:
                # the two traces straddle tau at the earlier stop, and agree there within the
                # distance the trace comparison above allows
                col = ref["trace"][:, norm - 1]
                assert a is not None and b is not None and abs(a - b) == 1, (tau, norm, a, b)
                j = min(a, b) - 1
                assert abs(col[j] - tau) <= abs(tr[j, norm - 1] - col[j]) <= TRACE_ATOL + 1e-9 * tau, \
                    (tau, norm, a, b, col[j], tr[j, norm - 1])
    # iterations fall as the norm goes from L1 to L2 to L-infinity at every tau (section 3)
    for tau in TAUS:
        assert readout[(tau, 1)] >= readout[(tau, 2)] >= readout[(tau, 3)], tau
    print("scale-22 readout (tau: L1/L2/Linf):",
          {t: tuple(readout[(t, n)] for n in (1, 2, 3)) for t in TAUS})


@pytest.mark.parametrize("norm", [1, 2, 3])
def test_scale22_mixed_against_oracle(pr, ctx, rmat22, norm):
    g = rmat22
    dg = pr.DeviceGraph.from_host(g)
    res = pr.pull(ctx, dg, alpha=0.85, tau=1e-10, norm=norm, precision=pr.PR_MIXED)
    assert res["converged"] and res["fp64_iters"] >= 1
    assert res["err"][norm - 1] < 1e-10
    ref, d1, dinf = check_mixed_result(g, res["ranks"].cpu().numpy(), res["err"], 0.85, 1e-10, norm)
    # the mixed form may not cost more than a few updates over float64 alone
    assert res["iterations"] <= ref["iterations"] + 3, (res["iterations"], ref["iterations"])
    print("scale-22 mixed norm %d: iterations %d (fp32 %d + fp64 %d) vs fp64 oracle %d; L1 %.3e Linf %.3e"
          % (norm, res["iterations"], res["fp32_iters"], res["fp64_iters"], ref["iterations"], d1, dinf))


# ------------------------------------------------------------------ scale 24: the timed sweep

@pytest.fixture(scope="module")
def rmat24():
    return gg.rmat(24, edge_factor=16, seed=24)


@pytest.fixture(scope="module")
def dev24(pr, ctx, rmat24):
    # prepared as the benchmark prepares it: tile partitions plus the source-segmented layout
    dg = pr.DeviceGraph.from_host(rmat24)
    dg.prepare_segmented(ctx, seg_len=1 << 19)
    yield dg
    del dg
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def sweep24(pr, ctx, dev24):
    """The benchmark's step: eleven columns, mixed precision, default launch settings."""
    probs = [dict(alpha=a, tau=1e-10, norm=3, max_iter=500) for a in gg.ALPHA_SWEEP]
    res = pr.pull_batch(ctx, dev24, probs, precision=pr.PR_MIXED)
    for r in res:
        r["ranks"] = r["ranks"].cpu().numpy()
    return probs, res


@pytest.fixture(scope="module")
def series24(pr, ctx, dev24):
    """The same eleven columns as one power-series sweep (pr_pull_sweep, float64)."""
    probs = [dict(alpha=a, tau=1e-10, norm=3, max_iter=500) for a in gg.ALPHA_SWEEP]
    res = pr.pull_sweep(ctx, dev24, probs, trace=True)
    for r in res:
        r["ranks"] = r["ranks"].cpu().numpy()
        r["trace"] = r["trace"].cpu().numpy()
    return probs, res


def test_scale24_sweep_as_benchmarked(sweep24):
    probs, res = sweep24
    report = []
    for r, p in zip(res, probs):
        a = p["alpha"]
        assert r["converged"] and r["fp64_iters"] >= 1 and r["err"][2] < 1e-10, (p, r["iterations"])
        # mass: the map sends sum(r) - 1 to alpha * (sum(r) - 1), so after a last change e1 in L1
        # the excess is at most alpha/(1-alpha) * e1; at alpha = 1 the map keeps whatever the
        # float32 phase left, a drift of float32 rounding (bounded here by 2^-16)
        m = abs(r["ranks"].sum() - 1.0)
        assert m <= (a / (1 - a) * r["err"][0] + 1e-12 if a < 1 else 2.0 ** -16), (a, m)
        report.append((a, r["iterations"], r["fp32_iters"], r["fp64_iters"], "%.2e" % m))
    print("scale-24 sweep (alpha, iterations, fp32, fp64, |sum-1|):", report)


@pytest.mark.parametrize("alpha", gg.ALPHA_SWEEP)
def test_scale24_columns_against_full_oracle(pr, ctx, rmat24, dev24, sweep24, series24, alpha):
    g = rmat24
    p = dict(alpha=alpha, tau=1e-10, norm=3, max_iter=500)
    ref = oracle.pagerank_graph(g, trace=True, **p)
    # the sequential float64 solve of the benchmark's baseline (source-segmented updates)
    f64 = pr.pull(ctx, dev24, precision=pr.PR_FP64, trace=True, **p)
    check_fp64_result(g, f64["ranks"].cpu().numpy(), f64["iterations"], f64["converged"], alpha, 1e-10, 3, 500,
                      gpu_trace=f64["trace"].cpu().numpy(), ref=ref)
    # the same column of the power-series sweep: the float64 bar
    k = list(gg.ALPHA_SWEEP).index(alpha)
    ser = series24[1][k]
    check_fp64_result(g, ser["ranks"], ser["iterations"], ser["converged"], alpha, 1e-10, 3, 500,
                      gpu_trace=ser["trace"], ref=ref)
    # the same column of the eleven-column mixed batch: the L1 bound for alpha < 1 and the stated
    # L-infinity tolerance (tests/parity.py)
    col = sweep24[1][k]
    _, d1, dinf = check_mixed_result(g, col["ranks"], col["err"], alpha, 1e-10, 3, ref=ref)
    print("scale-24 alpha %.2f: series %d, mixed batch %d (fp32 %d + fp64 %d), fp64 %d, oracle %d; mixed vs oracle "
          "L1 %.3e Linf %.3e" % (alpha, ser["iterations"], col["iterations"], col["fp32_iters"], col["fp64_iters"],
                                 f64["iterations"], ref["iterations"], d1, dinf))


# ------------------------------------------------------------------ 64 uneven graphs, full recipe

def test_uneven_batch_full_recipe(pr, ctx):
    specs = gg.many_graph_specs()
    hosts = [gg.make_spec_graph(s) for s in specs]
    graphs = [pr.DeviceGraph.from_host(h) for h in hosts]
    probs = [dict(alpha=s["alpha"], tau=s["tau"], norm=s["norm"], max_iter=500) for s in specs]
    res = pr.pull_multi(ctx, graphs, probs)
    for r, h, p in zip(res, hosts, probs):
        check_column(r, h, p)
    print("64 graphs: sum E = %d, iterations %s" % (sum(h.E for h in hosts), [r["iterations"] for r in res]))
