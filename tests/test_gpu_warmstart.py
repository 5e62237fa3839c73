"""Learned warm start: GPU kernels against oracle.mlp, and what the trained network gains.

Both sides store the hidden activations as bfloat16 (the network's specification); the oracle
accumulates in float64, the GPU in float32, so a pre-activation that lies within float32 noise of
a bfloat16 rounding boundary can round the other way.  Forward tolerance (per vertex): every
activation may be one bfloat16 ulp (2^-8 relative) off, so
|y_gpu - y| <= 2^-8 * (sum_j |W3_j| h2_j + sum_j |W3_j| sum_k |W2_jk| h1_k) + 1e-5.
The gradient is checked against the oracle's own forward and backward; the rare rounding flips
and float32 accumulation stay below 1e-3 of the same chain rule applied to absolute values.
No oracle input comes from the GPU.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pr():
    import paper_2108_02997_amd as pr
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return pr


@pytest.fixture(scope="module")
def ws(pr):
    from paper_2108_02997_amd import warmstart
    return warmstart


@pytest.fixture(scope="module")
def ctx(pr):
    c = pr.Context(0)
    yield c
    c.close()


def test_features_and_target(pr, ws, ctx):
    rng = np.random.default_rng(0)
    N = 40000
    src, dst = [], []
    for v, deg in ((0, 20000), (1, 9000), (2, 3000)):
        src.extend(rng.choice(N, size=deg, replace=False).tolist())
        dst.extend([v] * deg)
    src.extend(rng.integers(0, N, 100000).tolist())
    dst.extend(rng.integers(0, N, 100000).tolist())
    g = gg.from_edges(N, src, dst)
    r85 = oracle.pagerank_graph(g, alpha=0.85, tau=1e-12)["ranks"]
    r95 = oracle.pagerank_graph(g, alpha=0.95, tau=1e-12)["ranks"]
    dg = pr.DeviceGraph.from_host(g)
    feat, target = ws.features(ctx, dg, torch.from_numpy(r85).cuda(), 0.95, torch.from_numpy(r95).cuda())
    ref = omlp.features(g.N, g.off, g.idx, g.outdeg, r85, 0.95)
    np.testing.assert_allclose(feat.cpu().numpy(), ref, rtol=2e-6, atol=2e-6)
    np.testing.assert_allclose(target.cpu().numpy(), np.log(r95 / r85), rtol=2e-6, atol=2e-6)


def forward_bound(W, cache):
    p = omlp.unpack(W)
    a3 = np.abs(p["W3"])
    t1 = cache["h2"] @ a3
    t2 = cache["h1"] @ (np.abs(p["W2"]).T @ a3)
    return 2.0 ** -8 * (t1 + t2) + 1e-5


@pytest.mark.parametrize("n", [5000, 1, 33, 4096])
def test_forward_backward_adam_against_oracle(pr, ws, ctx, n):
    # 32-vertex tiles: a ragged last tile (5000, 33), a single vertex, whole tiles only (4096)
    rng = np.random.default_rng(1)
    X = np.column_stack([rng.uniform(0, 6, n), rng.uniform(0, 6, n), rng.normal(0, 2, n), rng.normal(0, 2, n),
                         np.full(n, 0.9)]).astype(np.float32)
    # seeded weights drawn here, given to both sides: He-uniform scales, small biases
    parts = []
    for name, shape in omlp.SIZES:
        fan_in = 5 if name in ("W1", "b1") else 32
        lim = np.sqrt(6.0 / fan_in) if name.startswith("W") else 0.1
        parts.append(rng.uniform(-lim, lim, size=int(np.prod(shape))))
    W = np.concatenate(parts)
    W64 = W.astype(np.float32).astype(np.float64)
    Wt = torch.from_numpy(W.astype(np.float32)).cuda()
    feat = torch.from_numpy(X).cuda()
    y, act = ws.forward(ctx, Wt, feat, keep_activations=True)
    yr, cache = omlp.forward(W64, X.astype(np.float64), activations="bf16")
    bound = forward_bound(W64, cache)
    err = np.abs(y.cpu().numpy() - yr)
    assert np.all(err <= bound), float(np.max(err / bound))
    # the GPU's stored activations are the oracle's, but for the rare boundary flips
    bits = act.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    hv = bits.view(np.float32).astype(np.float64)
    flips = int((hv[:, :32] != cache["h1"]).sum() + (hv[:, 32:] != cache["h2"]).sum())
    assert flips <= 1e-3 * hv.size, flips
    # loss and gradient of the mean squared error, each side from its own forward
    target = (yr + rng.normal(0, 0.5, n)).astype(np.float32)
    dW, loss = ws.backward(ctx, Wt, feat, act, y, torch.from_numpy(target).cuda())
    lref, dy = omlp.mse(yr, target)
    dyr = np.abs(yr - target.astype(np.float64))
    assert abs(loss - lref) <= np.mean(2 * dyr * bound + bound * bound) + 1e-12
    gref = omlp.backward(W64, cache, dy)
    acache = dict(X=np.abs(cache["X"]), z1=cache["z1"], h1=cache["h1"], z2=cache["z2"], h2=cache["h2"])
    gabs = omlp.backward(np.abs(W64), acache, np.abs(dy) + 2.0 * bound / n)
    g = dW.cpu().numpy()
    assert np.all(np.abs(g - gref) <= 1e-3 * gabs + 1e-12), float(np.max(np.abs(g - gref) / (gabs + 1e-30)))
    # repeatable: fixed-order reductions
    dW2, loss2 = ws.backward(ctx, Wt, feat, act, y, torch.from_numpy(target).cuda())
    assert torch.equal(dW, dW2) and loss == loss2
    # Adam from zero moments, two steps, on a seeded gradient given to both sides
    gs = rng.normal(0, 1e-2, W.size).astype(np.float32)
    m = torch.zeros_like(Wt)
    v = torch.zeros_like(Wt)
    Wg = Wt.clone()
    gt = torch.from_numpy(gs).cuda()
    ws.adam_step(ctx, Wg, gt, m, v, 1, lr=1e-2)
    ws.adam_step(ctx, Wg, gt, m, v, 2, lr=1e-2)
    Wr, mr, vr = omlp.adam(W64, gs.astype(np.float64), np.zeros_like(W), np.zeros_like(W), 1, lr=1e-2)
    Wr, mr, vr = omlp.adam(Wr, gs.astype(np.float64), mr, vr, 2, lr=1e-2)
    np.testing.assert_allclose(Wg.cpu().numpy(), Wr, rtol=1e-5, atol=1e-6)


def test_start_vector(pr, ws, ctx):
    rng = np.random.default_rng(2)
    n = 3000
    X = np.zeros((n, 5), np.float32)
    X[:, 2] = rng.normal(0, 2, n)
    y = rng.normal(0, 0.3, n).astype(np.float32)
    r0 = ws.start_vector(ctx, torch.from_numpy(X).cuda(), torch.from_numpy(y).cuda()).cpu().numpy()
    np.testing.assert_allclose(r0, omlp.start_vector(X.astype(np.float64), y.astype(np.float64)), rtol=1e-12)
    assert abs(r0.sum() - 1.0) < 1e-13


def test_trained_network_gains_over_uniform_start(pr, ws, ctx):
    # train on six seeded R-MAT scale-14 graphs, evaluate on an unseen scale-15 graph
    model = ws.WarmStart(ctx, seed=0)
    train_alphas = [0.5, 0.6, 0.7, 0.75, 0.8, 0.9, 0.95, 0.99]
    samples = []
    for s in range(6):
        samples += model.make_samples(pr.DeviceGraph.from_host(gg.rmat(14, seed=2000 + s)), train_alphas)
    hist = model.train(samples, epochs=25, lr=3e-3)
    assert hist[-1] < 0.5 * hist[0]
    g = gg.rmat(15, seed=3000)
    dg = pr.DeviceGraph.from_host(g)
    r85 = pr.pull(ctx, dg, alpha=0.85, tau=1e-12, norm=1)["ranks"]
    report = []
    for alpha in (0.9, 0.95, 0.99):
        uni = pr.pull(ctx, dg, alpha=alpha, tau=1e-10, norm=3)
        from85 = pr.pull(ctx, dg, alpha=alpha, tau=1e-10, norm=3, init=r85)
        mlp_r0 = model.propose(dg, r85, alpha)
        frommlp = pr.pull(ctx, dg, alpha=alpha, tau=1e-10, norm=3, init=mlp_r0)
        chosen, name, e, steps, _ = model.start(dg, r85, alpha, norm=3)
        judged = pr.pull(ctx, dg, alpha=alpha, tau=1e-10, norm=3, init=chosen)
        report.append((alpha, uni["iterations"], from85["iterations"], frommlp["iterations"], name,
                       steps + judged["iterations"]))
        # the judged column's last change is never above the uniform start's
        assert e[("mlp", "r085", "uniform").index(name)] <= e[2]
        # corrected ranks agree with the oracle's (L1 a-posteriori bound of the section-2 map)
        ref = oracle.pagerank_graph(g, alpha=alpha, tau=1e-10, norm=3)
        d = np.abs(frommlp["ranks"].cpu().numpy() - ref["ranks"]).sum()
        assert d <= alpha / (1 - alpha) * (frommlp["err"][0] + ref["err"][0]) + 1e-12
    print("warm start iterations (alpha, uniform, r085, mlp, judged choice, judged):", report)
    assert sum(r[3] for r in report) < sum(r[1] for r in report)
    assert sum(r[5] for r in report) <= sum(r[1] for r in report)


def test_scale24_warm_started_column_against_oracle(pr, ws, ctx):
    """A warm-started column of the scale-24 evaluation graph (seed 3000), alpha = 0.95, tau = 1e-10
    (L-infinity): the judged start (network, alpha = 0.85 ranks or uniform, three float64
    look-ahead updates) and the solve from it, checked against the float64 oracle started from
    the same vector (float64 parity), and against the oracle's uniform-start solve (the section-2
    map's L1 fixed-point bound and the stated L-infinity tolerance)."""
    from parity import check_fp64_result, mixed_linf_bound
    model = ws.WarmStart(ctx, seed=0)
    samples = []
    for s in range(4):  # a short training: the check is on the solve from whatever start it proposes
        samples += model.make_samples(pr.DeviceGraph.from_host(gg.rmat(16, seed=2000 + s)), [0.8, 0.9, 0.95, 0.99])
    model.train(samples, epochs=10, lr=3e-3)
    del samples
    g = gg.rmat(24, edge_factor=16, seed=3000)
    dg = pr.DeviceGraph.from_host(g).prepare(ctx)
    alpha, tau, norm = 0.95, 1e-10, 3
    r85 = pr.pull(ctx, dg, alpha=0.85, tau=tau, norm=norm)["ranks"]
    chosen, name, e, steps, _ = model.start(dg, r85, alpha, norm=norm)
    res = pr.pull(ctx, dg, alpha=alpha, tau=tau, norm=norm, init=chosen, trace=True)
    assert res["converged"]
    init = chosen.cpu().numpy()
    got = res["ranks"].cpu().numpy()
    check_fp64_result(g, got, res["iterations"], res["converged"], alpha, tau, norm, 500, init=init,
                      gpu_trace=res["trace"].cpu().numpy())
    ref = oracle.pagerank_graph(g, alpha=alpha, tau=tau, norm=norm)
    diff = np.abs(got - ref["ranks"])
    d1, dinf = float(diff.sum()), float(diff.max())
    assert d1 <= alpha / (1 - alpha) * (res["err"][0] + ref["err"][0]) + 1e-13
    assert dinf <= mixed_linf_bound(alpha, res["err"][2], ref["err"][2])
    print("scale 24, alpha 0.95: judged start %s (+%d look-ahead updates), %d updates from it; oracle from "
          "uniform %d; L1 %.2e, Linf %.2e" % (name, steps, res["iterations"], ref["iterations"], d1, dinf))


@pytest.mark.parametrize("make", [lambda: gg.edgeless(5), lambda: gg.cycle(7), lambda: gg.in_star(40),
                                  lambda: gg.out_star(9), gg.two_triangles, lambda: gg.complete(1)])
def test_features_on_tiny_and_degenerate_graphs(pr, ws, ctx, make):
    g = make()
    r85 = oracle.pagerank_graph(g, alpha=0.85, tau=1e-12)["ranks"]
    dg = pr.DeviceGraph.from_host(g)
    feat, _ = ws.features(ctx, dg, torch.from_numpy(r85).cuda(), 0.9)
    ref = omlp.features(g.N, g.off, g.idx, g.outdeg, r85, 0.9)
    np.testing.assert_allclose(feat.cpu().numpy(), ref, rtol=2e-6, atol=2e-6)
