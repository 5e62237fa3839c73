"""Many graphs in one persistent launch (pr_pull_multi): every graph equals its own oracle solve."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from test_gpu_batch import check_column  # noqa: E402


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


def small_specs(count, seed):
    # the many-graph recipe with N scaled down to [1e3, 3e4] so the oracle stays fast
    specs = gg.many_graph_specs(count, seed)
    for s in specs:
        s["N"] = max(1000, min(30000, s["N"] // 30))
    return specs


def test_uneven_batch_each_graph_matches_oracle(pr, ctx):
    specs = small_specs(24, 500)
    hosts = [gg.make_spec_graph(s) for s in specs]
    graphs = [pr.DeviceGraph.from_host(h) for h in hosts]
    probs = [dict(alpha=s["alpha"], tau=s["tau"], norm=s["norm"], max_iter=500) for s in specs]
    res = pr.pull_multi(ctx, graphs, probs, trace=True)
    for r, h, p in zip(res, hosts, probs):
        check_column(r, h, p)  # ranks, iteration count and the whole trace


def test_multi_edge_cases(pr, ctx):
    rng = np.random.default_rng(1)
    N = 30000
    src, dst = [], []
    for v, deg in ((0, 20000), (7, 9000), (8, 1500)):
        src.extend(rng.choice(N, size=deg, replace=False).tolist())
        dst.extend([v] * deg)
    src.extend(rng.integers(0, N, 50000).tolist())
    dst.extend(rng.integers(0, N, 50000).tolist())
    hosts = [gg.edgeless(1), gg.cycle(3), gg.in_star(4), gg.from_edges(N, src, dst), gg.workload_c1(),
             gg.complete(30)]
    probs = [dict(alpha=0.85, tau=1e-12, norm=1, max_iter=500), dict(alpha=0.5, tau=1e-12, norm=2, max_iter=500),
             dict(alpha=0.95, tau=1e-11, norm=3, max_iter=500), dict(alpha=0.85, tau=1e-11, norm=1, max_iter=500),
             dict(alpha=0.85, tau=0.0, norm=1, max_iter=9), dict(alpha=1.0, tau=1e-12, norm=1, max_iter=500)]
    res = pr.pull_multi(ctx, [pr.DeviceGraph.from_host(h) for h in hosts], probs)
    for r, h, p in zip(res, hosts, probs):
        check_column(r, h, p)
    assert res[4]["status"] == pr.PR_NOT_CONVERGED and not res[4]["converged"] and res[4]["iterations"] == 9


def test_multi_with_starts_and_grid(pr, ctx):
    hosts = [gg.rmat(12, seed=s) for s in range(5)]
    rng = np.random.default_rng(3)
    starts = []
    for h in hosts:
        x = rng.random(h.N)
        starts.append(x / x.sum())
    graphs = [pr.DeviceGraph.from_host(h) for h in hosts]
    probs = [dict(alpha=0.85, tau=1e-10, norm=3, max_iter=500)] * 5
    try:
        ctx.set_option("grid", 37)
        res = pr.pull_multi(ctx, graphs, probs, inits=[torch.from_numpy(s).cuda() for s in starts])
    finally:
        ctx.set_option("grid", 0)
    for r, h, p, s0 in zip(res, hosts, probs, starts):
        check_column(r, h, p, init=s0)


def test_multi_errors(pr, ctx):
    g = pr.DeviceGraph.from_host(gg.cycle(4))
    with pytest.raises(pr.PrError):
        pr.pull_multi(ctx, [g], [dict(alpha=0.85, tau=-1.0, norm=1, max_iter=10)])


def test_tau_norm_stops_from_one_launch(pr, ctx):
    # section 4 readout: every (tau, norm) stop of the 21-tolerance sweep read off the traces of
    # one many-graph launch equals the stop read off the oracle's traces (tie rule of the module)
    from paper_2108_02997_amd import report
    specs = small_specs(12, 77)
    hosts = [gg.make_spec_graph(s) for s in specs]
    graphs = [pr.DeviceGraph.from_host(h) for h in hosts]
    taus = gg.tau_sweep_21()
    probs = [dict(alpha=0.85, tau=1e-10, norm=1, max_iter=500)] * len(hosts)
    res = pr.pull_multi(ctx, graphs, probs, trace=True)
    for r, h in zip(res, hosts):
        ref = oracle.pagerank_graph(h, alpha=0.85, tau=1e-10, norm=1, trace=True)
        got = report.stops(r["trace"].cpu().numpy(), taus)
        want = report.stops(ref["trace"], taus)
        for i, tau in enumerate(taus):
            for n in range(3):
                if got[i, n] != want[i, n]:
                    col = ref["trace"][:, n]
                    k = min(got[i, n], want[i, n])
                    assert abs(got[i, n] - want[i, n]) == 1 and abs(col[k - 1] - tau) <= 1e-4 * tau, (tau, n)


def test_barrier_time_limit_ends_the_launch(pr, ctx):
    # With a zero wait limit every workgroup leaves at its first grid-barrier wait that is not
    # already met, so the launch ends normally and the call reports PR_EDEVICE; the next solve
    # (default limit) is unaffected.
    specs = small_specs(8, 900)
    hosts = [gg.make_spec_graph(s) for s in specs]
    graphs = [pr.DeviceGraph.from_host(h) for h in hosts]
    probs = [dict(alpha=s["alpha"], tau=s["tau"], norm=s["norm"], max_iter=500) for s in specs]
    assert sum(h.E for h in hosts) > 100000  # many tiles, so the launch spans every XCD
    try:
        ctx.set_option("barrier_ms", 0)
        with pytest.raises(pr.PrError) as ei:
            pr.pull_multi(ctx, graphs, probs)
        assert ei.value.status == pr._lib.PR_EDEVICE and "time limit" in str(ei.value)
    finally:
        ctx.set_option("barrier_ms", 5000)
    with pytest.raises(pr.PrError):
        ctx.set_option("barrier_ms", -1)
    for r, h, p in zip(pr.pull_multi(ctx, graphs, probs), hosts, probs):
        check_column(r, h, p)


def test_the_largest_batch_of_graphs(pr, ctx):
    # G = 4096 (the limit): the graphs' flags are staged in LDS 256 at a time and every graph is
    # finished by workgroup g % grid; each of them equals its own oracle solve
    G = 4096
    rng = np.random.default_rng(2024)
    hosts, probs = [], []
    for k in range(G):
        N = int(rng.integers(1, 120))
        hosts.append(gg.random_small(N, int(rng.integers(0, 5 * N)), 10000 + k))
        probs.append(dict(alpha=float(rng.choice([0.5, 0.85, 1.0])), tau=float(rng.choice([1e-6, 1e-10])),
                          norm=int(rng.integers(1, 4)), max_iter=int(rng.choice([7, 500]))))
    graphs = [pr.DeviceGraph.from_host(h) for h in hosts]
    res = pr.pull_multi(ctx, graphs, probs)
    assert len(res) == G
    for r, h, p in zip(res, hosts, probs):
        check_column(r, h, p)
    with pytest.raises(pr.PrError) as ei:
        pr.pull_multi(ctx, graphs + graphs[:1], probs + probs[:1])
    assert ei.value.status == pr._lib.PR_EINVAL
