"""Pins of the CPU oracle against what the paper and the mathematics fix (no GPU).

Each test names the passage or the closed form it checks.  They are chosen so that a dropped
term (the dangling teleport, the (1-alpha)/N term), a wrong sign or index (summing out-edges
instead of in-edges, dividing by the in-degree), a wrong error function or a wrong stopping
rule (<= instead of <, off-by-one iteration count) fails at least one of them.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import L1, L2, LINF, dense, estimate

NORMS = (L1, L2, LINF)


def run(g, **kw):
    return oracle.pagerank_graph(g, **kw)


# ----------------------------------------------------------------- closed forms

@pytest.mark.parametrize("N", [1, 2, 7, 1000])
@pytest.mark.parametrize("alpha", [0.0, 0.5, 0.85, 1.0])
@pytest.mark.parametrize("norm", NORMS)
def test_cycle_is_uniform_after_one_iteration(N, alpha, norm):
    # Directed cycle: in = out = 1 everywhere, so 1/N is the fixed point (section 2 update).
    g = gg.cycle(N) if N > 1 else gg.edgeless(1)
    res = run(g, alpha=alpha, tau=1e-15 if N < 1000 else 1e-14, norm=norm)
    assert res["iterations"] == 1 and res["converged"]
    np.testing.assert_allclose(res["ranks"], 1.0 / N, rtol=1e-15, atol=0)


@pytest.mark.parametrize("N", [2, 3, 50])
@pytest.mark.parametrize("alpha", [0.5, 0.85, 1.0])
def test_complete_digraph_uniform(N, alpha):
    g = gg.complete(N)
    res = run(g, alpha=alpha, tau=1e-12, norm=L1)
    assert res["iterations"] == 1
    np.testing.assert_allclose(res["ranks"], 1.0 / N, rtol=1e-13)


@pytest.mark.parametrize("alpha", [0.0, 0.3, 0.85, 1.0])
def test_edgeless_graph_all_dangling(alpha):
    # All vertices dangling: c0 = (1-alpha)/N + alpha*1/N = 1/N (the dangling teleport term).
    g = gg.edgeless(37)
    res = run(g, alpha=alpha, tau=1e-12, norm=L1)
    assert res["iterations"] == 1
    np.testing.assert_allclose(res["ranks"], 1.0 / 37, rtol=1e-14)


def test_large_dangling_sum_is_exact_to_rounding():
    # A million equal dangling ranks: uniform 1/N is the exact fixed point, so one update must
    # return it to within a few ulps and the three errors must vanish to rounding.  A plain
    # running sum of the equal terms drifts by about 2e-11 relative here, which
    # would move every rank by that much and the L1 change to ~1.5e-11.
    N = 1_000_003
    g = gg.edgeless(N)
    res = run(g, alpha=0.85, tau=0.0, norm=L1, max_iter=2)
    assert np.max(np.abs(res["ranks"] * N - 1.0)) <= 8 * 2.0 ** -52
    assert res["err"][0] <= 1e-15 and res["err"][2] <= 8 * 2.0 ** -52 / N


@pytest.mark.parametrize("rows,cols", [(3, 3), (20, 30), (50, 40)])
def test_lattice_first_update_by_hand(rows, cols):
    # Road-like lattice (every cell linked both ways to its 4 neighbours), uniform start, no
    # dangling vertices.  A corner has two in-neighbours of out-degree 3, so its first update is
    # (1-alpha)/N + alpha*(2/3)/N: it falls by alpha/(3N), the largest change of any vertex (an
    # edge cell changes by alpha/(12N), interior cells by at most that).  Hence L-infinity meets
    # any tau above alpha/(3N) in a single update -- the paper's observation on road networks.
    g = gg.grid2d(rows, cols)
    N = rows * cols
    alpha = 0.85
    res = run(g, alpha=alpha, tau=0.0, norm=LINF, max_iter=1, trace=True)
    assert abs(res["trace"][0, 2] - alpha / (3 * N)) <= 1e-15 / N
    corner = res["ranks"][0]
    assert abs(corner - ((1 - alpha) / N + alpha * (2.0 / 3.0) / N)) <= 4e-16 / N * 4
    assert run(g, alpha=alpha, tau=1.01 * alpha / (3 * N), norm=LINF)["iterations"] == 1
    assert run(g, alpha=alpha, tau=0.99 * alpha / (3 * N), norm=LINF)["iterations"] > 1


def in_star_closed_form(L, alpha, k):
    """In-star (leaves -> hub, hub dangling), uniform start: leaves l_k and the three errors at step k."""
    N = L + 1
    lstar = 1.0 / (1.0 + L * (1.0 + alpha))
    rho = alpha * L / N
    e0 = alpha * L / (N * (N + alpha * L))
    lk = lstar + (-rho) ** k * e0
    base = (1.0 + rho) * rho ** (k - 1) * e0
    return lk, (2 * L * base, math.sqrt(L + L * L) * base, L * base)


def test_in_star_worked_value():
    # L = 1, alpha = .85: r* = (1.85/2.85, 1/2.85) for (hub, leaf)
    g = gg.in_star(1)
    res = run(g, alpha=0.85, tau=1e-15, norm=L1)
    np.testing.assert_allclose(res["ranks"], [1.85 / 2.85, 1.0 / 2.85], rtol=1e-13)
    assert abs(res["ranks"][1] - 0.350877193) < 1e-9 and abs(res["ranks"][0] - 0.649122807) < 1e-9


@pytest.mark.parametrize("L", [1, 3, 10])
@pytest.mark.parametrize("alpha", [0.5, 0.85, 0.95])
@pytest.mark.parametrize("norm", NORMS)
def test_in_star_exact_iterations_and_trace(L, alpha, norm):
    g = gg.in_star(L)
    # errors at every step from the hand solution
    errs = [in_star_closed_form(L, alpha, k)[1] for k in range(1, 200)]
    # choose tau between two successive errors, far from both (no tie)
    e = [x[norm - 1] for x in errs]
    kstar = 6
    tau = math.sqrt(e[kstar - 1] * e[kstar - 2])
    res = run(g, alpha=alpha, tau=tau, norm=norm, trace=True)
    assert res["iterations"] == kstar
    tr = res["trace"]
    for k in range(kstar):
        np.testing.assert_allclose(tr[k], errs[k], rtol=1e-9)
    lk, _ = in_star_closed_form(L, alpha, kstar)
    np.testing.assert_allclose(res["ranks"][1:], lk, rtol=1e-12)
    np.testing.assert_allclose(res["ranks"][0], 1.0 - L * lk, rtol=1e-12)


@pytest.mark.parametrize("L", [1, 4, 9])
@pytest.mark.parametrize("alpha", [0.5, 0.85])
def test_out_star_fixed_point(L, alpha):
    g = gg.out_star(L)
    N = L + 1
    res = run(g, alpha=alpha, tau=1e-15, norm=L1)
    h = 1.0 / (N + alpha)
    leaf = (1.0 + alpha / L) / (N + alpha)
    np.testing.assert_allclose(res["ranks"][0], h, rtol=1e-13)
    np.testing.assert_allclose(res["ranks"][1:], leaf, rtol=1e-13)


@pytest.mark.parametrize("alpha,tau,norm,expect", [
    (0.85, 1e-6, L1, 75),
])
def test_two_triangles_worked_example(alpha, tau, norm, expect):
    g = gg.two_triangles()
    init = np.array([1 / 3, 1 / 3, 1 / 3, 0, 0, 0])
    assert run(g, alpha=alpha, tau=tau, norm=norm, init=init)["iterations"] == expect


@pytest.mark.parametrize("alpha", [0.5, 0.7, 0.85, 0.95])
@pytest.mark.parametrize("norm", NORMS)
@pytest.mark.parametrize("tau", [3e-2, 1e-4, 2e-7, 1e-9])
def test_two_triangles_rate_is_alpha(alpha, norm, tau):
    # Two disjoint K3 from (1/3,1/3,1/3,0,0,0): r_k = (1 +- alpha^k)/6, so the error shrinks by
    # exactly alpha per iteration -- the rate law behind log(tau)/log(alpha) (section 1).
    g = gg.two_triangles()
    init = np.array([1 / 3, 1 / 3, 1 / 3, 0, 0, 0])
    c = {L1: 1.0, L2: 1.0 / math.sqrt(6.0), LINF: 1.0 / 6.0}[norm]
    x = math.log(tau / (c * (1 - alpha))) / math.log(alpha)
    if abs(x - round(x)) < 1e-6:
        pytest.skip("tie")
    expect = 1 if tau > c * (1 - alpha) else math.floor(x) + 2
    res = run(g, alpha=alpha, tau=tau, norm=norm, init=init, trace=True)
    assert res["iterations"] == expect
    k = res["iterations"]
    np.testing.assert_allclose(res["ranks"][:3], (1 + alpha ** k) / 6, rtol=1e-12)
    np.testing.assert_allclose(res["ranks"][3:], (1 - alpha ** k) / 6, rtol=1e-10, atol=1e-15)
    for i, row in enumerate(res["trace"], start=1):
        l1 = (1 - alpha) * alpha ** (i - 1)
        np.testing.assert_allclose(row, [l1, l1 / math.sqrt(6), l1 / 6], rtol=1e-9, atol=1e-15)


# ----------------------------------------------------------------- dense solve

@pytest.mark.parametrize("seed", range(12))
def test_dense_fixed_point_random_multigraphs(seed):
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(2, 64))
    m = int(rng.integers(0, 4 * N))
    g = gg.random_small(N, m, seed, dedupe=False, self_loops=True)  # duplicates, self-loops, dangling
    alpha = float(rng.uniform(0.0, 0.99))
    rstar = dense.fixed_point(g.N, g.off, g.idx, g.outdeg, alpha)
    res = run(g, alpha=alpha, tau=1e-13, norm=L1, max_iter=5000)
    assert res["converged"]
    bound = alpha / (1 - alpha) * res["err"][0] + 1e-13
    assert np.abs(res["ranks"] - rstar).sum() <= bound
    if alpha == 0.0:
        assert res["iterations"] == 1


@pytest.mark.parametrize("seed", range(6))
def test_one_step_equals_matrix_form(seed):
    # one update of the oracle equals alpha*S^T r + (1-alpha)/N with the dense row-stochastic S
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 40))
    g = gg.random_small(N, int(rng.integers(0, 3 * N)), seed + 50, dedupe=False, self_loops=True)
    r0 = rng.random(N)
    r0 /= r0.sum()
    alpha = float(rng.uniform(0, 1))
    res = run(g, alpha=alpha, tau=0.0, norm=L1, max_iter=1, init=r0)
    np.testing.assert_allclose(res["ranks"], dense.apply_map(g.N, g.off, g.idx, g.outdeg, alpha, r0),
                               rtol=1e-13, atol=1e-16)
    d = res["ranks"] - r0
    np.testing.assert_allclose(res["err"], [np.abs(d).sum(), np.sqrt((d * d).sum()), np.abs(d).max()],
                               rtol=1e-12, atol=1e-18)


def test_alpha_zero_is_uniform_in_one_iteration():
    g = gg.random_small(30, 90, 3)
    res = run(g, alpha=0.0, tau=1e-15, norm=L1)
    assert res["iterations"] == 1
    np.testing.assert_allclose(res["ranks"], 1 / 30, rtol=1e-15)


# ----------------------------------------------------------------- invariants and bounds

@pytest.fixture(scope="module")
def c1():
    return gg.workload_c1()


@pytest.fixture(scope="module")
def rmat14():
    return gg.rmat(14, seed=5)


def test_sum_is_one(c1, rmat14):
    for g in (c1, rmat14):
        for alpha in (0.5, 0.85, 1.0):
            r = run(g, alpha=alpha, tau=1e-10, norm=L1)["ranks"]
            assert abs(math.fsum(r) - 1.0) <= 1e-12


@pytest.mark.parametrize("alpha", [0.5, 0.85, 0.95])
def test_l1_contraction_and_norm_order(rmat14, alpha):
    res = run(rmat14, alpha=alpha, tau=0.0, norm=L1, max_iter=60, trace=True)
    tr = res["trace"]
    e1 = tr[:, 0]
    # L1 errors shrink at least by alpha per iteration (alpha-contraction), checked while the
    # error is far above the FP64 rounding floor (about avg-degree * 1e-16 here)
    for k in range(1, len(e1)):
        if e1[k - 1] > 1e-12:
            assert e1[k] <= alpha * e1[k - 1] * (1 + 1e-9)
    # ||.||inf <= ||.||2 <= ||.||1 at every iteration, hence iter(Linf) <= iter(L2) <= iter(L1)
    assert np.all(tr[:, 2] <= tr[:, 1] * (1 + 1e-15)) and np.all(tr[:, 1] <= tr[:, 0] * (1 + 1e-15))
    for tau in (1e-3, 1e-6, 1e-9):
        its = [oracle.iterations_from_trace(tr, tau, p) for p in NORMS]
        assert its[2] <= its[1] <= its[0]


@pytest.mark.parametrize("alpha", [0.5, 0.85, 0.99])
def test_l1_iteration_bound(c1, alpha):
    # from the uniform start e1 <= 2 alpha, and e_k <= alpha^(k-1) e1, so
    # iterations <= 2 + floor(log(tau/(2 alpha))/log(alpha)); alpha=.85, tau=1e-6 -> <= 90
    for tau in (1e-3, 1e-6, 1e-9):
        res = run(c1, alpha=alpha, tau=tau, norm=L1)
        assert res["iterations"] <= 2 + math.floor(math.log(tau / (2 * alpha)) / math.log(alpha))
    assert 2 + math.floor(math.log(1e-6 / 1.7) / math.log(0.85)) == 90


def test_trace_readout_equals_separate_runs(c1):
    res = run(c1, alpha=0.85, tau=0.0, norm=L1, max_iter=60, trace=True)
    for tau in gg.TAU_DECADES:
        for p in NORMS:
            k = oracle.iterations_from_trace(res["trace"], tau, p)
            assert run(c1, alpha=0.85, tau=tau, norm=p)["iterations"] == k


def test_tau_monotone(c1):
    its = [run(c1, alpha=0.85, tau=t, norm=L1)["iterations"] for t in gg.tau_sweep_21()]
    assert all(a <= b for a, b in zip(its, its[1:]))


def test_max_iter_halt_returns_last_iterate(c1):
    res = run(c1, alpha=0.85, tau=0.0, norm=L1, max_iter=7)
    ref = run(c1, alpha=0.85, tau=0.0, norm=L1, max_iter=500)
    assert not res["converged"] and res["iterations"] == 7
    assert not ref["converged"] and ref["iterations"] == 500
    seven = run(c1, alpha=0.85, tau=0.0, norm=L1, max_iter=7)
    assert np.array_equal(res["ranks"], seven["ranks"])


# ----------------------------------------------------------------- determinism, resume, relabel

def test_bitwise_repeatable_and_thread_independent(rmat14):
    a = run(rmat14, alpha=0.85, tau=1e-10, norm=L2, threads=1)
    b = run(rmat14, alpha=0.85, tau=1e-10, norm=L2, threads=4)
    c = run(rmat14, alpha=0.85, tau=1e-10, norm=L2, threads=4)
    assert a["iterations"] == b["iterations"] == c["iterations"]
    assert np.array_equal(a["ranks"], b["ranks"]) and np.array_equal(b["ranks"], c["ranks"])


def test_resume_is_bitwise(c1):
    full = run(c1, alpha=0.85, tau=0.0, norm=L1, max_iter=11)
    part = run(c1, alpha=0.85, tau=0.0, norm=L1, max_iter=4)
    rest = run(c1, alpha=0.85, tau=0.0, norm=L1, max_iter=7, init=part["ranks"])
    assert np.array_equal(full["ranks"], rest["ranks"])


def test_relabel_equivariance():
    g = gg.rmat(12, seed=9)
    p = gg.permutation(g.N, 77)
    h = gg.relabel(g, p)
    a = run(g, alpha=0.85, tau=1e-12, norm=L1)
    b = run(h, alpha=0.85, tau=1e-12, norm=L1)
    assert np.abs(b["ranks"][p] - a["ranks"]).sum() <= 1e-14


def test_pure_python_definition_agrees_bitwise():
    g = gg.random_small(25, 70, 11, dedupe=False, self_loops=True)
    for p in NORMS:
        a = run(g, alpha=0.85, tau=1e-9, norm=p)
        b = oracle.pagerank_py(g.N, g.off, g.idx, g.outdeg, alpha=0.85, tau=1e-9, norm=p)
        assert a["iterations"] == b["iterations"]
        assert np.array_equal(a["ranks"], b["ranks"])


def test_invalid_arguments():
    g = gg.cycle(4)
    for kw in (dict(alpha=-0.1), dict(alpha=1.5), dict(tau=-1.0), dict(tau=float("nan")), dict(norm=4),
               dict(max_iter=0)):
        with pytest.raises(ValueError):
            run(g, **kw)


# ----------------------------------------------------------------- section 1 estimate

@pytest.mark.parametrize("tau,alpha,expect", [(1e-6, 0.85, 85), (1e-6, 0.95, 269), (1e-6, 0.75, 48),
                                              (1e-9, 0.85, 128), (1e-3, 0.85, 43)])
def test_iteration_estimate_matches_paper(tau, alpha, expect):
    assert estimate.rounded(tau, alpha) == expect


# ------------------------------------------------------------------ the sweep as a power series
# The GPU's one-iteration sweep (pr_pull_sweep) rests on an identity of the section-2 map, checked
# here on the oracle alone: from the uniform start, k updates at damping factor a give
# a^k v_k + (1 - a) sum_{j<k} a^j v_j with v_j the iterates at a = 1 from the same start, and the
# change of update k is a^k times the a = 1 change, in every norm.

@pytest.mark.parametrize("seed", [3, 4])
def test_power_series_identity_of_the_update(seed):
    g = gg.rmat(11, seed=seed)  # with dangling vertices, duplicates removed
    K = 25
    v = [oracle.pagerank_graph(g, alpha=1.0, tau=0.0, max_iter=k, trace=True) if k else None for k in range(K + 1)]
    vs = [np.full(g.N, 1.0 / g.N)] + [x["ranks"] for x in v[1:]]
    e1 = v[K]["trace"]  # the a = 1 changes of updates 1..K
    for a in (0.0, 0.5, 0.85, 0.99, 1.0):
        ref = oracle.pagerank_graph(g, alpha=a, tau=0.0, max_iter=K, trace=True)
        for k in (1, 7, K):
            rk = oracle.pagerank_graph(g, alpha=a, tau=0.0, max_iter=k)["ranks"]
            series = a ** k * vs[k] + (1 - a) * sum(a ** j * vs[j] for j in range(k))
            assert np.abs(series - rk).sum() <= 1e-13
        # the changes agree up to the rounding of the iterates themselves (a few float64 ulps of
        # sum(r) = 1 summed over the vertices), which dominates once the changes near 1e-12
        for k in range(1, K + 1):
            np.testing.assert_allclose(ref["trace"][k - 1], a ** k * e1[k - 1], rtol=1e-9, atol=1e-15)


def test_power_series_stops_like_separate_solves():
    # every column's stop (first k with a^k e_k < tau in its norm) equals its own solve's count
    g = gg.workload_c1()
    one = oracle.pagerank_graph(g, alpha=1.0, tau=0.0, max_iter=200, trace=True)["trace"]
    for a in (0.5, 0.7, 0.85, 0.95):
        for norm in (L1, L2, LINF):
            for tau in (1e-4, 1e-8, 1e-11):
                own = oracle.pagerank_graph(g, alpha=a, tau=tau, norm=norm)
                ks = [k for k in range(1, 201) if a ** k * one[k - 1, norm - 1] < tau]
                assert ks and ks[0] == own["iterations"], (a, norm, tau, ks[:1], own["iterations"])
