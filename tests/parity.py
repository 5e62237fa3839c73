"""Acceptance rules shared by the GPU parity tests (imported by the test modules, not collected).

Float64 (sections 2 and 3 computed in float64 on both sides):
  * the GPU's ranks lie within 1e-12 in L1 of the oracle's ranks after the SAME number of
    updates, and the norm traces agree row by row (rtol 1e-9, atol TRACE_ATOL);
  * the iteration counts are equal, or differ by one at a tie: the two sides sum in different
    orders, so their errors at one update differ by at most the distance of their iterates at that
    update plus the distance at the update before.  With d the measured L1 distance of the two
    sides' final iterates, a count that differs by one is accepted only when the oracle's error at
    the earlier stop lies within 4 d + 1e-9 tau of tau (the factor 4 covers the two iterates and
    the slow growth of d over the updates).  The ranks are then still compared: the oracle is
    run again with tau = 0 for exactly the GPU's number of updates.

Mixed precision (float32 gather, float64 norms, a float64 update decides) and the float32-only
ablation, against the float64 oracle solved with the same settings:
  * L1: the section-2 map is an alpha-contraction in L1, so an iterate whose last L1 change is
    e lies within alpha/(1-alpha) e of the fixed point; two solves are within
    alpha/(1-alpha) (e_gpu + e_oracle) + 1e-13 of each other (mixed_bound).  Rigorous.
  * L-infinity (the stated per-vertex tolerance): near convergence the change between updates
    decays along modes that contract by at most alpha per update, so each side is within about
    e_inf alpha/(1-alpha) of the fixed point in L-infinity; before that regime the ratio of two
    successive changes can exceed alpha for a while, and the stated tolerance doubles the
    asymptotic figure:
        max_v |r_gpu - r_oracle| <= 2 (e_inf_gpu + e_inf_oracle) / (1 - alpha) + 1e-15
    for alpha < 1 (mixed_linf_bound; a float32 emulation on R-MAT scale 15 over alpha 0.5..0.99,
    tau 1e-6..1e-10 and the three norms reached at most 0.43 of it).  At alpha = 1 the map has
    no contraction factor, and where the graph has closed classes (vertex sets that no edge
    leaves and that hold no dangling vertex) its fixed point is not unique: the float32 phase's
    roundings move mass between those classes and no later float64 update moves it back (on a
    40,000-vertex random graph with hubs: 3.0e-9 at a rank of 0.19, one float32 ulp there being
    1.5e-8).  The stated tolerance at alpha = 1 is 10 tau (the last L-infinity change of a
    converged solve was below tau in every norm, since L-infinity <= L2 <= L1) plus 16 float32
    ulps of the largest rank, 2^-20 max(r).  The float32-only ablation adds the distance of the
    float32 map's fixed point: 4 * 2^-24 * max(r) / (1 - alpha) per vertex, 4 * 2^-24 / (1 - alpha)
    in L1.
"""
import numpy as np

import oracle

TRACE_ATOL = 3e-12
FP64_L1 = 1e-12


def mixed_bound(alpha, e_gpu, e_ref):
    """L1 distance allowed between two solves whose last L1 changes are e_gpu and e_ref."""
    return alpha / (1 - alpha) * (e_gpu + e_ref) + 1e-13


def mixed_linf_bound(alpha, einf_gpu, einf_ref, tau=None, norm=None, fp32_only=False, rmax=0.0):
    """Stated L-infinity distance allowed between a mixed (or float32-only) solve and its oracle."""
    if alpha >= 1.0:
        # the L-infinity change is at most the L2 or L1 change, so every converged stop had
        # e_inf < tau; with no contraction factor (and a fixed point that need not be unique)
        # the stated tolerance is ten times tau plus 16 float32 ulps of the largest rank
        assert tau is not None and tau > 0
        return 10.0 * tau + 2.0 ** -20 * rmax
    b = 2.0 * (einf_gpu + einf_ref) / (1.0 - alpha) + 1e-15
    if fp32_only:
        b += 4.0 * 2.0 ** -24 * rmax / (1.0 - alpha)
    return b


def tie_ok(ref, gpu_it, tau, norm, d):
    """A count one away from the oracle's, explained by the oracle's error at the earlier stop
    lying within 4 d + 1e-9 tau of tau (d: L1 distance of the two sides' final iterates)."""
    k = ref["iterations"]
    if abs(gpu_it - k) != 1:
        return False
    j = min(gpu_it, k) - 1
    e = ref["trace"][j, norm - 1]
    return abs(e - tau) <= 4.0 * d + 1e-9 * tau


def check_fp64_result(g, gpu_ranks, gpu_it, gpu_converged, alpha, tau, norm, max_iter, init=None, gpu_trace=None,
                      ref=None, l1_tol=FP64_L1):
    """Float64 parity of one GPU solve against the oracle; returns the oracle's run with the
    same settings.  gpu_ranks: host float64 array; gpu_trace: host [iterations][3] or None."""
    if ref is None:
        ref = oracle.pagerank_graph(g, alpha=alpha, tau=tau, norm=norm, max_iter=max_iter, init=init, trace=True)
    same = ref
    if gpu_it != ref["iterations"]:
        # the oracle for exactly the GPU's number of updates
        same = oracle.pagerank_graph(g, alpha=alpha, tau=0.0, norm=norm, max_iter=gpu_it, init=init, trace=True)
    d = float(np.abs(gpu_ranks - same["ranks"]).sum())
    assert d <= l1_tol, ("ranks", gpu_it, ref["iterations"], d)
    if gpu_trace is not None:
        np.testing.assert_allclose(gpu_trace[:gpu_it], same["trace"][:gpu_it], rtol=1e-9, atol=TRACE_ATOL)
    if gpu_it == ref["iterations"]:
        assert bool(gpu_converged) == bool(ref["converged"]), (gpu_converged, ref["converged"])
    else:
        assert tie_ok(ref, gpu_it, tau, norm, d), ("iterations", gpu_it, ref["iterations"], d,
                                                    ref["trace"][min(gpu_it, ref["iterations"]) - 1])
        # a solve that stopped before max_iter stopped because an update met tau
        if gpu_it < max_iter:
            assert gpu_converged, (gpu_it, max_iter)
    return ref


def check_mixed_result(g, gpu_ranks, gpu_err, alpha, tau, norm, max_iter=500, ref=None, fp32_only=False):
    """Mixed-precision (or float32-only) solve against the float64 oracle with the same settings:
    the L1 bound (alpha < 1) and the stated L-infinity tolerance.  Returns (ref, d1, dinf)."""
    if ref is None:
        ref = oracle.pagerank_graph(g, alpha=alpha, tau=tau, norm=norm, max_iter=max_iter)
    diff = np.abs(gpu_ranks - ref["ranks"])
    d1, dinf = float(diff.sum()), float(diff.max()) if diff.size else 0.0
    if alpha < 1.0:
        b1 = mixed_bound(alpha, gpu_err[0], ref["err"][0])
        if fp32_only:
            b1 += 4.0 * 2.0 ** -24 / (1.0 - alpha)  # sum(r) = 1, float32 rounding per vertex
        assert d1 <= b1, ("L1", alpha, tau, norm, d1, b1)
    lb = mixed_linf_bound(alpha, gpu_err[2], ref["err"][2], tau=tau, norm=norm, fp32_only=fp32_only,
                          rmax=float(ref["ranks"].max()) if ref["ranks"].size else 0.0)
    assert dinf <= lb, ("Linf", alpha, tau, norm, dinf, lb)
    return ref, d1, dinf
