"""Host-side reports (paper sections 3 and 4) of the package against the oracle's definitions."""
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle import ratios as oratios

from paper_2108_02997_amd import report


@pytest.mark.parametrize("seed", range(6))
def test_composite_ratios_match_the_definitions(seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.5, 500.0, size=(int(rng.integers(3, 30)), 3))
    for b in range(3):
        got = report.composite(X, b)
        ref = oratios.all_six(X.tolist(), b)
        assert set(got) == set(ref)
        for k in ref:
            np.testing.assert_allclose(got[k], ref[k], rtol=1e-12)
        # mean-first rows do not depend on the baseline; RATIO-GM equals GM-RATIO (section 3)
        np.testing.assert_allclose(got["GM-RATIO"], got["RATIO-GM"], rtol=1e-12)


@pytest.mark.parametrize("kind", ["AM", "GM", "HM"])
def test_nested_mean_matches_the_definition(kind):
    rng = np.random.default_rng(7)
    Y = rng.uniform(1.0, 100.0, size=(21, 9, 3))
    np.testing.assert_allclose(report.nested(Y, 0, kind), oratios.nested_mean_ratio(Y.tolist(), 0, kind), rtol=1e-12)


def test_stops_match_the_oracle_readout():
    g = gg.rmat(12, seed=4)
    ref = oracle.pagerank_graph(g, alpha=0.85, tau=1e-10, norm=1, trace=True)
    taus = gg.tau_sweep_21()
    got = report.stops(ref["trace"], taus)
    for i, tau in enumerate(taus):
        for n in (1, 2, 3):
            want = oracle.iterations_from_trace(ref["trace"], tau, n)
            assert got[i, n - 1] == (want or 0), (tau, n)
    # a tolerance no iterate reaches reads as 0
    assert report.stops(ref["trace"], [1e-300]).tolist() == [[0, 0, 0]]


def test_composite_rejects_non_positive_tables():
    with pytest.raises(ValueError):
        report.composite([[1.0, 0.0, 2.0]], 0)


def _golden_fig41():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sensitivity_fig41.txt")
    kv = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.split()
    return kv


def test_sensitivity_and_single_iteration_on_the_figure_41_description():
    kv = _golden_fig41()
    taus = [float(x) for x in kv["taus"]]
    max_iter = int(kv["max_iter"][0])
    onset = {n: taus.index(float(kv["onset " + n][0])) for n in ("L1", "L2", "Linf")}
    single = {n: taus.index(float(kv["single_iteration_down_to " + n][0])) for n in ("L2", "Linf")}
    # an iteration table with exactly the stated behaviour: counts grow as tau falls, one update
    # while the single-iteration range lasts, then the abrupt jump to the limit
    table = np.zeros((len(taus), 3), dtype=np.int64)
    for j, n in enumerate(("L1", "L2", "Linf")):
        for i in range(len(taus)):
            if i >= onset[n]:
                table[i, j] = max_iter
            elif n in single and i <= single[n]:
                table[i, j] = 1
            else:
                table[i, j] = 2 + 3 * i
    assert report.sensitivity(table, max_iter) == [onset["L1"], onset["L2"], onset["Linf"]]
    got = report.single_iteration(table)
    assert got[0] == [] and got[1] == list(range(single["L2"] + 1)) and got[2] == list(range(single["Linf"] + 1))
    # L1 is the first to suffer (section 4)
    assert taus[report.sensitivity(table[:, 0], max_iter)] > taus[report.sensitivity(table[:, 1], max_iter)]


def test_sensitivity_edge_cases():
    assert report.sensitivity([3, 5, 9, 14], 500) is None
    assert report.sensitivity([500, 500], 500) == 0
    assert report.sensitivity([4, 7, 0, 0], 500) == 2        # a stop read off a trace as 0: never reached
    assert report.sensitivity([4, 7, 499, 500, 500], 500) == 3
    assert report.single_iteration([1, 1, 2, 1]) == [0, 1, 3]
    assert report.sensitivity(np.array([[1, 500], [2, 500]]), 500) == [None, 0]
