"""Host-side reports (paper sections 3 and 4) of the package against the oracle's definitions."""
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
