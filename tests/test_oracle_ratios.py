"""Pins of the composite mean ratios (paper section 1, tables 3.1 and 3.2) -- no GPU."""
import math

import numpy as np
import pytest

from oracle import ratios

# Table 3.1 (mean times, ms) and table 3.2 (mean iterations): [L1, L2, Linf] per mean
T31 = {"AM": (4645, 2052, 1070), "GM": (1291, 626, 236), "HM": (351, 198, 118)}
T32 = {"AM": (57.29, 28.82, 18.94), "GM": (56.91, 27.50, 10.21), "HM": (56.51, 26.32, 3.55)}
# printed ratio rows relative to L1 and to Linf
T31_MR_L1 = {"AM": (1.00, 0.44, 0.23), "GM": (1.00, 0.48, 0.18), "HM": (1.00, 0.56, 0.34)}
T31_MR_LINF = {"AM": (4.34, 1.92, 1.00), "GM": (5.46, 2.65, 1.00), "HM": (2.98, 1.68, 1.00)}
T32_MR_L1 = {"AM": (1.00, 0.50, 0.33), "GM": (1.00, 0.48, 0.18), "HM": (1.00, 0.47, 0.06)}
T32_MR_LINF = {"AM": (3.02, 1.52, 1.00), "GM": (5.57, 2.69, 1.00), "HM": (15.91, 7.41, 1.00)}
T31_RM_L1 = {"AM": (1.00, 0.50, 0.33), "GM": (1.00, 0.48, 0.18), "HM": (1.00, 0.47, 0.06)}
T31_RM_LINF = {"AM": (15.92, 5.66, 1.00), "GM": (5.46, 2.65, 1.00), "HM": (3.03, 1.75, 1.00)}


@pytest.mark.parametrize("table,l1rows,linfrows", [(T31, T31_MR_L1, T31_MR_LINF), (T32, T32_MR_L1, T32_MR_LINF)])
def test_mean_then_ratio_rows_follow_from_the_means(table, l1rows, linfrows):
    # X-RATIO rows are the printed means divided by the baseline's mean (to the printed rounding)
    for m, means in table.items():
        X = [list(means)]  # one "case" whose values are the means: mean_then_ratio of it is a plain ratio
        for a in range(3):
            assert abs(ratios.mean_then_ratio(X, a, 0, "AM") - l1rows[m][a]) <= 0.011
            assert abs(ratios.mean_then_ratio(X, a, 2, "AM") - linfrows[m][a]) <= 0.011 * max(1, linfrows[m][a])


def test_ratio_then_mean_identities_in_table_3_1():
    # RATIO-HM(x wrt y) = 1/RATIO-AM(y wrt x): Linf wrt L1 (0.06) vs L1 wrt Linf (15.92)
    assert abs(1 / T31_RM_LINF["AM"][0] - T31_RM_L1["HM"][2]) <= 0.005
    assert abs(1 / T31_RM_L1["AM"][2] - T31_RM_LINF["HM"][0]) <= 0.01
    # RATIO-GM equals GM-RATIO
    assert T31_RM_L1["GM"] == T31_MR_L1["GM"] and T31_RM_LINF["GM"] == T31_MR_LINF["GM"]


@pytest.mark.parametrize("seed", range(5))
def test_properties_on_random_data(seed):
    rng = np.random.default_rng(seed)
    X = rng.uniform(0.1, 100, (17, 3)).tolist()
    six0 = ratios.all_six(X, 0)
    six2 = ratios.all_six(X, 2)
    for a in range(3):
        assert math.isclose(six0["GM-RATIO"][a], six0["RATIO-GM"][a], rel_tol=1e-12)
        for m in ("AM", "GM", "HM"):  # mean-first forms do not depend on the baseline
            assert math.isclose(six2[m + "-RATIO"][a], six0[m + "-RATIO"][a] / six0[m + "-RATIO"][2], rel_tol=1e-12)
        assert math.isclose(ratios.ratio_then_mean(X, a, 2, "HM"), 1 / ratios.ratio_then_mean(X, 2, a, "AM"),
                            rel_tol=1e-12)
    assert ratios.am([1, 2, 3]) == 2 and math.isclose(ratios.gm([1, 4]), 2) and math.isclose(ratios.hm([1, 3]), 1.5)
