"""The six composite mean ratios of the paper's section 1 -- TEST INFRASTRUCTURE.

For values X[case][approach] (times or iterations, all positive) and a baseline approach b:
  RATIO-AM / RATIO-GM / RATIO-HM : per case the ratio X[c][a] / X[c][b], then the
                                    arithmetic / geometric / harmonic mean over cases;
  AM-RATIO / GM-RATIO / HM-RATIO : the arithmetic / geometric / harmonic mean of each
                                    approach over cases first, then the ratio to b's mean.
The mean-first forms do not depend on the baseline; GM-RATIO equals RATIO-GM.
Section 4 nests the means: a mean over graphs for each tolerance, then a mean of those.
"""
from __future__ import annotations

import math


def am(xs):
    xs = list(xs)
    return sum(xs) / len(xs)


def gm(xs):
    xs = list(xs)
    return math.exp(sum(math.log(x) for x in xs) / len(xs))


def hm(xs):
    xs = list(xs)
    return len(xs) / sum(1.0 / x for x in xs)


MEANS = {"AM": am, "GM": gm, "HM": hm}


def ratio_then_mean(X, a, b, mean):
    """RATIO-<mean> of approach a with respect to baseline b."""
    return MEANS[mean]([row[a] / row[b] for row in X])


def mean_then_ratio(X, a, b, mean):
    """<mean>-RATIO of approach a with respect to baseline b."""
    f = MEANS[mean]
    return f([row[a] for row in X]) / f([row[b] for row in X])


def all_six(X, b):
    """dict name -> list over approaches of the composite ratio with respect to baseline b."""
    n = len(X[0])
    out = {}
    for m in ("AM", "GM", "HM"):
        out[m + "-RATIO"] = [mean_then_ratio(X, a, b, m) for a in range(n)]
        out["RATIO-" + m] = [ratio_then_mean(X, a, b, m) for a in range(n)]
    return out


def nested_mean_ratio(Y, b, mean):
    """Section 4: Y[tau][graph][approach]; mean over graphs per tau, mean over tau, then ratio to b."""
    f = MEANS[mean]
    per_tau = [[f([g[a] for g in Yt]) for a in range(len(Yt[0]))] for Yt in Y]
    tot = [f([pt[a] for pt in per_tau]) for a in range(len(per_tau[0]))]
    return [t / tot[b] for t in tot]
