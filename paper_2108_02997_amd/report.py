"""Reports of the paper's sections 3 and 4, computed from solver outputs (host arithmetic only).

* `stops`: the iteration at which each (tolerance, error function) pair would have stopped a
  solve, read off one norm trace (section 3: the iterates do not depend on tau or the norm, only
  the stopping point does, so one traced solve to the smallest tau answers every pair).
* `composite`: the six composite mean ratios of section 1 (tables 3.1 and 3.2): for a table
  X[case][approach] of positive times or iterations and a baseline approach, the mean-first forms
  (AM-/GM-/HM-RATIO: mean of each approach over the cases, divided by the baseline's mean) and the
  ratio-first forms (RATIO-AM/GM/HM: per-case ratio to the baseline, then the mean).
* `nested`: section 4's two-level mean -- over the graphs for each tolerance, then over the
  tolerances -- relative to a baseline approach.
* `sensitivity` and `single_iteration`: the two iteration-count checks of sections 4 and 5. An
  approach has a sensitivity issue from the first tolerance (taken in decreasing order) at which
  it abruptly needs the maximum number of iterations while the tolerance before did not; and it
  converges in a single iteration at the tolerances where one update already meets tau.
"""
from __future__ import annotations

import numpy as np

KINDS = ("AM", "GM", "HM")


def stops(trace, taus) -> np.ndarray:
    """trace: [iterations][3] errors (L1, L2, Linf) of one solve.  Returns int array
    [len(taus)][3]: the first iteration (1-based) whose error is strictly below tau, 0 where the
    trace never gets there."""
    tr = np.asarray(trace, dtype=np.float64)
    out = np.zeros((len(taus), 3), dtype=np.int64)
    for i, tau in enumerate(taus):
        below = tr < tau                      # [iterations][3]
        hit = below.any(axis=0)
        out[i] = np.where(hit, below.argmax(axis=0) + 1, 0)
    return out


def _mean(a: np.ndarray, kind: str, axis: int = 0) -> np.ndarray:
    a = np.asarray(a, dtype=np.float64)
    if kind == "AM":
        return a.mean(axis=axis)
    if kind == "GM":
        return np.exp(np.log(a).mean(axis=axis))
    if kind == "HM":
        return a.shape[axis] / (1.0 / a).sum(axis=axis)
    raise ValueError("mean kind must be AM, GM or HM")


def composite(X, baseline: int) -> dict:
    """The six composite ratios of every approach against `baseline` (lists over approaches)."""
    X = np.asarray(X, dtype=np.float64)
    if X.ndim != 2 or not np.all(X > 0):
        raise ValueError("X must be a positive [case][approach] table")
    out = {}
    for k in KINDS:
        m = _mean(X, k, axis=0)
        out[k + "-RATIO"] = (m / m[baseline]).tolist()
        out["RATIO-" + k] = _mean(X / X[:, baseline:baseline + 1], k, axis=0).tolist()
    return out


def nested(Y, baseline: int, kind: str) -> list:
    """Y[tau][graph][approach] -> mean over graphs per tau, mean over taus, ratio to baseline."""
    Y = np.asarray(Y, dtype=np.float64)
    per_tau = _mean(Y, kind, axis=1)           # [tau][approach]
    total = _mean(per_tau, kind, axis=0)       # [approach]
    return (total / total[baseline]).tolist()


def _per_approach(iterations):
    a = np.asarray(iterations)
    return a.reshape(-1, 1) if a.ndim == 1 else a


def sensitivity(iterations, max_iter: int):
    """iterations: [tau] or [tau][approach] iteration counts, tolerances in decreasing order (a
    count >= max_iter means the solve halted at the limit; a stop read off a trace as 0 -- never
    reached -- counts as halted too).  Returns, per approach, the index of the first tolerance at
    which the count jumps to max_iter from below it (index 0 when the first one is already
    there), or None if it never does; a scalar for a one-dimensional table."""
    a = _per_approach(iterations)
    halted = (a >= max_iter) | (a == 0)
    out = []
    for j in range(a.shape[1]):
        onset = None
        for i in range(a.shape[0]):
            if halted[i, j] and (i == 0 or not halted[i - 1, j]):
                onset = i
                break
        out.append(onset)
    return out[0] if np.asarray(iterations).ndim == 1 else out


def single_iteration(iterations):
    """Per approach, the indices of the tolerances at which one iteration is enough."""
    a = _per_approach(iterations)
    out = [[int(i) for i in np.nonzero(a[:, j] == 1)[0]] for j in range(a.shape[1])]
    return out[0] if np.asarray(iterations).ndim == 1 else out
