"""Exact fixed point of the pull iteration by a dense linear solve -- TEST INFRASTRUCTURE.

The update of the paper's section 2 is the affine map G(r) = alpha * S^T r + (1 - alpha)/N * 1
where S is row-stochastic: S[u, v] = (number of u->v entries)/d_u when u has out-edges, and
S[u, v] = 1/N for every v when u is dangling (the common teleport contribution spreads a
dangling vertex's rank over all N vertices).  For alpha < 1, G is an alpha-contraction in L1,
so its unique fixed point solves (I - alpha S^T) r = (1 - alpha)/N * 1, and sums to 1.
Only for tiny graphs (N up to a few hundred).
"""
from __future__ import annotations

import numpy as np


def transition_matrix(N, off, idx, outdeg):
    """Row-stochastic S of the section-2 update, built from the in-edge CSR (FP64, dense)."""
    S = np.zeros((N, N), dtype=np.float64)
    for v in range(N):
        for j in range(int(off[v]), int(off[v + 1])):
            u = int(idx[j])
            S[u, v] += 1.0 / float(outdeg[u])
    for u in range(N):
        if outdeg[u] == 0:
            S[u, :] = 1.0 / N
    return S


def fixed_point(N, off, idx, outdeg, alpha):
    """r* with (I - alpha S^T) r* = (1 - alpha)/N * 1, by LAPACK's partial-pivot LU (numpy.linalg.solve)."""
    if not alpha < 1.0:
        raise ValueError("the dense system is singular for alpha = 1")
    S = transition_matrix(N, off, idx, outdeg)
    A = np.eye(N) - alpha * S.T
    b = np.full(N, (1.0 - alpha) / N)
    return np.linalg.solve(A, b)


def apply_map(N, off, idx, outdeg, alpha, r):
    """One application of G written with the dense matrix: alpha * S^T r + (1 - alpha)/N."""
    S = transition_matrix(N, off, idx, outdeg)
    return alpha * (S.T @ np.asarray(r, dtype=np.float64)) + (1.0 - alpha) / N
