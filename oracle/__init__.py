"""CPU oracle for the pull-PageRank path -- TEST INFRASTRUCTURE, not part of the product.

Plain, slow, obviously correct reference implementations of what the GPU library computes,
written from the paper (Sahu, Kothapalli, Banerjee, "Adjusting PageRank parameters and
Comparing results", arXiv 2108.02997) and, for the learned warm start, from the textbook
definitions of a multilayer perceptron and of Adam.  Only tests/, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code with the GPU
library and never imports it.

Contents
  pagerank()             FP64 pull PageRank (section 2 update, section 3 error functions),
                         native C in pagerank_oracle.c, bitwise reproducible
  pagerank_py()          the same definition as pure-Python loops, for tiny graphs only
  dense.fixed_point()    the exact fixed point by a dense linear solve (tiny graphs)
  iterations_from_trace  the first iteration whose error meets (tau, norm)
  estimate.iterations    the log10(tau)/log10(alpha) estimate of section 1
  ratios                 the six composite mean ratios of sections 1 and 3
  mlp                    FP64 forward/backward of the warm-start MLP, its features, Adam
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pagerank_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_pr.so")
_lib = None

L1, L2, LINF = 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the C oracle (gcc -O2, OpenMP for the per-vertex gather only, no FP contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i32p, f64p = ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
        lib.oracle_pagerank.argtypes = [ctypes.c_int64, i32p, i32p, i32p, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_int, ctypes.c_int32, f64p, f64p, f64p, i32p, i32p, f64p,
                                        ctypes.c_int]
        lib.oracle_pagerank.restype = ctypes.c_int
        lib.oracle_max_threads.argtypes = []
        lib.oracle_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def max_threads() -> int:
    return int(_load().oracle_max_threads())


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def pagerank(N, off, idx, outdeg, alpha=0.85, tau=1e-6, norm=L1, max_iter=500, init=None, trace=False,
             threads=0):
    """FP64 pull PageRank.  Returns dict(ranks, iterations, converged, err=(e1,e2,einf), trace)."""
    off_a, off_p = _i32(off)
    idx_a, idx_p = _i32(idx if len(idx) else np.zeros(1, np.int32))
    deg_a, deg_p = _i32(outdeg)
    ranks = np.empty(N, dtype=np.float64)
    tr = np.full((max_iter, 3), np.nan) if trace else None
    if init is not None:
        init_a, init_p = _f64(init)
    else:
        init_a, init_p = None, None
    it = ctypes.c_int32(0)
    cv = ctypes.c_int32(0)
    err = np.zeros(3, dtype=np.float64)
    rc = _load().oracle_pagerank(N, off_p, idx_p, deg_p, float(alpha), float(tau), int(norm), int(max_iter),
                                 init_p, ranks.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                 tr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if trace else None,
                                 ctypes.byref(it), ctypes.byref(cv),
                                 err.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(threads))
    if rc < 0:
        raise ValueError("oracle_pagerank: invalid arguments (status %d)" % rc)
    k = int(it.value)
    return dict(ranks=ranks, iterations=k, converged=bool(cv.value), err=tuple(float(x) for x in err),
                trace=tr[:k] if trace else None)


def pagerank_graph(g, **kw):
    return pagerank(g.N, g.off, g.idx, g.outdeg, **kw)


def _compensated_sum(xs):
    """Neumaier's compensated running sum, step for step as in the C oracle."""
    s = c = 0.0
    for x in xs:
        t = s + x
        if abs(s) >= abs(x):
            c += (s - t) + x
        else:
            c += (x - t) + s
        s = t
    return s + c


def pagerank_py(N, off, idx, outdeg, alpha=0.85, tau=1e-6, norm=L1, max_iter=500, init=None):
    """The same definition as pure-Python loops (tiny graphs only)."""
    r = [1.0 / N] * N if init is None else [float(x) for x in init]
    errs = (0.0, 0.0, 0.0)
    for k in range(1, max_iter + 1):
        D = _compensated_sum(r[u] for u in range(N) if outdeg[u] == 0)
        c0 = (1.0 - alpha) / N + (alpha * D) / N
        rn = []
        for v in range(N):
            s = 0.0
            for j in range(int(off[v]), int(off[v + 1])):
                u = int(idx[j])
                s += r[u] / float(outdeg[u])
            rn.append(c0 + alpha * s)
        d = [abs(a - b) for a, b in zip(rn, r)]
        errs = (_compensated_sum(d), math.sqrt(_compensated_sum(x * x for x in d)), max(d))
        r = rn
        if errs[norm - 1] < tau:
            return dict(ranks=np.array(r), iterations=k, converged=True, err=errs)
    return dict(ranks=np.array(r), iterations=max_iter, converged=False, err=errs)


def iterations_from_trace(trace, tau, norm):
    """First iteration (1-based) whose error in `norm` is strictly below tau, or None."""
    col = np.asarray(trace)[:, norm - 1]
    hit = np.nonzero(col < tau)[0]
    return int(hit[0]) + 1 if hit.size else None


from . import dense, estimate, ratios, mlp  # noqa: E402,F401
