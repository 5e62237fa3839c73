"""Seeded synthetic graph inputs for the pull-PageRank path and its CPU oracle.

This module is shared by the GPU path's tests/benchmarks and by the oracle's tests, and it
holds none of PageRank's arithmetic: it draws edges (R-MAT, Erdos-Renyi with a forced
dangling set, hand-made tiny graphs) and builds the in-edge CSR a pull iteration reads:

    off[N+1]  int32   row offsets, row v lists the sources of v's in-edges
    idx[E]    int32   source vertex ids, ascending inside each row
    outdeg[N] int32   out-degree of every vertex = its number of CSR entries

The paper's seventeen SuiteSparse graphs are not available; R-MAT graphs stand in for
its web and social graphs and Erdos-Renyi graphs serve as the non-skewed control.
The native part lives in graphgen.c and is compiled into libgraphgen.so next to it.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.c")
_LIB = os.path.join(_HERE, "libgraphgen.so")

_lib = None


def build(force: bool = False) -> str:
    """Compile graphgen.c into libgraphgen.so (gcc, -O3, OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O3", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        i64, i32p, u64 = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.c_uint64
        lib.gg_hash3.argtypes = [u64, u64, u64]
        lib.gg_hash3.restype = u64
        lib.gg_rmat_edges.argtypes = [i64, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, u64,
                                      i32p, i32p, ctypes.c_int]
        lib.gg_rmat_edges.restype = ctypes.c_int
        lib.gg_er_edges.argtypes = [i64, i64, i64, u64, i32p, i32p]
        lib.gg_er_edges.restype = ctypes.c_int
        lib.gg_permutation.argtypes = [i64, u64, i32p]
        lib.gg_permutation.restype = ctypes.c_int
        lib.gg_build_in_csr.argtypes = [i64, i64, i32p, i32p, ctypes.c_int, ctypes.c_int, i32p, i32p, i32p,
                                        ctypes.c_int]
        lib.gg_build_in_csr.restype = i64
        _lib = lib
    return _lib


def _p32(a: np.ndarray):
    assert a.dtype == np.int32 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class Graph:
    """In-edge CSR of a directed graph (see module docstring for the layout)."""

    N: int
    off: np.ndarray
    idx: np.ndarray
    outdeg: np.ndarray
    name: str = ""

    @property
    def E(self) -> int:
        return int(self.off[-1])

    @property
    def indeg(self) -> np.ndarray:
        return np.diff(self.off).astype(np.int32)

    def edges(self):
        """(src, dst) arrays of every CSR entry, in CSR order."""
        dst = np.repeat(np.arange(self.N, dtype=np.int32), np.diff(self.off))
        return self.idx.copy(), dst

    def stats(self) -> dict:
        indeg = self.indeg
        return {
            "N": self.N,
            "E": self.E,
            "dangling": int((self.outdeg == 0).sum()),
            "isolated": int(((self.outdeg == 0) & (indeg == 0)).sum()),
            "max_indeg": int(indeg.max()) if self.N else 0,
            "max_outdeg": int(self.outdeg.max()) if self.N else 0,
        }


def _threads() -> int:
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0)


def from_edges(N: int, src, dst, dedupe: bool = True, drop_self_loops: bool = True, name: str = "") -> Graph:
    """In-edge CSR of the edge list src[e] -> dst[e]."""
    src = np.ascontiguousarray(np.asarray(src, dtype=np.int32))
    dst = np.ascontiguousarray(np.asarray(dst, dtype=np.int32))
    if src.shape != dst.shape or src.ndim != 1:
        raise ValueError("src and dst must be 1-D arrays of equal length")
    m = int(src.shape[0])
    off = np.zeros(N + 1, dtype=np.int32)
    idx = np.zeros(max(m, 1), dtype=np.int32)
    outdeg = np.zeros(N, dtype=np.int32)
    E = _load().gg_build_in_csr(N, m, _p32(src), _p32(dst), int(dedupe), int(drop_self_loops), _p32(off),
                                _p32(idx), _p32(outdeg), _threads())
    if E < 0:
        raise ValueError("gg_build_in_csr failed (status %d): ids out of range or sizes invalid" % E)
    idx = idx[:E].copy() if E < idx.shape[0] else idx
    return Graph(N, off, idx, outdeg, name)


def rmat(scale: int | None = None, edge_factor: float = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, N: int | None = None, dedupe: bool = True, drop_self_loops: bool = True) -> Graph:
    """R-MAT graph.  Either scale (N = 2**scale, m = edge_factor * N) or N (m = round(edge_factor * N))."""
    if N is None:
        if scale is None:
            raise ValueError("give scale or N")
        N = 1 << int(scale)
        m = int(edge_factor) * N if float(edge_factor).is_integer() else int(round(edge_factor * N))
    else:
        m = int(round(edge_factor * N))
    src = np.empty(m, dtype=np.int32)
    dst = np.empty(m, dtype=np.int32)
    rc = _load().gg_rmat_edges(N, m, a, b, c, seed, _p32(src), _p32(dst), _threads())
    if rc != 0:
        raise ValueError("gg_rmat_edges failed (%d)" % rc)
    g = from_edges(N, src, dst, dedupe, drop_self_loops,
                   name="rmat(N=%d,ef=%g,a=%g,b=%g,c=%g,seed=%d)" % (N, edge_factor, a, b, c, seed))
    return g


def er(N: int, avg_degree: float, dangling_frac: float = 0.0, seed: int = 1) -> Graph:
    """Directed Erdos-Renyi graph: m = round(avg_degree * N) distinct pairs (u, v), v != u, u outside the
    forced dangling set of round(dangling_frac * N) vertices."""
    m = int(round(avg_degree * N))
    nd = int(round(dangling_frac * N))
    src = np.empty(max(m, 1), dtype=np.int32)
    dst = np.empty(max(m, 1), dtype=np.int32)
    rc = _load().gg_er_edges(N, m, nd, seed, _p32(src), _p32(dst))
    if rc != 0:
        raise ValueError("gg_er_edges failed (%d)" % rc)
    return from_edges(N, src[:m], dst[:m], True, True,
                      name="er(N=%d,deg=%g,dang=%g,seed=%d)" % (N, avg_degree, dangling_frac, seed))


def permutation(N: int, seed: int) -> np.ndarray:
    p = np.empty(max(N, 1), dtype=np.int32)
    rc = _load().gg_permutation(N, seed, _p32(p))
    if rc != 0:
        raise ValueError("gg_permutation failed")
    return p[:N]


def relabel(g: Graph, perm: np.ndarray) -> Graph:
    """Same graph with vertex v renamed perm[v] (duplicates and self-loops kept as they are)."""
    src, dst = g.edges()
    perm = np.asarray(perm, dtype=np.int32)
    return from_edges(g.N, perm[src], perm[dst], dedupe=False, drop_self_loops=False, name=g.name + "+relabel")


def degree_order(g: Graph) -> np.ndarray:
    """perm[v] = new id of v when vertices are ordered by decreasing out-degree, ties by id: the
    most cited sources get consecutive ids (a locality ordering for the pull gather)."""
    order = np.argsort(-np.asarray(g.outdeg, dtype=np.int64), kind="stable")
    perm = np.empty(g.N, dtype=np.int32)
    perm[order] = np.arange(g.N, dtype=np.int32)
    return perm


def hash3(seed: int, stream: int, counter: int) -> int:
    return int(_load().gg_hash3(seed, stream, counter))


# ------------------------------------------------------------------ tiny hand-made graphs

def cycle(N: int) -> Graph:
    v = np.arange(N)
    return from_edges(N, v, (v + 1) % N, name="cycle(%d)" % N)


def complete(N: int) -> Graph:
    u, v = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    m = u != v
    return from_edges(N, u[m], v[m], name="complete(%d)" % N)


def grid2d(rows: int, cols: int) -> Graph:
    """Road-like graph: a rows x cols lattice, each cell linked both ways to its 4 neighbours
    (out-degree 2..4, no dangling vertices, diameter rows + cols - 2).  A stand-in for the paper's
    road networks: large, low-degree, with every rank near 1/N."""
    i, j = np.meshgrid(np.arange(rows, dtype=np.int64), np.arange(cols, dtype=np.int64), indexing="ij")
    v = (i * cols + j).ravel()
    src, dst = [], []
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        ok = ((i + di >= 0) & (i + di < rows) & (j + dj >= 0) & (j + dj < cols)).ravel()
        src.append(v[ok])
        dst.append(((i + di) * cols + (j + dj)).ravel()[ok])
    return from_edges(rows * cols, np.concatenate(src), np.concatenate(dst), name="grid(%dx%d)" % (rows, cols))


def load_mtx(path: str, dedupe: bool = True, drop_self_loops: bool = True) -> Graph:
    """A graph from a MatrixMarket coordinate file (the format of the paper's SuiteSparse inputs):
    entry (i, j) is the edge i -> j (1-based in the file); `symmetric` files list each undirected
    edge once and get both directions; values, if any, are ignored (pattern graph).  Array-format
    files are refused."""
    with open(path) as fh:
        head = fh.readline().split()
        if len(head) < 5 or head[0] != "%%MatrixMarket" or head[1].lower() != "matrix":
            raise ValueError("%s: not a MatrixMarket matrix file" % path)
        fmt, sym = head[2].lower(), head[4].lower()
        if fmt != "coordinate":
            raise ValueError("%s: only coordinate (sparse) files hold graphs" % path)
        if sym not in ("general", "symmetric", "skew-symmetric", "hermitian"):
            raise ValueError("%s: unknown symmetry %r" % (path, sym))
        line = fh.readline()
        while line.startswith("%") or not line.strip():
            line = fh.readline()
        rows, cols, nnz = (int(x) for x in line.split()[:3])
        data = np.loadtxt(fh, dtype=np.float64, ndmin=2, max_rows=nnz, comments="%")
    if data.shape[0] != nnz or (nnz and data.shape[1] < 2):
        raise ValueError("%s: expected %d entries, found %d" % (path, nnz, data.shape[0]))
    N = max(rows, cols)
    src = data[:, 0].astype(np.int64) - 1 if nnz else np.zeros(0, np.int64)
    dst = data[:, 1].astype(np.int64) - 1 if nnz else np.zeros(0, np.int64)
    if nnz and (src.min() < 0 or dst.min() < 0 or src.max() >= N or dst.max() >= N):
        raise ValueError("%s: an entry lies outside the %d x %d matrix" % (path, rows, cols))
    if sym != "general":
        off = src != dst
        src, dst = np.concatenate([src, dst[off]]), np.concatenate([dst, src[off]])
    return from_edges(N, src, dst, dedupe=dedupe, drop_self_loops=drop_self_loops,
                      name=os.path.basename(path))


def edgeless(N: int) -> Graph:
    return from_edges(N, np.zeros(0, np.int32), np.zeros(0, np.int32), name="edgeless(%d)" % N)


def in_star(L: int) -> Graph:
    """Leaves 1..L each point to hub 0; the hub has no out-edges."""
    leaves = np.arange(1, L + 1)
    return from_edges(L + 1, leaves, np.zeros(L, np.int64), name="in_star(%d)" % L)


def out_star(L: int) -> Graph:
    """Hub 0 points to leaves 1..L; the leaves have no out-edges."""
    leaves = np.arange(1, L + 1)
    return from_edges(L + 1, np.zeros(L, np.int64), leaves, name="out_star(%d)" % L)


def two_triangles() -> Graph:
    """Two disjoint complete digraphs K3 on vertices 0-2 and 3-5."""
    src, dst = [], []
    for base in (0, 3):
        for i in range(3):
            for j in range(3):
                if i != j:
                    src.append(base + i)
                    dst.append(base + j)
    return from_edges(6, src, dst, name="two_K3")


def random_small(N: int, m: int, seed: int, dedupe: bool = False, self_loops: bool = True) -> Graph:
    """Small random multigraph (duplicates and self-loops allowed unless asked otherwise) for brute-force checks."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, N, m)
    dst = rng.integers(0, N, m)
    return from_edges(N, src, dst, dedupe=dedupe, drop_self_loops=not self_loops, name="small(%d,%d,%d)" % (N, m, seed))


# ------------------------------------------------------------------ workload recipes

ALPHA_SWEEP = tuple((10 + k) / 20.0 for k in range(11))   # 0.50, 0.55, ..., 1.00, one division each
TAU_DECADES = tuple(float("1e-%d" % k) for k in range(3, 11))  # 1e-3 ... 1e-10, nearest doubles


def tau_sweep_21():
    """1, 5e-1, 1e-1, 5e-2, ..., 1e-10: the tolerance sweep read from the paper's list."""
    out = [1.0]
    for k in range(1, 11):
        out.append(float("5e-%d" % k))
        out.append(float("1e-%d" % k))
    return tuple(out)


def many_graph_specs(count: int = 64, seed: int = 1000):
    """Per-graph draws of the uneven many-graph batch: N log-uniform in [1e3, 1e6], even i R-MAT
    (a,b,c = .57,.19,.19), odd i Erdos-Renyi (no forced dangling), average degree from {4,8,16,32},
    alpha from {.75,.85,.95}, tau from {1e-6,1e-8,1e-10}, norm from {L1,L2,Linf}."""
    specs = []
    for i in range(count):
        h = [hash3(seed + i, 0x4D47, k) for k in range(6)]
        u = (h[0] >> 11) * (1.0 / 9007199254740992.0)
        N = int(round(10 ** (3 + 3 * u)))
        specs.append(dict(
            index=i, N=N, kind="rmat" if i % 2 == 0 else "er", avg_degree=(4, 8, 16, 32)[h[1] % 4],
            alpha=(0.75, 0.85, 0.95)[h[2] % 3], tau=(1e-6, 1e-8, 1e-10)[h[3] % 3], norm=1 + int(h[4] % 3),
            seed=seed + i))
    return specs


def make_spec_graph(spec) -> Graph:
    if spec["kind"] == "rmat":
        return rmat(N=spec["N"], edge_factor=spec["avg_degree"], seed=spec["seed"])
    return er(spec["N"], spec["avg_degree"], 0.0, seed=spec["seed"])


def workload_c1() -> Graph:
    """Erdos-Renyi N=10,000, average out-degree 8, 5% forced dangling, seed 1."""
    return er(10000, 8.0, 0.05, seed=1)
