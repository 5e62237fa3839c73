"""MI355X (gfx950) pull PageRank: Python front end of libprpull.so.

The solver computes the standard power-iteration pull PageRank of Sahu, Kothapalli and
Banerjee (arXiv 2108.02997, section 2 update and teleport term, section 3 error functions)
in hand-written HIP kernels behind a C ABI (include/prpull.h).  This module only moves
arguments: graphs and vectors are torch tensors on the GPU, the stream is torch's current
stream, and every step of a solve runs in the library.  There is no CPU path: without a GPU
or without the built library every call raises.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field

import torch

from . import _lib
from ._lib import (MAX_COLS, PR_FP32, PR_FP64, PR_L1, PR_L2, PR_LINF, PR_MIXED, PR_NOT_CONVERGED, PR_OK,  # noqa: F401
                   PrError, pr_graph_problem, pr_problem, pr_result)

__all__ = ["Context", "DeviceGraph", "pull", "pull_batch", "pull_multi", "unpermute", "PR_L1", "PR_L2", "PR_LINF",
           "PR_FP64", "PR_MIXED", "PR_FP32", "PrError"]


def _require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("paper_2108_02997_amd needs a ROCm GPU (torch.cuda.is_available() is False)")


class Context:
    """A pr_ctx bound to one device (host-side caches only)."""

    def __init__(self, device: int = 0):
        _require_gpu()
        self.lib = _lib.load()
        self.device = device
        h = ctypes.c_void_p()
        with torch.cuda.device(device):
            _lib.check("pr_create", self.lib.pr_create(ctypes.byref(h), device))
        self.handle = h

    def set_option(self, key: str, value: int):
        _lib.check("pr_set_option", self.lib.pr_set_option(self.handle, key.encode(), int(value)))

    def stats(self, kind: int):
        """(launches, milliseconds) of kernel `kind` timed with HIP events (option "timing")."""
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        _lib.check("pr_get_stats", self.lib.pr_get_stats(self.handle, kind, ctypes.byref(n), ctypes.byref(ms)))
        return n.value, ms.value

    def reset_stats(self):
        _lib.check("pr_reset_stats", self.lib.pr_reset_stats(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.pr_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def stream(self) -> int:
        return _lib.stream_handle(self.device)


@dataclass
class DeviceGraph:
    """In-edge CSR on the device (int32 off[N+1], idx[E], outdeg[N]) plus its tile partition."""

    N: int
    E: int
    off: torch.Tensor
    idx: torch.Tensor
    outdeg: torch.Tensor
    prep: torch.Tensor | None = None
    _ws: dict = field(default_factory=dict)
    seg_pairs: int = 0

    @classmethod
    def from_host(cls, g, device: int = 0):
        dev = torch.device("cuda", device)
        off = torch.from_numpy(g.off).to(dev)
        idx = torch.from_numpy(g.idx if g.E > 0 else g.idx[:0]).to(dev)
        outdeg = torch.from_numpy(g.outdeg).to(dev)
        return cls(g.N, g.E, off, idx, outdeg)

    def prepare(self, ctx: Context):
        """pr_prepare: tile partition of this graph (kept on the object)."""
        nbytes = ctx.lib.pr_prep_bytes(self.N, self.E)
        self.prep = torch.empty(nbytes, dtype=torch.uint8, device=self.off.device)
        _lib.check("pr_prepare", ctx.lib.pr_prepare(ctx.handle, ctx.stream, self.off.data_ptr(), self.N, self.E,
                                                    self.prep.data_ptr(), nbytes))
        return self

    def prepare_segmented(self, ctx: Context, seg_len: int = 1 << 19):
        """pr_segment_count + pr_prepare_segmented: the tile partitions plus the source-segmented
        layout (segments of seg_len source ids), kept on the object; pr_pull then runs its
        updates in two steps (per-segment partial sums, then the merge)."""
        dev = self.off.device
        if self.E == 0:
            return self.prepare(ctx)
        cnt_ws = torch.empty(16384, dtype=torch.uint8, device=dev)
        pairs = ctypes.c_int64()
        _lib.check("pr_segment_count", ctx.lib.pr_segment_count(
            ctx.handle, ctx.stream, self.off.data_ptr(), self.idx.data_ptr(), self.N, self.E, int(seg_len),
            cnt_ws.data_ptr(), cnt_ws.numel(), ctypes.byref(pairs)))
        nbytes = ctx.lib.pr_segment_bytes(ctx.handle, self.N, self.E, int(seg_len), pairs.value)
        if nbytes == 0:
            raise PrError("pr_segment_bytes", _lib.PR_EINVAL, _lib.last_error())
        self.prep = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _lib.check("pr_prepare_segmented", ctx.lib.pr_prepare_segmented(
            ctx.handle, ctx.stream, self.off.data_ptr(), self.idx.data_ptr(), self.N, self.E, int(seg_len),
            pairs.value, self.prep.data_ptr(), nbytes))
        self.seg_pairs = pairs.value
        return self

    def relabelled(self, ctx: Context):
        """pr_relabel: the graph in out-degree order (most cited sources first) and perm, the new id
        of every vertex.  Ranks solved on the returned graph map back with unpermute(ctx, perm, r)."""
        dev = self.off.device
        perm = torch.empty(self.N, dtype=torch.int32, device=dev)
        off = torch.empty(self.N + 1, dtype=torch.int32, device=dev)
        idx = torch.empty(max(self.E, 1), dtype=torch.int32, device=dev)[:self.E]
        outdeg = torch.empty(self.N, dtype=torch.int32, device=dev)
        nbytes = ctx.lib.pr_relabel_workspace_bytes(ctx.handle, self.N, self.E)
        if nbytes == 0:
            raise PrError("pr_relabel_workspace_bytes", _lib.PR_EINVAL, _lib.last_error())
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _lib.check("pr_relabel", ctx.lib.pr_relabel(
            ctx.handle, ctx.stream, self.off.data_ptr(), _lib.ptr(self.idx) if self.E else None,
            self.outdeg.data_ptr(), self.N, self.E, perm.data_ptr(), off.data_ptr(),
            _lib.ptr(idx) if self.E else None, outdeg.data_ptr(), ws.data_ptr(), nbytes))
        return DeviceGraph(self.N, self.E, off, idx, outdeg), perm

    def workspace(self, ctx: Context, precision: int, with_prep: bool, K: int = 0) -> torch.Tensor:
        key = (precision, with_prep, K)
        ws = self._ws.get(key)
        if ws is None:
            if K:
                nbytes = ctx.lib.pr_batch_workspace_bytes(self.N, self.E, K, precision, int(with_prep))
            else:
                nbytes = ctx.lib.pr_workspace_bytes(self.N, self.E, precision, int(with_prep))
            ws = torch.empty(nbytes, dtype=torch.uint8, device=self.off.device)
            self._ws[key] = ws
        return ws

    def autotune(self, ctx: Context) -> dict:
        """pr_autotune: choose the tile windows (written into this graph's prep), the degree-bin
        thresholds and the grids of the single-vector and K-column updates (kept in ctx)."""
        if self.prep is None:
            self.prepare(ctx)
        ranks = torch.empty(self.N, dtype=torch.float64, device=self.off.device)
        nbytes = ctx.lib.pr_tune_workspace_bytes(self.N, self.E, 0)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.off.device)
        out = _lib.pr_tune_result()
        _lib.check("pr_autotune", ctx.lib.pr_autotune(ctx.handle, ctx.stream, self.off.data_ptr(),
                                                      _lib.ptr(self.idx) if self.E else None, self.outdeg.data_ptr(),
                                                      self.N, self.E, self.prep.data_ptr(), ranks.data_ptr(),
                                                      ws.data_ptr(), ws.numel(), ctypes.byref(out)))
        return {n: getattr(out, n) for n, _ in _lib.pr_tune_result._fields_ if n != "pad"}

    def validate(self, ctx: Context) -> None:
        nbytes = 4 * self.N + 512
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.off.device)
        _lib.check("pr_validate_graph", ctx.lib.pr_validate_graph(
            ctx.handle, ctx.stream, self.off.data_ptr(), _lib.ptr(self.idx) if self.E else None,
            self.outdeg.data_ptr(), self.N, self.E, ws.data_ptr(), nbytes))


def pr_pull(ctx: Context, g: DeviceGraph, alpha: float, tau: float, norm: int, max_iter: int, precision: int,
            init: torch.Tensor | None, ranks: torch.Tensor, norm_trace: torch.Tensor | None,
            workspace: torch.Tensor, use_prep: bool = True) -> tuple[int, dict]:
    """The C entry point pr_pull with tensors for device buffers; returns (status, result)."""
    for t, n in ((ranks, g.N), (init, g.N)):
        if t is not None and (t.dtype != torch.float64 or t.numel() != n or not t.is_contiguous() or
                              t.device != g.off.device):
            raise ValueError("rank vectors must be contiguous float64 tensors of N elements on the graph's device")
    if norm_trace is not None and (norm_trace.dtype != torch.float64 or norm_trace.numel() < 3 * max_iter):
        raise ValueError("norm_trace must be float64 with max_iter*3 elements")
    res = pr_result()
    prep = g.prep if use_prep else None
    st = ctx.lib.pr_pull(ctx.handle, ctx.stream, g.off.data_ptr(), _lib.ptr(g.idx) if g.E else None,
                         g.outdeg.data_ptr(), g.N, g.E, _lib.ptr(prep), float(alpha), float(tau), int(norm),
                         int(max_iter), int(precision), _lib.ptr(init), ranks.data_ptr(), _lib.ptr(norm_trace),
                         workspace.data_ptr(), workspace.numel(), ctypes.byref(res))
    _lib.check("pr_pull", st)
    return st, res.as_dict()


def pull_snapshots(ctx: Context, g: DeviceGraph, snaps, alpha: float = 0.85, tau: float = 1e-10,
                   norm: int = PR_L1, max_iter: int = 500, precision: int = PR_FP64,
                   init: torch.Tensor | None = None, trace: bool = False) -> dict:
    """pr_pull_snapshots: one solve that also keeps the ranks at the first update meeting each
    (tau_i, norm_i) of `snaps`; returns pull's dict plus snapshots (S x N float64; rows of
    snapshots not taken are NaN) and snap_iter (0 where the solve stopped first)."""
    if g.prep is None:
        g.prepare(ctx)
    dev = g.off.device
    S = len(snaps)
    if init is not None and (init.dtype != torch.float64 or init.numel() != g.N or not init.is_contiguous()):
        raise ValueError("init must be a contiguous float64 tensor of N elements")
    ranks = torch.empty(g.N, dtype=torch.float64, device=dev)
    out = torch.full((max(S, 1), g.N), float("nan"), dtype=torch.float64, device=dev)
    tr = torch.full((max_iter, 3), float("nan"), dtype=torch.float64, device=dev) if trace else None
    stau = (ctypes.c_double * max(S, 1))(*[float(t) for t, _ in snaps])
    snorm = (ctypes.c_int32 * max(S, 1))(*[int(n) for _, n in snaps])
    siter = (ctypes.c_int32 * max(S, 1))()
    ws = g.workspace(ctx, precision, False)
    res = pr_result()
    st = ctx.lib.pr_pull_snapshots(ctx.handle, ctx.stream, g.off.data_ptr(), _lib.ptr(g.idx) if g.E else None,
                                   g.outdeg.data_ptr(), g.N, g.E, _lib.ptr(g.prep), float(alpha), float(tau),
                                   int(norm), int(max_iter), int(precision), _lib.ptr(init), ranks.data_ptr(),
                                   _lib.ptr(tr), S, stau, snorm, out.data_ptr(), siter, ws.data_ptr(), ws.numel(),
                                   ctypes.byref(res))
    _lib.check("pr_pull_snapshots", st)
    d = res.as_dict()
    d.update(status=st, ranks=ranks, trace=tr[:d["iterations"]] if trace else None, snapshots=out[:S],
             snap_iter=[int(siter[i]) for i in range(S)])
    return d


def unpermute(ctx: Context, perm: torch.Tensor, ranks: torch.Tensor) -> torch.Tensor:
    """pr_unpermute: out[v] = ranks[perm[v]], ranks of a relabelled graph back in the original ids."""
    out = torch.empty_like(ranks)
    _lib.check("pr_unpermute", ctx.lib.pr_unpermute(ctx.handle, ctx.stream, perm.data_ptr(), ranks.numel(),
                                                    ranks.data_ptr(), out.data_ptr()))
    return out


def pull(ctx: Context, g: DeviceGraph, alpha: float = 0.85, tau: float = 1e-6, norm: int = PR_L1,
         max_iter: int = 500, precision: int = PR_FP64, init: torch.Tensor | None = None, trace: bool = False,
         ranks: torch.Tensor | None = None) -> dict:
    """Solve one PageRank problem; returns dict(ranks, iterations, converged, fp32_iters, fp64_iters, err, trace)."""
    if g.prep is None:
        g.prepare(ctx)
    if ranks is None:
        ranks = torch.empty(g.N, dtype=torch.float64, device=g.off.device)
    tr = torch.full((max_iter, 3), float("nan"), dtype=torch.float64, device=g.off.device) if trace else None
    ws = g.workspace(ctx, precision, False)
    st, res = pr_pull(ctx, g, alpha, tau, norm, max_iter, precision, init, ranks, tr, ws)
    res["status"] = st
    res["ranks"] = ranks
    res["trace"] = tr[:res["iterations"]] if trace else None
    return res


def l1_distance(ctx: Context, x: torch.Tensor, y: torch.Tensor) -> float:
    """pr_l1_distance: sum |x - y| of two float64 device vectors, reduced in the library."""
    if x.dtype != torch.float64 or y.dtype != torch.float64 or x.numel() != y.numel():
        raise ValueError("two float64 vectors of equal length are required")
    ws = torch.empty(8200, dtype=torch.uint8, device=x.device)
    out = ctypes.c_double()
    _lib.check("pr_l1_distance", ctx.lib.pr_l1_distance(ctx.handle, ctx.stream, x.data_ptr(), y.data_ptr(),
                                                        x.numel(), ws.data_ptr(), ws.numel(), ctypes.byref(out)))
    return out.value


def pr_pull_batch(ctx: Context, g: DeviceGraph, problems, precision: int, inits, ranks, traces,
                  workspace: torch.Tensor, use_prep: bool = True) -> tuple[int, list]:
    """The C entry point pr_pull_batch (at most 16 problems); returns (status, per-problem results)."""
    K = len(problems)
    if not 1 <= K <= MAX_COLS:
        raise ValueError("pr_pull_batch takes 1..16 problems")
    for t in list(ranks) + [x for x in (inits or []) if x is not None]:
        if t.dtype != torch.float64 or t.numel() != g.N or not t.is_contiguous() or t.device != g.off.device:
            raise ValueError("rank vectors must be contiguous float64 tensors of N elements on the graph's device")
    probs = (pr_problem * K)(*[pr_problem(float(p["alpha"]), float(p["tau"]), int(p["norm"]), int(p["max_iter"]))
                              for p in problems])
    for p, tr in zip(problems, traces or [None] * K):
        if tr is not None and (tr.dtype != torch.float64 or tr.numel() < 3 * int(p["max_iter"])):
            raise ValueError("a norm trace must be float64 with max_iter*3 elements")
    vp = ctypes.c_void_p
    init_arr = (vp * K)(*[_lib.ptr(x) for x in inits]) if inits is not None else None
    rank_arr = (vp * K)(*[r.data_ptr() for r in ranks])
    trace_arr = (vp * K)(*[_lib.ptr(x) for x in traces]) if traces is not None else None
    res = (pr_result * K)()
    prep = g.prep if use_prep else None
    st = ctx.lib.pr_pull_batch(ctx.handle, ctx.stream, g.off.data_ptr(), _lib.ptr(g.idx) if g.E else None,
                               g.outdeg.data_ptr(), g.N, g.E, _lib.ptr(prep), K, probs, int(precision), init_arr,
                               rank_arr, trace_arr, workspace.data_ptr(), workspace.numel(), res)
    _lib.check("pr_pull_batch", st)
    return st, [r.as_dict() for r in res]


def pull_batch(ctx: Context, g: DeviceGraph, problems, precision: int = PR_FP64, inits=None, trace: bool = False,
               ranks=None) -> list:
    """Solve several problems on one graph together (groups of up to 16 columns per pass).

    problems: list of dicts with alpha, tau, norm, max_iter.  Returns one dict per problem with
    ranks (tensor), iterations, converged, fp32_iters, fp64_iters, err and trace."""
    if g.prep is None:
        g.prepare(ctx)
    n = len(problems)
    if ranks is None:
        ranks = [torch.empty(g.N, dtype=torch.float64, device=g.off.device) for _ in range(n)]
    traces = ([torch.full((int(p["max_iter"]), 3), float("nan"), dtype=torch.float64, device=g.off.device)
               for p in problems] if trace else None)
    out = []
    for s0 in range(0, n, MAX_COLS):
        sl = slice(s0, min(n, s0 + MAX_COLS))
        K = sl.stop - sl.start
        ws = g.workspace(ctx, precision, False, K)
        st, res = pr_pull_batch(ctx, g, problems[sl], precision, inits[sl] if inits is not None else None,
                                ranks[sl], traces[sl] if traces is not None else None, ws)
        for j, r in enumerate(res):
            r["status"] = st
            r["ranks"] = ranks[sl.start + j]
            r["trace"] = traces[sl.start + j][:r["iterations"]] if trace else None
            out.append(r)
    return out


MAX_SWEEP = 64


def pull_sweep(ctx: Context, g: DeviceGraph, problems, trace: bool = False, ranks=None) -> list:
    """pr_pull_sweep: problems that differ only in alpha / tau / norm / max_iter, all from the
    uniform start, solved in float64 by one iteration (the sweep as a power series in the damping
    factor).  Returns one dict per problem like pull_batch."""
    if g.prep is None:
        g.prepare(ctx)
    K = len(problems)
    if not 1 <= K <= MAX_SWEEP:
        raise ValueError("pr_pull_sweep takes 1..64 problems")
    dev = g.off.device
    if ranks is None:
        ranks = [torch.empty(g.N, dtype=torch.float64, device=dev) for _ in range(K)]
    for r in ranks:
        if r.dtype != torch.float64 or r.numel() != g.N or not r.is_contiguous() or r.device != dev:
            raise ValueError("rank vectors must be contiguous float64 tensors of N elements on the graph's device")
    traces = ([torch.full((int(p["max_iter"]), 3), float("nan"), dtype=torch.float64, device=dev)
               for p in problems] if trace else None)
    probs = (pr_problem * K)(*[pr_problem(float(p["alpha"]), float(p["tau"]), int(p["norm"]), int(p["max_iter"]))
                              for p in problems])
    vp = ctypes.c_void_p
    rank_arr = (vp * K)(*[r.data_ptr() for r in ranks])
    trace_arr = (vp * K)(*[t.data_ptr() for t in traces]) if trace else None
    key = ("sweep",)
    ws = g._ws.get(key)
    if ws is None:
        nbytes = ctx.lib.pr_sweep_workspace_bytes(g.N, g.E, 0)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        g._ws[key] = ws
    res = (pr_result * K)()
    st = ctx.lib.pr_pull_sweep(ctx.handle, ctx.stream, g.off.data_ptr(), _lib.ptr(g.idx) if g.E else None,
                               g.outdeg.data_ptr(), g.N, g.E, g.prep.data_ptr(), K, probs, rank_arr, trace_arr,
                               ws.data_ptr(), ws.numel(), res)
    _lib.check("pr_pull_sweep", st)
    out = []
    for k, r in enumerate(res):
        d = r.as_dict()
        d["status"] = st
        d["ranks"] = ranks[k]
        d["trace"] = traces[k][:d["iterations"]] if trace else None
        out.append(d)
    return out


def multi_problems(ctx: Context, graphs, problems, inits=None, trace: bool = False, ranks=None):
    """The pr_graph_problem array of a many-graph call, with the given (or fresh) rank tensors and
    fresh trace tensors."""
    G = len(graphs)
    if G != len(problems) or G < 1:
        raise ValueError("one problem per graph is required")
    if ranks is not None and (len(ranks) != G or any(r.dtype != torch.float64 or r.numel() != g.N or
                                                     not r.is_contiguous() for r, g in zip(ranks, graphs))):
        raise ValueError("one contiguous float64 rank tensor of N elements per graph is required")
    given = ranks
    arr = (pr_graph_problem * G)()
    ranks, traces = [], []
    for k, (g, p) in enumerate(zip(graphs, problems)):
        if g.prep is None:
            g.prepare(ctx)
        r = given[k] if given is not None else torch.empty(g.N, dtype=torch.float64, device=g.off.device)
        tr = torch.full((int(p["max_iter"]), 3), float("nan"), dtype=torch.float64, device=g.off.device) if trace \
            else None
        ini = inits[k] if inits is not None else None
        arr[k] = pr_graph_problem(g.off.data_ptr(), _lib.ptr(g.idx) if g.E else None, g.outdeg.data_ptr(), g.N, g.E,
                                  g.prep.data_ptr(), float(p["alpha"]), float(p["tau"]), int(p["norm"]),
                                  int(p["max_iter"]), _lib.ptr(ini), r.data_ptr(), _lib.ptr(tr))
        ranks.append(r)
        traces.append(tr)
    return arr, ranks, traces


def pull_multi(ctx: Context, graphs, problems, inits=None, trace: bool = False, workspace=None, ranks=None) -> list:
    """Many graphs, each with its own problem, in one persistent launch (pr_pull_multi, float64).

    graphs: DeviceGraph list (prepared here if needed); problems: dicts with alpha, tau, norm,
    max_iter; ranks: optional output tensors (one per graph).  Returns one dict per graph (ranks,
    iterations, converged, err, trace)."""
    G = len(graphs)
    arr, ranks, traces = multi_problems(ctx, graphs, problems, inits, trace, ranks)
    nbytes = ctx.lib.pr_multi_workspace_bytes(G, arr)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=graphs[0].off.device)
    res = (pr_result * G)()
    st = ctx.lib.pr_pull_multi(ctx.handle, ctx.stream, G, arr, workspace.data_ptr(), workspace.numel(), res)
    _lib.check("pr_pull_multi", st)
    out = []
    for k in range(G):
        d = res[k].as_dict()
        d["status"] = st
        d["ranks"] = ranks[k]
        d["trace"] = traces[k][:d["iterations"]] if trace else None
        out.append(d)
    return out
