"""Learned warm start for new damping factors (not from the paper).

A per-vertex perceptron (5 -> 32 -> 32 -> 1, ReLU, float32 weights, bfloat16 activations) trained
on ranks the solver itself produces proposes the start vector of a solve at a new alpha from the
alpha = 0.85 ranks.  The power iteration then corrects it; a judge runs the candidate starts
(network, alpha = 0.85 ranks, uniform) as columns of one batched solve for a few updates and
keeps the column whose last change, in the norm the solve stops on, is smallest; the solve
continues from that column's iterate, so the judging updates are not lost and the uniform start
of the paper's method remains the fallback.  A look-ahead of a few updates rather than one:
the network's errors are local and die out within two or three updates, while the alpha = 0.85
ranks differ from the target along slowly contracting directions, so a one-update comparison
tends to prefer the latter even where it needs more updates in total.  Every numerical step runs in libprpull.so (pr_features, pr_mlp_forward,
pr_mlp_backward, pr_adam_step, pr_warm_start_vector, pr_pull_batch); this module only sequences
the calls and owns the tensors.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np
import torch

from . import _lib
from . import Context, DeviceGraph, PR_FP64, PR_L1, pull_batch

N_FEATURES = 5
HIDDEN = 32


def init_params(seed: int = 0, device="cuda") -> torch.Tensor:
    """He-uniform weights, zero biases; the last layer scaled down so the first proposal is near r_0.85."""
    rng = np.random.default_rng(seed)
    parts = []
    for fan_in, rows, scale in ((N_FEATURES, HIDDEN, 1.0), (None, HIDDEN, 0.0), (HIDDEN, HIDDEN, 1.0),
                                (None, HIDDEN, 0.0), (HIDDEN, 1, 0.1), (None, 1, 0.0)):
        if fan_in is None:
            parts.append(np.zeros(rows))
        else:
            lim = np.sqrt(6.0 / fan_in)
            parts.append(scale * rng.uniform(-lim, lim, size=rows * fan_in))
    W = np.concatenate(parts).astype(np.float32)
    assert W.size == _lib.load().pr_mlp_param_count()
    return torch.from_numpy(W).to(device)


def features(ctx: Context, g: DeviceGraph, r085: torch.Tensor, alpha: float, r_target: torch.Tensor | None = None):
    """pr_features: [N][5] float32 features (and the training target log(r_alpha / r_0.85))."""
    if g.prep is None:
        g.prepare(ctx)
    feat = torch.empty((g.N, N_FEATURES), dtype=torch.float32, device=g.off.device)
    target = torch.empty(g.N, dtype=torch.float32, device=g.off.device) if r_target is not None else None
    _lib.check("pr_features", ctx.lib.pr_features(
        ctx.handle, ctx.stream, g.off.data_ptr(), _lib.ptr(g.idx) if g.E else None, g.outdeg.data_ptr(), g.N, g.E,
        g.prep.data_ptr(), r085.data_ptr(), float(alpha), feat.data_ptr(), _lib.ptr(r_target), _lib.ptr(target)))
    return feat, target


def forward(ctx: Context, W: torch.Tensor, feat: torch.Tensor, keep_activations: bool = False):
    n = feat.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=feat.device)
    act = torch.empty((n, 2 * HIDDEN), dtype=torch.int16, device=feat.device) if keep_activations else None
    _lib.check("pr_mlp_forward", ctx.lib.pr_mlp_forward(ctx.handle, ctx.stream, W.data_ptr(), feat.data_ptr(), n,
                                                        y.data_ptr(), _lib.ptr(act)))
    return y, act


def backward(ctx: Context, W, feat, act, y, target, workspace=None):
    """Gradient of the mean squared error and the error itself."""
    n = feat.shape[0]
    dW = torch.empty_like(W)
    nbytes = ctx.lib.pr_mlp_backward_workspace_bytes(n)
    if workspace is None or workspace.numel() < nbytes:
        workspace = torch.empty(nbytes, dtype=torch.uint8, device=feat.device)
    loss = ctypes.c_double()
    _lib.check("pr_mlp_backward", ctx.lib.pr_mlp_backward(
        ctx.handle, ctx.stream, W.data_ptr(), feat.data_ptr(), act.data_ptr(), y.data_ptr(), target.data_ptr(), n,
        dW.data_ptr(), workspace.data_ptr(), workspace.numel(), ctypes.byref(loss)))
    return dW, loss.value


def adam_step(ctx: Context, W, dW, m, v, step: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    _lib.check("pr_adam_step", ctx.lib.pr_adam_step(ctx.handle, ctx.stream, W.data_ptr(), dW.data_ptr(), m.data_ptr(),
                                                    v.data_ptr(), W.numel(), lr, beta1, beta2, eps, int(step)))


def start_vector(ctx: Context, feat, y) -> torch.Tensor:
    n = feat.shape[0]
    r0 = torch.empty(n, dtype=torch.float64, device=feat.device)
    ws = torch.empty(8192, dtype=torch.uint8, device=feat.device)
    _lib.check("pr_warm_start_vector", ctx.lib.pr_warm_start_vector(ctx.handle, ctx.stream, feat.data_ptr(),
                                                                    y.data_ptr(), n, r0.data_ptr(), ws.data_ptr(),
                                                                    ws.numel()))
    return r0


class WarmStart:
    """The trained network plus the propose / judge steps."""

    def __init__(self, ctx: Context, seed: int = 0):
        self.ctx = ctx
        self.W = init_params(seed)
        self.m = torch.zeros_like(self.W)
        self.v = torch.zeros_like(self.W)
        self.step = 0
        self.history = []

    # ---------------------------------------------------------------- training data
    def make_samples(self, g: DeviceGraph, alphas, tau=1e-12, norm=PR_L1):
        """Label one graph: solve alpha = 0.85 and every training alpha together (FP64), then features/targets."""
        probs = [dict(alpha=0.85, tau=tau, norm=norm, max_iter=500)] + \
                [dict(alpha=a, tau=tau, norm=norm, max_iter=500) for a in alphas]
        res = pull_batch(self.ctx, g, probs, precision=PR_FP64)
        r085 = res[0]["ranks"]
        samples = []
        for a, r in zip(alphas, res[1:]):
            feat, target = features(self.ctx, g, r085, a, r["ranks"])
            samples.append((feat, target))
        return samples

    def train(self, samples, epochs: int = 30, lr: float = 3e-3, seed: int = 0):
        """Adam over whole (graph, alpha) samples, one sample per step, epochs in a seeded order."""
        rng = np.random.default_rng(seed)
        n_max = max(feat.shape[0] for feat, _ in samples)
        ws = torch.empty(self.ctx.lib.pr_mlp_backward_workspace_bytes(n_max), dtype=torch.uint8,
                         device=samples[0][0].device)
        for ep in range(epochs):
            losses = []
            for k in rng.permutation(len(samples)):
                feat, target = samples[k]
                y, act = forward(self.ctx, self.W, feat, keep_activations=True)
                dW, loss = backward(self.ctx, self.W, feat, act, y, target, ws)
                self.step += 1
                adam_step(self.ctx, self.W, dW, self.m, self.v, self.step, lr=lr)
                losses.append(loss)
            self.history.append(float(np.mean(losses)))
        return self.history

    # ---------------------------------------------------------------- inference and judging
    def propose(self, g: DeviceGraph, r085: torch.Tensor, alpha: float) -> torch.Tensor:
        feat, _ = features(self.ctx, g, r085, alpha)
        y, _ = forward(self.ctx, self.W, feat)
        return start_vector(self.ctx, feat, y)

    def judge(self, g: DeviceGraph, alpha: float, candidates, norm: int = PR_L1, steps: int = 3):
        """`steps` float64 updates from every candidate start as columns of one batch; the smallest
        last change in `norm` wins.  Returns (winner, last changes, iterates after `steps`)."""
        probs = [dict(alpha=alpha, tau=0.0, norm=norm, max_iter=steps)] * len(candidates)
        res = pull_batch(self.ctx, g, probs, precision=PR_FP64, inits=list(candidates))
        e = [r["err"][norm - 1] for r in res]
        best = int(np.argmin(e))
        return best, e, [r["ranks"] for r in res]

    def start(self, g: DeviceGraph, r085: torch.Tensor, alpha: float, norm: int = PR_L1, steps: int = 3):
        """Judged start for a solve at alpha stopping on `norm`.  Returns (iterate of the winning
        column after `steps` updates, its name, the candidates' last changes, `steps`, seconds spent
        on features, inference and judging).  A solve continued from the iterate has done `steps`
        updates more than its own count says."""
        t0 = time.perf_counter()
        mlp = self.propose(g, r085, alpha)
        uniform = torch.full((g.N,), 1.0 / g.N, dtype=torch.float64, device=g.off.device)
        best, e, iterates = self.judge(g, alpha, [mlp, r085, uniform], norm, steps)
        torch.cuda.synchronize()
        return iterates[best], ("mlp", "r085", "uniform")[best], e, steps, time.perf_counter() - t0
