"""FP64 reference of the learned warm start -- TEST INFRASTRUCTURE.

The warm start is not in the paper; it is a per-vertex multilayer perceptron with two hidden
layers of 32 ReLU units (5 -> 32 -> 32 -> 1) whose output, added to the feature log(N r_0.85),
predicts log(N r_alpha) for a target damping factor alpha.  Everything here is the textbook
definition in float64: dense layers, ReLU, mean squared error, backpropagation by the chain
rule, and Adam (Kingma and Ba, "Adam: a method for stochastic optimization", ICLR 2015,
Algorithm 1).

Packed parameter vector (float32 on the GPU, 1281 values):
  W1[32][5] | b1[32] | W2[32][32] | b2[32] | W3[32] | b3[1]
Features per vertex v (row of 5):
  0: log(1 + in-degree)        1: log(1 + out-degree)
  2: log(N * r085_v)           3: log(N * m_v), m_v = mean of r085 over v's in-edges (1/N if none)
  4: target alpha
"""
from __future__ import annotations

import numpy as np

F, H = 5, 32
SIZES = (("W1", (H, F)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)  # 1281


def unpack(W):
    W = np.asarray(W, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = W[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts):
    return np.concatenate([np.asarray(parts[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def init_params(seed=0):
    """He-uniform initialisation (float64), biases zero."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in SIZES:
        if name.startswith("W"):
            fan_in = shape[-1] if len(shape) == 2 else H
            lim = np.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-lim, lim, size=shape)
        else:
            p[name] = np.zeros(shape)
    p["W3"] *= 0.1
    return pack(p)


def features(N, off, idx, outdeg, r085, alpha_target):
    """[N][5] feature rows (float64), straight from the definitions above."""
    off = np.asarray(off, dtype=np.int64)
    indeg = np.diff(off).astype(np.float64)
    r = np.asarray(r085, dtype=np.float64)
    sums = np.zeros(N)
    for v in range(N):
        s = 0.0
        for j in range(off[v], off[v + 1]):
            s += r[idx[j]]
        sums[v] = s
    mean_in = np.where(indeg > 0, sums / np.maximum(indeg, 1.0), 1.0 / N)
    Fm = np.empty((N, F))
    Fm[:, 0] = np.log1p(indeg)
    Fm[:, 1] = np.log1p(np.asarray(outdeg, dtype=np.float64))
    Fm[:, 2] = np.log(N * r)
    Fm[:, 3] = np.log(N * mean_in)
    Fm[:, 4] = alpha_target
    return Fm


def round_bf16(a):
    """Round to bfloat16 (the upper 16 bits of a float32: 8-bit significand), nearest, ties to
    even, returned as float64.  The value is first held as a float32, the precision in which the
    network's activations are produced before they are stored as bfloat16."""
    a32 = np.asarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def forward(W, X, activations="fp64"):
    """y[N] and the cache for backward.  X is [N][5].  activations="bf16" stores both hidden
    layers rounded to bfloat16, as the warm start's network specifies; "fp64" keeps them exact."""
    p = unpack(W)
    X = np.asarray(X, dtype=np.float64)
    q = round_bf16 if activations == "bf16" else (lambda a: a)
    z1 = X @ p["W1"].T + p["b1"]
    h1 = q(np.maximum(z1, 0.0))
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = q(np.maximum(z2, 0.0))
    y = h2 @ p["W3"] + p["b3"][0]
    return y, dict(X=X, z1=z1, h1=h1, z2=z2, h2=h2)


def backward(W, cache, dy):
    """Gradient of sum_v dy_v * y_v with respect to the packed parameters (float64)."""
    p = unpack(W)
    dy = np.asarray(dy, dtype=np.float64)
    g = {}
    g["W3"] = cache["h2"].T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, p["W3"])
    dz2 = dh2 * (cache["z2"] > 0)
    g["W2"] = dz2.T @ cache["h1"]
    g["b2"] = dz2.sum(axis=0)
    dh1 = dz2 @ p["W2"]
    dz1 = dh1 * (cache["z1"] > 0)
    g["W1"] = dz1.T @ cache["X"]
    g["b1"] = dz1.sum(axis=0)
    return pack(g)


def mse(y, t):
    """Mean squared error and its gradient with respect to y."""
    d = np.asarray(y, dtype=np.float64) - np.asarray(t, dtype=np.float64)
    n = d.shape[0]
    return float(np.dot(d, d) / n), 2.0 * d / n


def adam(W, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1); step counts from 1.  Returns (W, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return W - lr * mhat / (np.sqrt(vhat) + eps), m, v


def start_vector(features_rows, y):
    """Warm start proposed by the network: r_v proportional to exp(log(N r085_v) + y_v), summing to 1."""
    z = np.asarray(features_rows, dtype=np.float64)[:, 2] + np.asarray(y, dtype=np.float64)
    w = np.exp(z - z.max())
    return w / w.sum()
