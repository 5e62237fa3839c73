"""Pins of the warm-start references (MLP, features, Adam) in oracle.mlp -- no GPU."""
import numpy as np
import pytest

import graphgen as gg
from oracle import mlp


def test_param_count():
    assert mlp.N_PARAMS == 32 * 5 + 32 + 32 * 32 + 32 + 32 + 1 == 1281


@pytest.mark.parametrize("seed", range(3))
def test_backward_matches_central_differences(seed):
    rng = np.random.default_rng(seed)
    W = mlp.init_params(seed) + rng.normal(0, 0.05, mlp.N_PARAMS)
    X = rng.normal(0, 1, (9, 5))
    t = rng.normal(0, 1, 9)

    def loss(w):
        return mlp.mse(mlp.forward(w, X)[0], t)[0]

    y, cache = mlp.forward(W, X)
    _, dy = mlp.mse(y, t)
    g = mlp.backward(W, cache, dy)
    h = 1e-6
    num = np.empty_like(W)
    for i in range(W.size):
        e = np.zeros_like(W)
        e[i] = h
        num[i] = (loss(W + e) - loss(W - e)) / (2 * h)
    scale = np.abs(num).max()
    assert np.abs(g - num).max() <= 1e-6 * scale


def test_forward_hand_weights():
    # W1 copies the 5 inputs into units 0..4, W2 = identity, W3 = ones: y = sum relu(x) + b3
    p = {k: np.zeros(s) for k, s in mlp.SIZES}
    p["W1"][np.arange(5), np.arange(5)] = 1.0
    p["W2"] = np.eye(32)
    p["W3"] = np.ones(32)
    p["b3"] = np.array([0.25])
    W = mlp.pack(p)
    X = np.array([[1.0, -2.0, 3.0, -4.0, 0.5], [-1.0, -1.0, -1.0, -1.0, -1.0]])
    y, _ = mlp.forward(W, X)
    np.testing.assert_allclose(y, [1 + 3 + 0.5 + 0.25, 0.25])


def test_adam_first_step_closed_form():
    # with zero moments, the bias-corrected first step is lr * g / (|g| + eps)
    rng = np.random.default_rng(1)
    W = rng.normal(size=50)
    g = rng.normal(size=50)
    W1, m, v = mlp.adam(W, g, np.zeros(50), np.zeros(50), step=1, lr=1e-2, eps=1e-8)
    np.testing.assert_allclose(W1, W - 1e-2 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)


def test_adam_constant_gradient_moves_lr_per_step():
    # a constant gradient keeps mhat = g and vhat = g^2 at every step
    W = np.zeros(4)
    g = np.array([1.0, -2.0, 0.5, 3.0])
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 6):
        W, m, v = mlp.adam(W, g, m, v, step=t, lr=0.1, eps=0.0)
    np.testing.assert_allclose(W, -0.5 * np.sign(g), rtol=1e-12)


def test_features_in_star_by_hand():
    g = gg.in_star(3)  # hub 0 <- leaves 1,2,3
    r = np.array([0.4, 0.1, 0.2, 0.3])
    Fm = mlp.features(g.N, g.off, g.idx, g.outdeg, r, 0.95)
    N = 4
    np.testing.assert_allclose(Fm[:, 0], np.log([4, 1, 1, 1]))
    np.testing.assert_allclose(Fm[:, 1], np.log([1, 2, 2, 2]))
    np.testing.assert_allclose(Fm[:, 2], np.log(N * r))
    np.testing.assert_allclose(Fm[:, 3], [np.log(N * 0.2), 0, 0, 0], atol=1e-15)
    np.testing.assert_allclose(Fm[:, 4], 0.95)


def test_start_vector_zero_output_is_r085():
    r = np.array([0.1, 0.2, 0.3, 0.4])
    Fm = np.zeros((4, 5))
    Fm[:, 2] = np.log(4 * r)
    np.testing.assert_allclose(mlp.start_vector(Fm, np.zeros(4)), r, rtol=1e-14)


def test_bf16_rounding_from_the_format():
    # bfloat16 keeps 8 significand bits: between 1 and 2 the spacing is 2^-7
    cases = [(1.0, 1.0), (1.0 + 2.0 ** -8, 1.0),                       # halfway, ties to the even 1.0
             (1.0 + 3 * 2.0 ** -8, 1.0 + 2.0 ** -6),                     # halfway, ties to the even 1+2^-6
             (1.0 + 2.0 ** -8 + 2.0 ** -20, 1.0 + 2.0 ** -7),            # just above halfway: up
             (1.0 + 2.0 ** -8 - 2.0 ** -20, 1.0),                         # just below halfway: down
             (-3.0, -3.0), (0.0, 0.0), (2.0 ** 100, 2.0 ** 100),
             (1.0 / 3.0, 171.0 / 512.0)]      # 1.0101010|1010..b x 2^-2: the dropped bits exceed half -> up
    got = mlp.round_bf16(np.array([c[0] for c in cases]))
    np.testing.assert_array_equal(got, [c[1] for c in cases])


def test_bf16_forward_stays_close_to_exact():
    W = mlp.init_params(5)
    X = np.random.default_rng(5).normal(size=(200, 5))
    y, c = mlp.forward(W, X)
    yb, cb = mlp.forward(W, X, activations="bf16")
    # every stored activation is a bfloat16 value, within half a bfloat16 ulp of its own float32 input
    for h in (cb["h1"], cb["h2"]):
        np.testing.assert_array_equal(h, mlp.round_bf16(h))
    np.testing.assert_allclose(cb["h1"], c["h1"], rtol=2.0 ** -8, atol=0)
    assert np.max(np.abs(yb - y)) <= 2.0 ** -7 * (np.abs(y).max() + 1.0)
