"""Pins of the FP64 surrogate oracle: finite differences, closed forms."""
import math

import numpy as np
import pytest

from oracle import mlp


def test_gelu_closed_forms():
    assert mlp.gelu(0.0) == 0.0
    # GELU(1) = Phi(1), the standard normal CDF at 1
    assert mlp.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-14)
    assert mlp.gelu(-1.0) == pytest.approx(-(1 - 0.8413447460685429), rel=1e-13)
    assert mlp.gelu(12.0) == pytest.approx(12.0, rel=1e-15)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (mlp.gelu(z + h) - mlp.gelu(z - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(z), fd, rtol=1e-8, atol=1e-9)


def test_backprop_matches_central_differences():
    rng = np.random.default_rng(0)
    params = mlp.init([4, 8, 8, 6], seed=1)
    x = rng.uniform(-1, 1, (5, 4))
    t = rng.standard_normal((5, 6))

    def loss(ps):
        y, _ = mlp.forward(ps, x)
        return mlp.mse(y, t)[0]

    y, cache = mlp.forward(params, x)
    _, dy = mlp.mse(y, t)
    grads = mlp.backward(params, cache, dy)
    h = 1e-6
    for li, (W, b) in enumerate(params):
        for arr_i, arr in enumerate((W, b)):
            g = grads[li][arr_i]
            for idx in [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]:
                plus = [(Wj.copy(), bj.copy()) for Wj, bj in params]
                minus = [(Wj.copy(), bj.copy()) for Wj, bj in params]
                plus[li][arr_i][idx] += h
                minus[li][arr_i][idx] -= h
                fd = (loss(plus) - loss(minus)) / (2 * h)
                assert g[idx] == pytest.approx(fd, rel=1e-6, abs=1e-10)


def test_mse_gradient_and_value():
    y = np.array([[1.0, 2.0], [3.0, 5.0]])
    t = np.array([[0.0, 2.0], [3.0, 1.0]])
    l, dy = mlp.mse(y, t)
    assert l == pytest.approx((1 + 0 + 0 + 16) / 4)
    assert np.allclose(dy, 2 * (y - t) / 4)


def test_adam_first_step_is_signed_learning_rate():
    params = [(np.array([[1.0, -2.0]]), np.array([0.5]))]
    grads = [(np.array([[0.3, -4.0]]), np.array([1e-3]))]
    st = {}
    new = mlp.adam_step(params, grads, st, lr=1e-2)
    # first bias-corrected step: m_hat = g, v_hat = g^2 -> lr * g / (|g| + eps)
    assert np.allclose(new[0][0], [[1.0 - 1e-2, -2.0 + 1e-2]], atol=1e-9)
    assert new[0][1][0] == pytest.approx(0.5 - 1e-2 * 1e-3 / (1e-3 + 1e-8), rel=1e-12)
    assert st["t"] == 1


def test_block_mean_and_init_bounds():
    u = np.arange(16.0).reshape(4, 4)
    bm = mlp.block_mean(u, 2)
    assert np.allclose(bm, [[2.5, 4.5], [10.5, 12.5]])
    ps = mlp.init([4, 512, 1024], seed=3)
    assert np.abs(ps[0][0]).max() <= 0.5 and np.abs(ps[1][0]).max() <= 1 / math.sqrt(512)
    assert abs(ps[1][0].std() - 1 / math.sqrt(3 * 512)) < 0.02 / math.sqrt(512)
