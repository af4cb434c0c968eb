"""FP64 oracle of the surrogate network and its training step.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The surrogate is not part of the paper: it is the first stage of a
delayed-acceptance sampler (Christen and Fox, J. Comput. Graph. Stat. 14(4),
2005) and maps sampling coordinates to a block-averaged u field.

Network: x in R^4 -> depth x [Linear(width) + GELU] -> Linear(out).
GELU(z) = z Phi(z), Phi the standard normal CDF (erf form).
Parameters follow the Linear convention W [out, in], b [out]; the default
initialisation is uniform on +-1/sqrt(fan_in) for weights and biases.
Loss: mean of squared errors over batch and outputs.
Adam (Kingma and Ba, ICLR 2015): beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
bias-corrected moments.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special


def gelu(z):
    return 0.5 * z * (1.0 + special.erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + special.erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2 * math.pi)


def init(sizes, seed=0):
    """sizes = [4, 512, 512, 512, 512, 1024] -> list of (W, b)."""
    rng = np.random.default_rng(seed)
    params = []
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        bound = 1.0 / math.sqrt(fi)
        params.append((rng.uniform(-bound, bound, (fo, fi)), rng.uniform(-bound, bound, fo)))
    return params


def forward(params, x):
    """Returns (y, cache) with cache = list of (input, pre-activation)."""
    h = np.asarray(x, dtype=np.float64)
    cache = []
    for i, (W, b) in enumerate(params):
        z = h @ W.T + b
        cache.append((h, z))
        h = gelu(z) if i < len(params) - 1 else z
    return h, cache


def mse(y, t):
    d = y - t
    return float((d * d).mean()), 2.0 * d / d.size


def backward(params, cache, dy):
    """Gradients [(dW, db)] of the scalar whose gradient w.r.t. y is dy."""
    grads = [None] * len(params)
    g = dy
    for i in range(len(params) - 1, -1, -1):
        h, z = cache[i]
        if i < len(params) - 1:
            g = g * gelu_grad(z)
        W, _ = params[i]
        grads[i] = (g.T @ h, g.sum(axis=0))
        g = g @ W
    return grads


def adam_step(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update; state = dict(t, m, v) (created when empty)."""
    if not state:
        state["t"] = 0
        state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
    state["t"] += 1
    t = state["t"]
    out = []
    for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
        new = []
        for j, (p, g) in enumerate(((W, gW), (b, gb))):
            m = b1 * state["m"][i][j] + (1 - b1) * g
            v = b2 * state["v"][i][j] + (1 - b2) * g * g
            mh = m / (1 - b1 ** t)
            vh = v / (1 - b2 ** t)
            new.append(p - lr * mh / (np.sqrt(vh) + eps))
            state["m"][i] = (m, state["m"][i][1]) if j == 0 else (state["m"][i][0], m)
            state["v"][i] = (v, state["v"][i][1]) if j == 0 else (state["v"][i][0], v)
        out.append(tuple(new))
    return out


def scale_inputs(phi, lo, hi):
    """Sampling coordinates -> [-1, 1] on the prior box."""
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    return 2.0 * (np.asarray(phi, float) - lo) / (hi - lo) - 1.0


def block_mean(u, out_side):
    """Non-overlapping block means of fields [..., n, n] -> [..., out, out]."""
    u = np.asarray(u, dtype=np.float64)
    n = u.shape[-1]
    f = n // out_side
    s = u.reshape(u.shape[:-2] + (out_side, f, out_side, f))
    return s.mean(axis=(-3, -1))


def surrogate_misfit(params, phi, lo, hi, mean, sd, ybar, sigma1):
    """Phi~ = |ybar - (mean + sd * net(x))|^2 / (2 sigma1^2) for each row of phi."""
    y, _ = forward(params, scale_inputs(np.atleast_2d(phi), lo, hi))
    u = mean + sd * y
    return 0.5 * ((ybar.ravel() - u) ** 2).sum(axis=1) / sigma1 ** 2
