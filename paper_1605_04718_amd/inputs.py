"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only draws random numbers and assembles input arrays; it holds
none of the method's arithmetic (no operator, no solver, no likelihood, no
sampler step).  Both sides of every parity test receive the arrays it makes.

Recipes (the paper's own data fields are not available, so these stand in for
them with the shapes and value distributions of its workloads):

* initial fields: the homogeneous steady state (u*, v*) = (a+b, b/(a+b)^2) of
  the kinetics (Sec. 3.1.1, eq. (ic_gturing)) with independent relative
  uniform perturbations of +-rel per cell (Sec. 3.1.2 fixes one known initial
  condition for all proposals);
* one-dimensional example: the printed initial condition of eq. (ic_gturing)
  (no random numbers);
* data: y = u(T; theta_true) + eta, eta ~ N(0, s^2) with s a fraction of the
  range (max - min) of the noise-free field (Sec. 3.1.1, Sec. 3.1.2);
* parameter draws: uniform on a box in sampling coordinates.
"""
from __future__ import annotations

import numpy as np

# Seeds of the input recipes (the method's own random numbers are drawn from
# the counter-based generator on each side).
SEED_IC = 1
SEED_DATA_NOISE = 2
SEED_CHAIN_INIT = 3
SEED_SAMPLER = 4
SEED_SURROGATE_INIT = 5
SEED_DATASET = 6


def homogeneous_state(a: float, b: float) -> tuple[float, float]:
    """(u*, v*) = (a + b, b / (a + b)^2), the IC centre of eq. (ic_gturing)."""
    return a + b, b / (a + b) ** 2


def initial_fields(n: int, a: float, b: float, rel: float = 0.01, seed: int = SEED_IC):
    """u0, v0 [n, n] float64: (u*, v*) times (1 + rel * U[-1, 1]) per cell."""
    rng = np.random.default_rng(seed)
    us, vs = homogeneous_state(a, b)
    xu = rng.uniform(-1.0, 1.0, size=(n, n))
    xv = rng.uniform(-1.0, 1.0, size=(n, n))
    return us * (1.0 + rel * xu), vs * (1.0 + rel * xv)


def initial_fields_1d(n: int):
    """u0, v0 [n] float64 of eq. (ic_gturing) on the cell centres (i + 1/2)/n
    of the unit interval: 1 and 0.9 plus 0.005 sum_{k=1..9} sin(k pi x)
    (the one-dimensional example's fixed initial condition)."""
    x = (np.arange(n) + 0.5) / n
    s = np.zeros(n)
    for k in range(1, 10):
        s += np.sin(k * np.pi * x)
    return 1.0 + 0.005 * s, 0.9 + 0.005 * s


def standard_normal_field(shape, seed: int = SEED_DATA_NOISE) -> np.ndarray:
    return np.random.default_rng(seed).standard_normal(size=shape)


def noisy_data(u_true: np.ndarray, noise_frac: float = 0.01, seed: int = SEED_DATA_NOISE):
    """y = u_true + s * eps with s = noise_frac * (max - min) of u_true."""
    u_true = np.asarray(u_true, dtype=np.float64)
    s = noise_frac * float(u_true.max() - u_true.min())
    y = u_true + s * standard_normal_field(u_true.shape, seed)
    return y, s


def box_draws(m: int, lo, hi, seed: int = SEED_CHAIN_INIT) -> np.ndarray:
    """[m, len(lo)] uniform draws on the box [lo, hi]."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    rng = np.random.default_rng(seed)
    return lo + (hi - lo) * rng.uniform(size=(m, lo.size))


def to_natural(phi: np.ndarray) -> np.ndarray:
    """Sampling coordinates (a, b, ln gamma, ln d) -> (a, b, gamma, d)."""
    phi = np.atleast_2d(np.asarray(phi, dtype=np.float64))
    return np.concatenate([phi[:, :2], np.exp(phi[:, 2:4])], axis=1)


def to_sampling(theta: np.ndarray) -> np.ndarray:
    theta = np.atleast_2d(np.asarray(theta, dtype=np.float64))
    return np.concatenate([theta[:, :2], np.log(theta[:, 2:4])], axis=1)
