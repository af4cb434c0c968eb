"""Shared set-up for the GPU parity tests (inputs come from the shared input
generators; expected values from the oracle only)."""
import numpy as np
import pytest

from paper_1605_04718_amd import inputs

THETA_TRUE = (0.1, 0.9, 200.0, 10.0)
TAU = 2.5e-4


def need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_1605_04718_amd import _lib
    _lib.lib()  # raises if the library is not built: no fallback


def make_problem(n, n_steps, *, precision=0, rtol=None, y=None, sigma=0.05, growth=0, rate=0.0,
                 lo=(0.0, 0.0, np.log(50.0), np.log(5.0)), hi=(1.0, 1.0, np.log(500.0), np.log(50.0)),
                 step=(0.02, 0.02, 0.046, 0.046), free_mask=0b1111, max_batch=64, maxit=0,
                 u0=None, v0=None, tau=TAU):
    from paper_1605_04718_amd.api import Grid, Problem
    if u0 is None:
        u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
    if rtol is None:
        rtol = 1e-12 if precision == 1 else 1e-7
    g = Grid(n=n, u0=u0, v0=v0, y=y, sigma=sigma, growth=growth, growth_rate=rate)
    p = Problem([g], tau, n_steps, rtol, precision=precision, cg_maxit=maxit, free_mask=free_mask,
                lo=lo, hi=hi, step=step, max_batch=max_batch)
    return p, u0, v0


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def theta_batch(m, seed=21):
    """Prior draws (sampling box of the 4-parameter configuration) in natural units."""
    phi = inputs.box_draws(m, (0.05, 0.5, np.log(100.0), np.log(8.0)),
                           (0.2, 1.0, np.log(300.0), np.log(15.0)), seed=seed)
    return inputs.to_natural(phi)
