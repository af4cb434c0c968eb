"""Pins of the oracle's steady-state stopping (Sec. 3.1.2: step until the
L2 norm of the discrete time derivative is below a threshold), CPU only."""
import math

import numpy as np

import oracle
from test_oracle_pins import cos_mode, imex_mode_matrix, lam1


def test_homogeneous_steady_state_stops_after_one_step():
    theta = (0.1, 0.9, 200.0, 10.0)
    u0, v0 = np.full((8, 8), 1.0), np.full((8, 8), 0.9)
    u, v, steps, _, st = oracle.forward_solve_steady(theta, u0, v0, 2.5e-4, 50, 1e-5)
    assert st == 0 and steps == 1
    assert np.abs(u - 1.0).max() < 1e-12 and np.abs(v - 0.9).max() < 1e-12


def test_norm_closed_form():
    """One cell changed by delta in u: norm = delta / (n tau)."""
    n, tau = 8, 1e-3
    u = np.zeros((n, n))
    u2 = u.copy()
    u2[3, 4] = 2e-6
    assert oracle.time_derivative_norm(u, u, u2, u, tau) == 2e-6 / (n * tau)


def test_stopping_step_of_a_decaying_mode_matches_the_mode_map():
    """A small single-mode perturbation outside the Turing space (d = 1)
    decays (with oscillation: the mode map has complex eigenvalues) as the
    2 x 2 IMEX mode map says; the first step at which the derivative norm
    from that map falls below the threshold is the stopping step."""
    theta, tau, n = (0.1, 0.9, 200.0, 1.0), 2.5e-4, 16
    a, b = theta[:2]
    us, vs = a + b, b / (a + b) ** 2
    k, l, eps = 1, 0, 1e-7
    phi = cos_mode(n, k, l)
    M = imex_mode_matrix(theta, lam1(n, k) + lam1(n, l), tau)
    amp = np.array([1.0, -0.5]) * eps
    scale = math.sqrt(float((phi * phi).sum())) / (n * tau)
    norms = []
    for _ in range(400):
        nxt = M @ amp
        norms.append(float(np.linalg.norm(nxt - amp)) * scale)
        amp = nxt
    tol = 2e-6
    first = next(i for i, x in enumerate(norms) if x < tol)
    assert 20 < first < 390
    # no step before it comes within the nonlinear and rounding error of tol
    assert min(abs(x - tol) for x in norms[:first + 1]) > 1e-4 * tol
    target = first + 1  # steps taken, the last one included
    u0, v0 = us + 1.0 * eps * phi, vs - 0.5 * eps * phi
    _, _, steps, _, st = oracle.forward_solve_steady(theta, u0, v0, tau, 400, tol, rtol=1e-15)
    assert st == 0 and steps == target


def test_cap_without_steady_state_is_flagged():
    theta = (0.1, 0.9, 200.0, 1.0)
    n = 8
    u0 = 1.0 + 1e-3 * cos_mode(n, 1, 0)
    v0 = np.full((n, n), 0.9)
    _, _, steps, _, st = oracle.forward_solve_steady(theta, u0, v0, 2.5e-4, 5, 1e-12)
    assert steps == 5 and st == oracle.ST_NOT_STEADY
