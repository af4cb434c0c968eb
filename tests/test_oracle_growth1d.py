"""Pins of the 1-D growing-domain oracle (Sec. 3.1.2, Example 1), CPU only."""
import math

import numpy as np
import pytest

from oracle import growth1d as g1


def test_growth_polynomial_meets_its_end_conditions():
    T, rho_T = 600.0, 1.8
    beta = (0.3, -0.2, 0.5)
    assert g1.rho_poly(beta, rho_T, T, 0.0)[0] == 1.0
    assert g1.rho_poly(beta, rho_T, T, T)[0] == pytest.approx(rho_T, abs=1e-14)
    for t in (10.0, 250.0, 590.0):
        h = 1e-3
        num = (g1.rho_poly(beta, rho_T, T, t + h)[0] - g1.rho_poly(beta, rho_T, T, t - h)[0]) / (2 * h)
        assert g1.rho_poly(beta, rho_T, T, t)[1] == pytest.approx(num, rel=1e-8)


def test_data_growth_laws():
    """Both laws start at 1 and end at (nearly) the same size at T = 600, as
    the text states for the reading with exp(0.6); as printed, exp(0.006)
    would end the logistic law at 1.006."""
    assert g1.rho_exp(0.0) == 1.0 and g1.rho_log(0.0) == 1.0
    assert abs(g1.rho_log(600.0) / g1.rho_exp(600.0) - 1.0) < 3e-3
    e6 = math.exp(6.0)
    assert abs(e6 / (1 + (e6 - 1) / math.exp(0.006)) - 1.006) < 1e-3
    for fn in (g1.rho_exp_pair, g1.rho_log_pair):
        for t in (5.0, 300.0):
            h = 1e-3
            num = (fn(t + h)[0] - fn(t - h)[0]) / (2 * h)
            assert fn(t)[1] == pytest.approx(num, rel=1e-7)


def test_uniform_fields_follow_the_scalar_recursion():
    """Constant fields have zero Laplacian: each step is the scalar IMEX
    update with the dilution term rho'/rho (checks reaction and dilution)."""
    theta = (0.1, 0.9, 1000.0, 10.0)
    a, b, g, d = theta
    n, tau, steps, T, rho_T = 20, 1e-4, 50, 600.0, 1.8
    beta = (0.4, 0.1, 0.2)
    u, v = np.full(n, 1.02), np.full(n, 0.88)
    us, vs = 1.02, 0.88
    for s in range(steps):
        rho, drho = g1.rho_poly(beta, rho_T, T, s * tau)
        u, v = g1.imex_step(theta, u, v, tau, rho, drho)
        dil = drho / rho
        us, vs = ((us / tau + g * a) / (1 / tau + dil + g * (1 - us * vs)),
                  (vs / tau + g * b) / (1 / tau + dil + g * us * us))
    assert np.abs(u - us).max() < 1e-13 and np.abs(v - vs).max() < 1e-13


def test_pure_diffusion_mode_on_a_growing_domain():
    """gamma = 0: a cosine mode k of amplitude A evolves as
    A' = (A / tau) / (1/tau + rho'/rho + lam / rho^2), lam = 4 n^2 sin^2(k pi / 2n)
    (checks the 3-point stencil, the mirror boundary and the rho^-2 scale)."""
    theta = (0.0, 0.0, 0.0, 3.0)
    n, tau, steps, T, rho_T = 32, 1e-3, 40, 1.0, 1.5
    beta = (0.2, 0.1, 0.05)
    x = (np.arange(n) + 0.5) / n
    k = 3
    phi = np.cos(k * math.pi * x)
    lam = 4.0 * n * n * math.sin(k * math.pi / (2 * n)) ** 2
    u, v = 0.3 * phi, -0.2 * phi
    Au, Av = 0.3, -0.2
    for s in range(steps):
        rho, drho = g1.rho_poly(beta, rho_T, T, s * tau)
        u, v = g1.imex_step(theta, u, v, tau, rho, drho)
        Au = (Au / tau) / (1 / tau + drho / rho + lam / rho ** 2)
        Av = (Av / tau) / (1 / tau + drho / rho + 3.0 * lam / rho ** 2)
    assert np.abs(u - Au * phi).max() < 1e-13 and np.abs(v - Av * phi).max() < 1e-13


def test_initial_fields_printed_form():
    u0, v0 = g1.initial_fields(100)
    x = (np.arange(100) + 0.5) / 100
    assert u0[37] == pytest.approx(1 + 0.005 * sum(math.sin(k * math.pi * x[37]) for k in range(1, 10)))
    assert np.allclose(v0 - u0, -0.1)


def test_non_positive_growth_is_outside_the_support():
    """beta = (-5, 0, 0) with rho(T) = 1.8: rho(T/2) = 1 - 2.5 + 5.8/16 < 0."""
    assert g1.rho_poly((-5.0, 0.0, 0.0), 1.8, 1.0, 0.5)[0] < 0
    assert not g1.growth_positive((-5.0, 0.0, 0.0), 1.8, 0.01, 100)
    assert g1.growth_positive((0.8, 0.0, 0.0), 1.8, 0.01, 100)
    n = 8
    u0, v0 = g1.initial_fields(n)
    y = np.stack([u0, v0])
    assert g1.loglik_beta((0.1, 0.9, 1000.0, 10.0), (-5.0, 0.0, 0.0), 1.8, u0, v0, 0.01, 100,
                          y, 0.1) == math.inf


def test_loglik_zero_steps_is_the_misfit_of_the_initial_fields():
    n = 16
    u0, v0 = g1.initial_fields(n)
    y = np.stack([u0 + 0.1, v0 - 0.2])
    th = (0.1, 0.9, 1000.0, 10.0)
    assert g1.loglik_beta(th, (0.1, 0.2, 0.3), 1.8, u0, v0, 1e-4, 0, y, 0.5, obs=1) == \
        pytest.approx(0.5 * n * 0.01 / 0.25, rel=1e-14)
    assert g1.loglik_beta(th, (0.1, 0.2, 0.3), 1.8, u0, v0, 1e-4, 0, y, 0.5, obs=3) == \
        pytest.approx(0.5 * n * 0.05 / 0.25, rel=1e-14)


def test_total_mass_follows_the_dilution_law_without_reactions():
    """gamma = 0: the mirror-boundary Laplacian sums to zero over the cells,
    so summing the step gives sum(u') (1/tau + rho'/rho) = sum(u)/tau exactly
    for any field (a wrong boundary row, a dropped or flipped dilution term
    breaks it); likewise for v."""
    theta = (0.3, 0.2, 0.0, 7.0)
    n, tau, steps, T, rho_T = 45, 2e-3, 30, 0.06, 2.2
    beta = (1.5, -0.4, 0.3)
    rng = np.random.default_rng(4)
    u, v = rng.uniform(0.5, 1.5, n), rng.uniform(0.2, 0.8, n)
    mu, mv = u.sum(), v.sum()
    m0 = mu
    for s in range(steps):
        rho, drho = g1.rho_poly(beta, rho_T, T, s * tau)
        u, v = g1.imex_step(theta, u, v, tau, rho, drho)
        mu /= 1.0 + tau * drho / rho
        mv /= 1.0 + tau * drho / rho
        assert u.sum() == pytest.approx(mu, rel=1e-12) and v.sum() == pytest.approx(mv, rel=1e-12)
    assert g1.rho_poly(beta, rho_T, T, 0.0)[1] > 0 and mu < 0.5 * m0  # growth dilutes
