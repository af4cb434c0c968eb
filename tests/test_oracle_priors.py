"""Pins of the oracle's priors beyond the uniform box (Sec. 3.1.2, Cases 2-4):
the Turing-space support of eq. (turing) and the log-normal prior, and the
sampler's invariance for each (CPU only)."""
import math

import numpy as np
import pytest

from oracle import sampler as osamp
from paper_1605_04718_amd import inputs


def _kinetics_jacobian(a, b, h=1e-6):
    """f = a - u + u^2 v, g = b - u^2 v differentiated numerically at the
    homogeneous steady state: independent of the printed entries."""
    us, vs = a + b, b / (a + b) ** 2

    def f(u, v):
        return a - u + u * u * v

    def g(u, v):
        return b - u * u * v

    fu = (f(us + h, vs) - f(us - h, vs)) / (2 * h)
    fv = (f(us, vs + h) - f(us, vs - h)) / (2 * h)
    gu = (g(us + h, vs) - g(us - h, vs)) / (2 * h)
    gv = (g(us, vs + h) - g(us, vs - h)) / (2 * h)
    return fu, fv, gu, gv


def _turing_from_jacobian(a, b, d):
    fu, fv, gu, gv = _kinetics_jacobian(a, b)
    det = fu * gv - fv * gu
    return (fu + gv < 0, det > 0, d * fu + gv > 0, (d * fu + gv) ** 2 - 4 * d * det > 0)


def test_turing_space_golden_rows():
    """a = 0.1, b = 0.9: inside at d = 10, outside at d = 1 (d f_u + g_v < 0)."""
    assert osamp.turing_space(0.1, 0.9, 10.0)
    assert not osamp.turing_space(0.1, 0.9, 1.0)


def test_turing_space_matches_the_kinetics_jacobian():
    """Membership agrees with the conditions built from a numerical Jacobian
    of the kinetics on random points away from the boundary."""
    rng = np.random.default_rng(7)
    checked = inside = 0
    for _ in range(4000):
        a, b = rng.uniform(0.0, 1.5, 2)
        d = math.exp(rng.uniform(0.0, math.log(100.0)))
        conds = _turing_from_jacobian(a, b, d)
        s = a + b
        margins = [abs((b - a) / s - s * s), s * s, abs(d * (b - a) / s - s * s),
                   abs((d * (b - a) / s - s * s) ** 2 - 4 * d * s * s)]
        if min(margins) < 1e-4:
            continue  # too close to a boundary for the numerical Jacobian
        checked += 1
        assert osamp.turing_space(a, b, d) == all(conds), (a, b, d)
        inside += all(conds)
    assert checked > 3000 and 0 < inside < checked


def test_case1_credible_region_lies_in_the_turing_space():
    """Sec. 3.1.2, Case 1: the 95 % region [0.126, 0.128] x [0.789, 0.796]
    lies inside the Turing space (d = 10); so does Table 1's (a, b)."""
    for a in np.linspace(0.126, 0.128, 5):
        for b in np.linspace(0.789, 0.796, 5):
            assert osamp.turing_space(a, b, 10.0)
    assert osamp.turing_space(0.126779, 0.792366, 10.0)


def test_prior_quad_closed_form():
    pr = osamp.Prior(kinds=(0, 0, 1, 1), mean=(0, 0, math.log(500.0), math.log(5.0)),
                     sd=(1, 1, 0.95, 0.95))
    phi = np.array([0.3, 0.7, math.log(500.0), math.log(5.0)])
    assert osamp.prior_quad(phi, pr) == 0.0
    phi2 = phi + np.array([5.0, -3.0, 0.95, -2 * 0.95])
    assert osamp.prior_quad(phi2, pr) == pytest.approx(0.5 * 1 + 0.5 * 4, rel=1e-14)
    assert osamp.log_prior_ratio(phi, phi2, pr) == pytest.approx(-2.5, rel=1e-14)
    assert osamp.log_prior_ratio(phi, phi2, None) == 0.0


def test_support_box_ignores_normal_coordinates():
    pr = osamp.Prior(kinds=(0, 0, 1, 1), mean=(0, 0, 6.0, 1.5), sd=(1, 1, 0.95, 0.95))
    lo, hi = (0.0, 0.0, 5.0, 1.0), (1.0, 1.0, 6.0, 2.0)
    assert osamp.in_support([0.5, 0.5, 9.0, -3.0], lo, hi, pr)
    assert not osamp.in_support([0.5, 0.5, 9.0, -3.0], lo, hi, None)
    assert not osamp.in_support([1.5, 0.5, 6.0, 1.5], lo, hi, pr)


def test_normal_prior_is_invariant_under_the_sampler():
    """With Phi = 0 the posterior is the prior: chains started from exact
    prior draws keep mean and s.d. of the log-normal coordinates (a sign
    error in the prior ratio moves the mean, a lost factor 1/2 shrinks the
    s.d. by sqrt 2)."""
    C, S = 1500, 40
    mu = (0.0, 0.0, math.log(500.0), math.log(5.0))
    sd = (1.0, 1.0, 0.95, 0.95)
    pr = osamp.Prior(kinds=(0, 0, 1, 1), mean=mu, sd=sd)
    rng = np.random.default_rng(11)
    phis = np.zeros((C, 4))
    phis[:, 0], phis[:, 1] = 0.3, 0.6
    phis[:, 2] = rng.normal(mu[2], sd[2], C)
    phis[:, 3] = rng.normal(mu[3], sd[3], C)
    lls = np.zeros(C)
    lo, hi = (0.0, 0.0, -50.0, -50.0), (1.0, 1.0, 50.0, 50.0)
    step = (0.0, 0.0, 1.2, 1.2)
    acc = 0
    for s in range(S):
        phis, lls, a, _ = osamp.rwm_batch_step(phis, lls, 21, s, lo, hi, step, 0b1100,
                                               lambda q: np.zeros(len(q)), prior=pr)
        acc += a.sum()
    assert 0.2 < acc / (C * S) < 0.8
    for i in (2, 3):
        m, s = phis[:, i].mean(), phis[:, i].std()
        assert abs(m - mu[i]) < 4 * sd[i] / math.sqrt(C), (i, m)
        assert abs(s - sd[i]) < 4 * sd[i] / math.sqrt(2 * C), (i, s)


def test_turing_prior_is_uniform_on_the_turing_space():
    """With Phi = 0 and the Turing support (d = 10 fixed), chains started
    uniformly on box and Turing space stay there and stay uniform: the mean
    of a matches the region's centroid from a fine grid."""
    d = 10.0
    lo, hi = (0.0, 0.4, math.log(200.0), math.log(d)), (0.25, 1.1, math.log(200.0), math.log(d))
    pr = osamp.Prior(turing=True)
    xa = np.linspace(lo[0], hi[0], 801)[:-1] + (hi[0] - lo[0]) / 1600
    xb = np.linspace(lo[1], hi[1], 801)[:-1] + (hi[1] - lo[1]) / 1600
    A, B = np.meshgrid(xa, xb, indexing="ij")
    s = A + B
    dfg = d * (B - A) / s - s * s
    mask = ((B - A) / s - s * s < 0) & (dfg > 0) & (dfg * dfg - 4 * d * s * s > 0)
    ca, cb = A[mask].mean(), B[mask].mean()
    rng = np.random.default_rng(5)
    C, S = 1500, 40
    start = []
    for _ in range(200 * C):
        a, b = rng.uniform(lo[0], hi[0]), rng.uniform(lo[1], hi[1])
        if osamp.turing_space(a, b, d):
            start.append((a, b, math.log(200.0), math.log(d)))
            if len(start) == C:
                break
    assert len(start) == C, "the Turing space fills too little of the box"
    phis = np.array(start)
    lls = np.zeros(C)
    step = (0.02, 0.05, 0.0, 0.0)
    for st in range(S):
        phis, lls, _, _ = osamp.rwm_batch_step(phis, lls, 33, st, lo, hi, step, 0b0011,
                                               lambda q: np.zeros(len(q)), prior=pr)
    assert all(osamp.turing_space(p[0], p[1], d) for p in phis)
    sa, sb = A[mask].std(), B[mask].std()
    assert abs(phis[:, 0].mean() - ca) < 4 * sa / math.sqrt(C)
    assert abs(phis[:, 1].mean() - cb) < 4 * sb / math.sqrt(C)


def test_inputs_box_draws_unchanged():
    """The shared input generator is untouched by the prior options."""
    x = inputs.box_draws(3, (0, 0, 0, 0), (1, 1, 1, 1), seed=3)
    assert x.shape == (3, 4) and np.all((x >= 0) & (x <= 1))
