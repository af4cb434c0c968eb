"""Pins of the oracle's parallel Metropolis-Hastings (Sec. 2, Algorithm 2),
CPU only."""
import math

import numpy as np
import pytest

import oracle
from oracle import sampler as osamp


def _softmax(logw):
    logw = np.asarray(logw, dtype=np.float64)
    m = np.max(logw)
    w = np.where(np.isfinite(logw), np.exp(logw - m), 0.0)
    return w / w.sum()


@pytest.mark.parametrize("n_prop", [1, 2, 7, 32])
def test_stationary_distribution_is_the_normalised_target(n_prop):
    """A is a Metropolis chain on the N + 1 points with a uniform choice of
    the other point, so detailed balance gives p_j proportional to w_j: the
    dense solve of the definition must return that closed form."""
    rng = np.random.default_rng(n_prop)
    for trial in range(20):
        logw = rng.normal(0.0, 3.0, n_prop + 1)
        if trial % 3 == 1 and n_prop > 1:
            logw[rng.integers(1, n_prop + 1)] = -np.inf  # proposal outside the support
        A = osamp.pmh_matrix(logw)
        assert np.all(A >= 0) and np.allclose(A.sum(1), 1.0, atol=1e-15)
        p = osamp.stationary(A)
        assert np.allclose(p, _softmax(logw), rtol=1e-10, atol=1e-15)
        assert np.allclose(p @ A, p, atol=1e-14)


def test_draws_follow_the_running_sum():
    p = np.array([0.1, 0.0, 0.6, 0.3])
    assert osamp.pmh_draw(p, 0.05) == 0
    assert osamp.pmh_draw(p, 0.1) == 2
    assert osamp.pmh_draw(p, 0.69) == 2
    assert osamp.pmh_draw(p, 0.71) == 3
    assert osamp.pmh_draw(p, 1.0 - 1e-17) == 3


def test_points_use_the_auxiliary_point():
    """Proposal j is z + s z_j with z = x + s z_aux (purposes 6 and 7)."""
    phi = np.array([0.2, 0.7, 5.0, 2.0])
    s = np.array([0.01, 0.02, 0.05, 0.05])
    pts = osamp.pmh_points(phi, 9, 4, 11, 3, s, 0b1111)
    z = phi + s * oracle.normals4_at(9, 4, 11, osamp.PURPOSE_PMH_AUX, 0)
    assert np.array_equal(pts[0], phi)
    for j in range(3):
        want = z + s * oracle.normals4_at(9, 4, 11, osamp.PURPOSE_PMH_PROP, 2 * j)
        assert np.allclose(pts[j + 1], want, rtol=0, atol=1e-15)


def _toy_run(n_prop, aux, C=1200, S=6, seed=17):
    """Chains started from exact draws of a 2-D Gaussian target; returns the
    draws of the last step.  aux=False draws the proposals around x_k as
    printed (no auxiliary point)."""
    mu = np.array([0.4, 0.6, 5.0, 2.0])
    sd = np.array([0.05, 0.08, 1.0, 1.0])
    step = np.array([0.06, 0.1, 0.0, 0.0])
    lo, hi = np.array([-5.0, -5.0, 5.0, 2.0]), np.array([5.0, 5.0, 5.0, 2.0])

    def phi_fn(q):
        return 0.5 * float((((np.asarray(q) - mu) / sd)[:2] ** 2).sum())

    rng = np.random.default_rng(seed)
    x = np.tile(mu, (C, 1))
    x[:, :2] = rng.normal(mu[:2], sd[:2], (C, 2))
    ll = np.array([phi_fn(q) for q in x])
    draws = None
    for s in range(S):
        out = []
        for c in range(C):
            if aux:
                d, dl, _, _, _, _ = osamp.pmh_step(x[c], ll[c], seed, c, s, n_prop, lo, hi, step,
                                                   0b0011, phi_fn)
            else:
                pts = [x[c]] + [x[c] + step * oracle.normals4_at(seed, c, s,
                                                                 osamp.PURPOSE_PMH_PROP, 2 * j)
                                for j in range(n_prop)]
                lw = np.array([-phi_fn(q) for q in pts])
                p = osamp.stationary(osamp.pmh_matrix(lw))
                idx = [osamp.pmh_draw(p, oracle.uniform_at(seed, c, s, osamp.PURPOSE_PMH_RESAMPLE,
                                                           n)) for n in range(n_prop)]
                d = np.stack([pts[i] for i in idx])
                dl = np.array([phi_fn(q) for q in d])
            out.append(d)
            x[c], ll[c] = d[-1], dl[-1]
        draws = np.concatenate(out)
    return draws, mu, sd


def test_auxiliary_point_leaves_the_target_invariant():
    """Draws after several steps keep the target's mean and s.d.; the
    printed variant (proposals around x_k) shrinks the spread."""
    draws, mu, sd = _toy_run(8, aux=True)
    n = len(draws) / 8  # draws within a step are correlated: a conservative count
    for i in (0, 1):
        assert abs(draws[:, i].mean() - mu[i]) < 4 * sd[i] / math.sqrt(n)
        assert abs(draws[:, i].std() / sd[i] - 1.0) < 0.05
    printed, _, _ = _toy_run(8, aux=False)
    assert printed[:, 0].std() / sd[0] < 0.93 and printed[:, 1].std() / sd[1] < 0.93
