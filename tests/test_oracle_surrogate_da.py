"""Pins of the surrogate misfit, Adam and the delayed-acceptance step.

Each pin is a check against a value fixed by the mathematics, not by the
oracle's own formula: closed forms of the first-stage misfit for networks
whose output is known exactly, Adam moments derived by hand (exact rational
moments, decimal square roots), and the stationary law of delayed
acceptance on Gaussian toy targets whose posterior is known in closed form.
Every check is also run on a planted mistake (a dropped 1/2, sigma1 instead
of sigma1^2, a constant bias correction, the prior ratio in the second
stage, a surrogate chain corrected by the plain Metropolis ratio) and must
fail there.
"""
import math

import numpy as np
import pytest

from oracle import mlp
from oracle import sampler as osamp


# --------------------------------------------------------------------------
# First-stage misfit Phi~ = |ybar - (mean + sd * net(x))|^2 / (2 sigma1^2)

def _constant_net(out, c):
    """4 -> 3 -> out, every weight zero, output bias c: net(x) = c."""
    return [(np.zeros((3, 4)), np.zeros(3)), (np.zeros((out, 3)), np.full(out, c))]


def _check_constant_offset(fn):
    # 4 x 4 output field, ybar - mean = 0.3 everywhere, sd = 2, net = 0.4:
    # every pixel misses by 0.3 - 2 * 0.4 = -0.5, so
    # Phi~ = 16 * 0.25 / (2 * 0.5^2) = 8 exactly.
    lo, hi = np.zeros(4), np.ones(4)
    mean = np.full(16, 1.7)
    ybar = np.full(16, 2.0)
    got = fn(_constant_net(16, 0.4), np.full(4, 0.5), lo, hi, mean, 2.0 * np.ones(16), ybar, 0.5)
    assert got.shape == (1,)
    assert got[0] == pytest.approx(8.0, rel=1e-14)
    # a network that predicts the data exactly has zero misfit
    got0 = fn(_constant_net(16, 0.0), np.full(4, 0.5), lo, hi, ybar, np.ones(16), ybar, 0.5)
    assert got0[0] == 0.0


def _selector_net(coord):
    """4 -> 1 -> 4 with net(x) = x_coord on every output: the hidden unit sees
    x_coord + 40, where GELU is the identity to double precision
    (erf(39 / sqrt 2) rounds to 1), and the output subtracts the 40."""
    W1 = np.zeros((1, 4))
    W1[0, coord] = 1.0
    return [(W1, np.array([40.0])), (np.ones((4, 1)), np.full(4, -40.0))]


def _check_input_scaling(fn):
    # prior box of the b coordinate [2, 6]: phi_b = 2, 6, 5 map to x = -1, 1, 0.5,
    # so Phi~ = 4 x^2 / 2 (2 x 2 field, mean 0, sd 1, ybar 0, sigma1 1)
    lo = np.array([0.0, 2.0, 1.0, -1.0])
    hi = np.array([1.0, 6.0, 3.0, 1.0])
    phis = np.array([[0.5, 2.0, 2.0, 0.0], [0.5, 6.0, 2.0, 0.0], [0.5, 5.0, 2.0, 0.0]])
    got = fn(_selector_net(1), phis, lo, hi, np.zeros(4), np.ones(4), np.zeros(4), 1.0)
    assert np.allclose(got, [2.0, 2.0, 0.5], rtol=0, atol=1e-12)


def test_surrogate_misfit_closed_forms():
    _check_constant_offset(mlp.surrogate_misfit)
    _check_input_scaling(mlp.surrogate_misfit)


def test_scale_inputs_maps_the_box_to_the_unit_interval():
    lo, hi = np.array([0.0, 2.0, -3.0, 1.0]), np.array([1.0, 6.0, 5.0, 1.5])
    assert np.array_equal(mlp.scale_inputs(lo, lo, hi), -np.ones(4))
    assert np.array_equal(mlp.scale_inputs(hi, lo, hi), np.ones(4))
    assert np.allclose(mlp.scale_inputs((lo + hi) / 2, lo, hi), 0.0, atol=1e-15)


def test_surrogate_misfit_pins_catch_planted_mistakes():
    def no_half(params, phi, lo, hi, mean, sd, ybar, sigma1):
        y, _ = mlp.forward(params, mlp.scale_inputs(np.atleast_2d(phi), lo, hi))
        return ((ybar.ravel() - (mean + sd * y)) ** 2).sum(axis=1) / sigma1 ** 2

    def sigma_not_squared(params, phi, lo, hi, mean, sd, ybar, sigma1):
        y, _ = mlp.forward(params, mlp.scale_inputs(np.atleast_2d(phi), lo, hi))
        return 0.5 * ((ybar.ravel() - (mean + sd * y)) ** 2).sum(axis=1) / sigma1

    def sd_dropped(params, phi, lo, hi, mean, sd, ybar, sigma1):
        y, _ = mlp.forward(params, mlp.scale_inputs(np.atleast_2d(phi), lo, hi))
        return 0.5 * ((ybar.ravel() - (mean + y)) ** 2).sum(axis=1) / sigma1 ** 2

    def unit_box(params, phi, lo, hi, mean, sd, ybar, sigma1):
        x = (np.atleast_2d(phi) - lo) / (hi - lo)  # [0, 1] instead of [-1, 1]
        y, _ = mlp.forward(params, x)
        return 0.5 * ((ybar.ravel() - (mean + sd * y)) ** 2).sum(axis=1) / sigma1 ** 2

    for bad in (no_half, sigma_not_squared, sd_dropped):
        with pytest.raises(AssertionError):
            _check_constant_offset(bad)
    with pytest.raises(AssertionError):
        _check_input_scaling(unit_box)


# --------------------------------------------------------------------------
# Adam over several steps

def _two_layer_params():
    return [(np.array([[1.0, -2.0, 0.5], [0.0, 3.0, -1.0]]), np.array([0.25, -0.75])),
            (np.array([[2.0, 1.0]]), np.array([-1.5]))]


def _check_constant_gradient(step_fn):
    # With a constant gradient g the moments are m_t = (1 - b1^t) g and
    # v_t = (1 - b2^t) g^2, so the bias-corrected moments are g and g^2 at
    # every t and each step moves a parameter by lr g / (|g| + eps).
    params = _two_layer_params()
    grads = [(np.array([[0.3, -4.0, 1e-9], [2.0, -0.5, 7.0]]), np.array([1e-3, -2.5])),
             (np.array([[-0.02, 5.0]]), np.array([-3e-9]))]
    lr, eps = 1e-2, 1e-8
    st = {}
    cur = params
    for _ in range(3):
        cur = step_fn(cur, grads, st, lr)
    for (W0, b0), (W3, b3), (gW, gb) in zip(params, cur, grads):
        for p0, p3, g in ((W0, W3, gW), (b0, b3, gb)):
            want = p0 - 3 * lr * g / (np.abs(g) + eps)
            assert np.allclose(p3, want, rtol=0, atol=1e-13), (p3, want)


def _check_hand_sequence(step_fn):
    # gradients 1, -2, 1/2 at lr 0.1 from p = 0; exact moments
    #   t=1: m = 1/10,     v = 1/1000,          m^ = 1,      v^ = 1
    #   t=2: m = -11/100,  v = 4999/10^6,       m^ = -11/19, v^ = 4999/1999
    #   t=3: m = -49/1000, v = 5244001/10^9,    m^ = -49/271, v^ = 749143/428143
    # and p_t = p_{t-1} - lr m^ / (sqrt(v^) + 1e-8) in 40-digit decimals:
    want = [-0.09999999900000000999999990000000099999999,
            -0.06338964652792491179449285107285070167998,
            -0.04972058032617827440666908045065548322021]
    params = [(np.array([[0.0]]), np.array([0.0]))]
    st = {}
    for g, w in zip((1.0, -2.0, 0.5), want):
        grads = [(np.array([[g]]), np.array([0.0]))]
        params = step_fn(params, grads, st, 0.1)
        assert params[0][0][0, 0] == pytest.approx(w, rel=1e-13, abs=1e-16)
    assert st["t"] == 3


def test_adam_several_steps_closed_forms():
    _check_constant_gradient(mlp.adam_step)
    _check_hand_sequence(mlp.adam_step)


def test_adam_pins_catch_a_constant_bias_correction():
    def constant_correction(params, grads, state, lr, b1=0.9, b2=0.999, eps=1e-8):
        # planted: divides by (1 - beta) instead of (1 - beta^t)
        if not state:
            state["t"] = 0
            state["m"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
            state["v"] = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        state["t"] += 1
        out = []
        for i, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new, ms, vs = [], [], []
            for j, (p, g) in enumerate(((W, gW), (b, gb))):
                m = b1 * state["m"][i][j] + (1 - b1) * g
                v = b2 * state["v"][i][j] + (1 - b2) * g * g
                new.append(p - lr * (m / (1 - b1)) / (np.sqrt(v / (1 - b2)) + eps))
                ms.append(m)
                vs.append(v)
            state["m"][i], state["v"][i] = tuple(ms), tuple(vs)
            out.append(tuple(new))
        return out

    with pytest.raises(AssertionError):
        _check_constant_gradient(constant_correction)
    with pytest.raises(AssertionError):
        _check_hand_sequence(constant_correction)


# --------------------------------------------------------------------------
# Delayed acceptance leaves the posterior invariant

BOX_LO = np.array([-1e3, -1e3, -1e3, -1e3])
BOX_HI = np.array([1e3, 1e3, 1e3, 1e3])


def _da_chains(phi0, loglik_fn, sur_fn, step_sd, free_mask, prior, S, seed):
    """S delayed-acceptance steps of every row of phi0 (chain index = row)."""
    phis = np.array(phi0, dtype=np.float64)
    ll = np.array([loglik_fn(p) for p in phis])
    ls = np.array([sur_fn(p) for p in phis])
    n1 = n2 = 0
    for s in range(S):
        for c in range(len(phis)):
            phis[c], ll[c], ls[c], a1, a, _ = osamp.da_step(
                phis[c], ll[c], ls[c], seed, c, s, BOX_LO, BOX_HI, step_sd, free_mask, loglik_fn,
                sur_fn, prior=prior)
            n1 += a1
            n2 += a
    return phis, n1, n2


# Normal prior N(0, 1) on coordinate 2 (a log-normal gamma, Case 3 of
# Sec. 3.1.2) and a Gaussian likelihood centred at 2 with s.d. 1: the
# posterior is N(1, 1/2).  The surrogate is a biased, wider Gaussian.
_PRIOR = osamp.Prior(kinds=(0, 0, 1, 0), mean=(0.0, 0.0, 0.0, 0.0), sd=(1.0, 1.0, 1.0, 1.0))


def _lik(p):
    return 0.5 * (float(p[2]) - 2.0) ** 2


def _sur(p):
    return 0.5 * (float(p[2]) - 2.4) ** 2 / 1.3 ** 2


def _check_normal_prior_posterior(loglik_fn, prior, C=300, S=120):
    rng = np.random.default_rng(41)
    phi0 = np.zeros((C, 4))
    phi0[:, 2] = rng.normal(1.0, math.sqrt(0.5), C)  # exact posterior draws
    phis, n1, n2 = _da_chains(phi0, loglik_fn, _sur, np.array([0, 0, 1.4, 0]), 0b0100, prior, S,
                              seed=77)
    x = phis[:, 2]
    assert 0.2 < n2 / (C * S) < 0.9
    assert n1 > n2  # the biased surrogate is not exact: stage 2 rejects some
    se = math.sqrt(0.5 / C)
    assert abs(x.mean() - 1.0) < 4.5 * se, x.mean()
    assert abs(x.std() - math.sqrt(0.5)) < 4.5 * math.sqrt(0.5) / math.sqrt(2 * C), x.std()


def test_da_with_normal_prior_and_biased_surrogate_keeps_the_posterior():
    _check_normal_prior_posterior(_lik, _PRIOR)


def test_da_invariance_pin_catches_a_prior_ratio_in_stage_two():
    # planted: the prior's log density also enters the second stage (as if
    # Phi carried it), so the chain targets prior^2 x likelihood = N(2/3, 1/3)
    def lik_with_prior(p):
        return _lik(p) + osamp.prior_quad(p, _PRIOR)

    with pytest.raises(AssertionError):
        _check_normal_prior_posterior(lik_with_prior, _PRIOR)
    # planted: no prior ratio at all (the chain targets the likelihood, N(2, 1))
    with pytest.raises(AssertionError):
        _check_normal_prior_posterior(_lik, None)


def test_da_with_biased_surrogate_recovers_a_correlated_gaussian():
    """Uniform (wide box) prior, 2-D correlated Gaussian target, surrogate
    with a shifted mean and a different, uncorrelated covariance: mean and
    covariance of the target are kept."""
    mu = np.array([0.5, -1.0])
    cov = np.array([[1.0, 0.6], [0.6, 2.0]])
    icov = np.linalg.inv(cov)
    mus = mu + np.array([0.3, -0.4])
    icovs = np.diag([1 / 1.5, 1 / 2.5])

    def lik(p):
        e = np.asarray(p)[:2] - mu
        return 0.5 * float(e @ icov @ e)

    def sur(p):
        e = np.asarray(p)[:2] - mus
        return 0.5 * float(e @ icovs @ e)

    C, S = 300, 60
    rng = np.random.default_rng(5)
    phi0 = np.zeros((C, 4))
    phi0[:, :2] = rng.multivariate_normal(mu, cov, C)
    phis, n1, n2 = _da_chains(phi0, lik, sur, np.array([1.5, 1.5, 0, 0]), 0b0011, None, S, seed=3)
    x = phis[:, :2]
    assert n1 > n2 > 0
    se = np.sqrt(np.diag(cov) / C)
    assert np.all(np.abs(x.mean(0) - mu) < 4.5 * se)
    emp = np.cov(x.T)
    bound = 4.5 * np.sqrt((cov ** 2 + np.outer(np.diag(cov), np.diag(cov))) / C)
    assert np.all(np.abs(emp - cov) < bound)


# --------------------------------------------------------------------------
# Delayed acceptance with a surrogate chain as the first stage

def _chain_run(phi0, step_fn, S, seed):
    phis = np.array(phi0, dtype=np.float64)
    ll = np.array([_lik(p) for p in phis])
    ls = np.array([_sur(p) for p in phis])
    moved = acc = 0
    for s in range(S):
        for c in range(len(phis)):
            phis[c], ll[c], ls[c], m1, a, _ = step_fn(phis[c], ll[c], ls[c], seed, c, s)
            moved += m1
            acc += a
    return phis, moved, acc


def test_surrogate_chain_with_one_substep_is_the_delayed_acceptance_step():
    """m = 1 uses the same random numbers as da_step and takes the same
    decisions: identical paths, bit for bit."""
    step_sd = np.array([0, 0, 1.4, 0])
    pa = pb = np.array([0.0, 0.0, 0.3, 0.0])
    la = lb = _lik(pa)
    sa = sb = _sur(pa)
    for s in range(200):
        pa, la, sa, a1, aa, _ = osamp.da_step(pa, la, sa, 9, 2, s, BOX_LO, BOX_HI, step_sd,
                                              0b0100, _lik, _sur, prior=_PRIOR)
        pb, lb, sb, b1, ab, _ = osamp.da_chain_step(pb, lb, sb, 9, 2, s, 1, BOX_LO, BOX_HI,
                                                    step_sd, 0b0100, _lik, _sur, prior=_PRIOR)
        assert a1 == b1 and aa == ab
        assert np.array_equal(pa, pb) and la == lb and sa == sb


def _check_chain_posterior(step_fn, C=300, S=40):
    rng = np.random.default_rng(43)
    phi0 = np.zeros((C, 4))
    phi0[:, 2] = rng.normal(1.0, math.sqrt(0.5), C)  # exact posterior draws
    phis, moved, acc = _chain_run(phi0, step_fn, S, seed=78)
    x = phis[:, 2]
    assert 0.2 < acc / (C * S) < 1.0 and moved > acc
    se = math.sqrt(0.5 / C)
    assert abs(x.mean() - 1.0) < 4.5 * se, x.mean()
    assert abs(x.std() - math.sqrt(0.5)) < 4.5 * math.sqrt(0.5) / math.sqrt(2 * C), x.std()


def _chain_step(m, prior=_PRIOR):
    def f(p, l, ls, seed, c, s):
        return osamp.da_chain_step(p, l, ls, seed, c, s, m, BOX_LO, BOX_HI,
                                   np.array([0, 0, 1.4, 0]), 0b0100, _lik, _sur, prior=prior)
    return f


def test_surrogate_chain_keeps_the_posterior():
    """Five substeps on a biased, wider surrogate with a normal prior: the
    posterior N(1, 1/2) is kept."""
    _check_chain_posterior(_chain_step(5))


def test_surrogate_chain_pin_catches_planted_mistakes():
    # planted: the second stage takes the plain Metropolis ratio
    # Phi(x) - Phi(y) on the end point of the surrogate chain, without the
    # surrogate's [Phi~(x) - Phi~(y)]; passing Phi + Phi~(y) - Phi~(x) as the
    # misfit of y makes da_chain_step's second stage exactly that
    def plain_second_stage(p, l, ls, seed, c, s):
        y, _, ls_y, m1, a, solved = osamp.da_chain_step(
            p, l, ls, seed, c, s, 5, BOX_LO, BOX_HI, np.array([0, 0, 1.4, 0]), 0b0100,
            lambda q: _lik(q) + _sur(q) - _sur(p), _sur, prior=_PRIOR)
        if a:
            return y, _lik(y), ls_y, m1, a, solved
        return p, l, ls, m1, a, solved

    with pytest.raises(AssertionError):
        _check_chain_posterior(plain_second_stage)
    # planted: the substeps leave out the prior ratio (they target exp(-Phi~) alone)
    with pytest.raises(AssertionError):
        _check_chain_posterior(_chain_step(5, prior=None))
