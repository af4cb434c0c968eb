"""The one-dimensional growing domain of Example 1 (Sec. 3.1.2) on the GPU
against the oracle, through the C ABI: forward fields for the polynomial and
the data growth laws, the fused misfit with non-positive growth, and
Metropolis chains over the growth coefficients."""
import math

import numpy as np
import pytest

from oracle import growth1d as og
from oracle import sampler as osamp
from gpu_common import need_gpu, rel_l2
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu

THETA1 = (0.1, 0.9, 1000.0, 10.0)  # Example 1's fixed a, b, gamma, d
TAU = 1e-4
RHO_T = 1.8


def make(n, steps, **kw):
    from paper_1605_04718_amd.api import Growth1D
    u0, v0 = inputs.initial_fields_1d(n)
    return Growth1D(n, steps, TAU, THETA1, u0, v0, rho_T=RHO_T, **kw), u0, v0


def betas(m, seed):
    return inputs.box_draws(m, (-0.5, -0.5, -0.5), (1.5, 1.0, 1.0), seed=seed)


@pytest.mark.parametrize("n,steps", [(100, 1500), (37, 800), (128, 600), (64, 500), (2, 300)])
def test_polynomial_growth_fields_match_oracle(n, steps):
    """Several reduction depths (n = 2 .. 128, ragged and power-of-two) with
    a fast-changing rho (T = steps tau)."""
    import torch
    need_gpu()
    g, u0, v0 = make(n, steps, max_batch=8)
    B = betas(5, seed=40 + n)
    u, v, st = g.forward(torch.tensor(B, device="cuda"))
    torch.cuda.synchronize()
    u, v, st = u.cpu().numpy(), v.cpu().numpy(), st.cpu().numpy()
    for k in range(len(B)):
        assert og.growth_positive(B[k], RHO_T, TAU, steps)
        uo, vo = og.forward_beta(THETA1, B[k], RHO_T, u0, v0, TAU, steps)
        assert st[k] == 0
        assert rel_l2(u[k], uo) < 1e-11 and rel_l2(v[k], vo) < 1e-11, (k, rel_l2(u[k], uo))
    g.close()


@pytest.mark.parametrize("law", [1, 2])
def test_data_growth_laws_match_oracle(law):
    """Exponential and logistic growth of eq. (grates), over a window that
    starts at t = 0."""
    import torch
    need_gpu()
    n, steps = 100, 2000
    g, u0, v0 = make(n, steps, law=law, max_batch=2)
    u, v, st = g.forward(None, m=2)
    torch.cuda.synchronize()
    fn = og.rho_exp_pair if law == 1 else og.rho_log_pair
    uo, vo = og.forward(THETA1, u0, v0, TAU, steps, fn)
    u, v = u.cpu().numpy(), v.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    assert rel_l2(u[0], uo) < 1e-11 and rel_l2(v[1], vo) < 1e-11
    assert np.array_equal(u[0], u[1])
    g.close()


@pytest.mark.parametrize("obs", [1, 2, 3])
def test_loglik_matches_oracle_and_rejects_negative_growth(obs):
    import torch
    need_gpu()
    n, steps = 100, 600
    u0, v0 = inputs.initial_fields_1d(n)
    uo, vo = og.forward(THETA1, u0, v0, TAU, steps, og.rho_exp_pair)
    ytrue = np.stack([uo, vo])
    y, sigma = inputs.noisy_data(ytrue, 0.05, seed=9)
    g, _, _ = make(n, steps, y=y, obs=obs, sigma=sigma, max_batch=16)
    B = betas(12, seed=7)
    B[3] = (-5.0, 0.0, 0.0)   # rho < 0 inside [0, T]
    B[8] = (0.6, 0.0, 0.0)
    phi, st = g.log_likelihood(torch.tensor(B, device="cuda"))
    torch.cuda.synchronize()
    phi, st = phi.cpu().numpy(), st.cpu().numpy()
    for k in range(len(B)):
        want = og.loglik_beta(THETA1, B[k], RHO_T, u0, v0, TAU, steps, y, sigma, obs)
        if math.isinf(want):
            assert math.isinf(phi[k]) and st[k] == 8, k
        else:
            assert st[k] == 0 and phi[k] == pytest.approx(want, rel=1e-10), k
    assert math.isinf(phi[3]) and np.isfinite(phi).sum() == 11
    g.close()


def test_chains_over_growth_coefficients_match_oracle():
    """Metropolis chains over beta with a normal prior on beta_1 and
    uniform priors on beta_2, beta_3: the GPU follows the oracle's chains
    (decisions within 1e-7 of a tie are not compared)."""
    import torch
    from paper_1605_04718_amd.api import ChainState
    need_gpu()
    n, steps, C, S = 32, 150, 12, 8
    u0, v0 = inputs.initial_fields_1d(n)
    beta_true = (0.7, 0.1, 0.0)
    uo, vo = og.forward_beta(THETA1, beta_true, RHO_T, u0, v0, TAU, steps)
    y, sigma = inputs.noisy_data(np.stack([uo, vo]), 0.05, seed=12)
    lo, hi = (-1.0, -2.0, -2.0), (3.0, 2.0, 2.0)
    step = (0.3, 0.3, 0.3)
    pk, pm, ps = (1, 0, 0), (0.8, 0.0, 0.0), (0.5, 1.0, 1.0)
    g, _, _ = make(n, steps, y=y, obs=3, sigma=sigma, max_batch=C, lo=lo, hi=hi, step=step,
                   prior_kind=pk, prior_mean=pm, prior_sd=ps)
    phi0 = np.zeros((C, 4))
    phi0[:, :3] = beta_true
    phi0[:, 0] += np.linspace(-0.2, 0.2, C)

    def ll(q):
        return og.loglik_beta(THETA1, q[:3], RHO_T, u0, v0, TAU, steps, y, sigma, obs=3)

    ll0 = np.array([ll(q) for q in phi0])
    ch = ChainState.create(torch.tensor(phi0, device="cuda"), torch.tensor(ll0, device="cuda"),
                           seed=17, trace_steps=S)
    g.mcmc_step(ch, S)
    torch.cuda.synchronize()
    assert ch.step == S
    trace = ch.trace.cpu().numpy()
    prior = osamp.Prior(kinds=pk + (0,), mean=pm + (0.0,), sd=ps + (1.0,))
    olo, ohi = lo + (-math.inf,), hi + (math.inf,)
    ostep = step + (0.0,)
    compared = accepted = 0
    for c in range(C):
        x, lx = phi0[c].copy(), ll0[c]
        for s in range(S):
            prop = osamp.propose(x, 17, c, s, ostep, 0b0111)
            tie = False
            if osamp.in_support(prop, olo, ohi, prior):
                lp = ll(prop)
                la = (lx - lp) + osamp.log_prior_ratio(x, prop, prior)
                lu = math.log(oracle_uniform(17, c, s))
                tie = abs(lu - la) < 1e-7
                if lu < la:
                    x, lx = prop, lp
                    accepted += 1
            if tie:
                break
            assert np.allclose(trace[s, c], x, rtol=1e-13, atol=1e-14), (c, s)
            compared += 1
    assert compared >= C * S - 2 * S and accepted > 0
    assert int(ch.n_solves.sum()) > 0
    g.close()


def oracle_uniform(seed, c, s):
    import oracle
    return oracle.uniform1(seed, c, s, osamp.PURPOSE_ACCEPT)


def test_arguments_are_checked():
    from paper_1605_04718_amd._lib import RDError
    need_gpu()
    for n in (1, 129):
        with pytest.raises(RDError):
            make(n, 10)
    g, _, _ = make(16, 10, max_batch=4)
    import torch
    with pytest.raises(RDError):
        g.log_likelihood(torch.zeros((2, 3), dtype=torch.float64, device="cuda"))  # no data
    with pytest.raises(RDError):
        g.forward(torch.zeros((5, 3), dtype=torch.float64, device="cuda"))  # > max_batch
    g.close()


def test_bench_launch_sampled_items_match_oracle():
    """The launch the 1-D bench leg times (4096 growth-coefficient draws,
    n = 100, 20 000 steps, data from exponential growth with 5 % noise):
    misfits of sampled items against the oracle's."""
    import torch
    need_gpu()
    n, steps, m = 100, 20000, 4096
    u0, v0 = inputs.initial_fields_1d(n)
    ud, vd = og.forward(THETA1, u0, v0, TAU, steps, og.rho_exp_pair)
    y, sigma = inputs.noisy_data(np.stack([ud, vd]), 0.05, seed=inputs.SEED_DATA_NOISE)
    rho_T = math.exp(0.001 * steps * TAU)
    from paper_1605_04718_amd.api import Growth1D
    g = Growth1D(n, steps, TAU, THETA1, u0, v0, rho_T=rho_T, y=y, obs=3, sigma=sigma,
                 max_batch=m)
    B = inputs.box_draws(m, (-0.2, -0.2, -0.2), (0.4, 0.2, 0.2), seed=inputs.SEED_DATASET)
    phi, st = g.log_likelihood(torch.tensor(B, device="cuda"))
    torch.cuda.synchronize()
    phi, st = phi.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0) and np.all(np.isfinite(phi))
    for k in (0, 1234, m - 1):
        want = og.loglik_beta(THETA1, B[k], rho_T, u0, v0, TAU, steps, y, sigma, obs=3)
        assert phi[k] == pytest.approx(want, rel=1e-9), k
    g.close()
