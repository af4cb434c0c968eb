"""Priors of Sec. 3.1.2 on the GPU sampler (Turing-space support, Case 2;
log-normal gamma and d, Case 3) against the oracle, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from oracle import sampler as osamp
from gpu_common import THETA_TRUE, TAU, need_gpu
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu

LO = np.array([0.0, 0.0, math.log(50.0), math.log(5.0)])
HI = np.array([1.0, 1.0, math.log(500.0), math.log(50.0)])
NORMAL = dict(prior_kind=(0, 0, 1, 1), prior_mean=(0.0, 0.0, math.log(500.0), math.log(5.0)),
              prior_sd=(1.0, 1.0, 0.95, 0.95))
ORACLE_NORMAL = osamp.Prior(kinds=(0, 0, 1, 1), mean=(0.0, 0.0, math.log(500.0), math.log(5.0)),
                            sd=(1.0, 1.0, 0.95, 0.95))


def problem(n=32, steps=1, max_batch=512, **kw):
    """A problem for sampler-kernel tests (no data: Phi comes from the test)."""
    from paper_1605_04718_amd.api import Grid, Problem
    u0, v0 = inputs.initial_fields(n, 0.1, 0.9)
    args = dict(lo=LO, hi=HI, free_mask=0b1111, max_batch=max_batch, step=(0.02, 0.02, 0.05, 0.05))
    args.update(kw)
    return Problem([Grid(n=n, u0=u0, v0=v0)], TAU, steps, 1e-7, **args)


def chains_at(phi, ll, seed, **kw):
    import torch
    from paper_1605_04718_amd.api import ChainState
    return ChainState.create(torch.tensor(phi, dtype=torch.float64, device="cuda"),
                             torch.tensor(ll, dtype=torch.float64, device="cuda"), seed=seed, **kw)


def _turing_margin(a, b, d):
    s = a + b
    tr = (b - a) / s - s * s
    dfg = d * ((b - a) / s) - s * s
    disc = dfg * dfg - 4.0 * d * s * s
    return min(abs(tr), abs(dfg), abs(disc) / (1.0 + dfg * dfg))


def test_turing_support_proposals_match_oracle():
    """Inside flags with the Turing support equal the oracle's wherever the
    Turing inequalities are not within rounding of their boundary."""
    import torch
    need_gpu()
    C = 600
    lo = np.array([0.0, 0.4, math.log(200.0), math.log(5.0)])
    hi = np.array([0.3, 1.1, math.log(200.0), math.log(20.0)])
    p = problem(lo=lo, hi=hi, step=(0.03, 0.05, 0.0, 0.2), free_mask=0b1011, turing_support=True,
                max_batch=C)
    phi = inputs.box_draws(C, lo, hi, seed=14)
    ch = chains_at(phi, np.zeros(C), seed=91)
    ch.step = 777
    prop, inside = p.propose(ch)
    torch.cuda.synchronize()
    prop, inside = prop.cpu().numpy(), inside.cpu().numpy()
    pr = osamp.Prior(turing=True)
    compared = n_in = 0
    for c in range(C):
        want = osamp.propose(phi[c], 91, c, 777, (0.03, 0.05, 0.0, 0.2), 0b1011)
        assert np.allclose(prop[c], want, rtol=1e-14, atol=1e-14)
        if _turing_margin(want[0], want[1], math.exp(want[3])) < 1e-9:
            continue
        flag = osamp.in_support(want, lo, hi, pr)
        assert bool(inside[c]) == flag, (c, want)
        compared += 1
        n_in += flag
    assert compared > C - 5 and 0 < n_in < compared
    p.close()


def test_normal_prior_accept_decisions_bitwise():
    """log U < [Phi - Phi'] + [log pi(phi') - log pi(phi)]: the same FP64
    arithmetic on both sides, so every decision agrees."""
    import torch
    need_gpu()
    C = 500
    p = problem(max_batch=C, **NORMAL)
    rng = np.random.default_rng(8)
    phi = inputs.box_draws(C, LO, HI, seed=15)
    phi[:, 2] = rng.normal(math.log(500.0), 1.5, C)  # normal coordinates range past the box
    phi[:, 3] = rng.normal(math.log(5.0), 1.5, C)
    ll = rng.uniform(0, 3, C)
    ch = chains_at(phi, ll, seed=61)
    ch.step = 5
    prop, inside = p.propose(ch)
    llp = torch.tensor(rng.uniform(0, 3, C), dtype=torch.float64, device="cuda")
    p.accept(ch, prop, inside, llp)
    torch.cuda.synchronize()
    prop_h, inside_h, llp_h = prop.cpu().numpy(), inside.cpu().numpy(), llp.cpu().numpy()
    n_acc = ch.n_accept.cpu().numpy()
    outside_box = 0
    for c in range(C):
        flag = osamp.in_support(prop_h[c], LO, HI, ORACLE_NORMAL)
        assert bool(inside_h[c]) == flag
        outside_box += flag and not osamp.in_box(prop_h[c], LO, HI)
        acc = False
        if flag:
            u = oracle.uniform1(61, c, 5, osamp.PURPOSE_ACCEPT)
            acc = math.log(u) < (ll[c] - llp_h[c]) + osamp.log_prior_ratio(phi[c], prop_h[c],
                                                                           ORACLE_NORMAL)
        assert bool(n_acc[c]) == acc, c
    assert outside_box > 0  # proposals beyond lo/hi on normal coordinates are kept
    p.close()


def test_normal_prior_toy_chain_matches_oracle_chain():
    """Gaussian toy likelihood times the log-normal prior: the GPU chains
    follow the oracle's chains step for step."""
    import torch
    need_gpu()
    C, S = 64, 120
    mu = np.array([0.3, 0.6, 5.5, 2.0])
    sd = np.array([0.05, 0.08, 0.6, 0.5])
    step = 1.0 * sd

    def phi_np(q):
        return 0.5 * (((np.atleast_2d(q) - mu) / sd) ** 2).sum(1)

    p = problem(max_batch=C, step=step, **NORMAL)
    start = np.tile(mu, (C, 1))
    ch = chains_at(start, phi_np(start), seed=44)
    mu_t, sd_t = torch.tensor(mu, device="cuda"), torch.tensor(sd, device="cuda")
    phis, lls = start.copy(), phi_np(start)
    for s in range(S):
        prop, inside = p.propose(ch)
        llp = 0.5 * (((prop - mu_t) / sd_t) ** 2).sum(1)
        p.accept(ch, prop, inside, llp.contiguous())
        phis, lls, _, _ = osamp.rwm_batch_step(phis, lls, 44, s, LO, HI, step, 0b1111, phi_np,
                                               prior=ORACLE_NORMAL)
    torch.cuda.synchronize()
    assert np.allclose(ch.phi.cpu().numpy(), phis, rtol=1e-12, atol=1e-12)
    p.close()


def test_da_first_stage_carries_the_prior_ratio():
    """Constant surrogate: stage 1 is the prior ratio alone, stage 2 the
    likelihood ratio; DA steps on a 32^2 FP64 problem agree with the
    oracle's DA step (decisions within 1e-6 of a tie are not compared)."""
    import torch
    from paper_1605_04718_amd.api import DA, ChainState
    need_gpu()
    steps = 6
    u0, v0 = inputs.initial_fields(32, 0.1, 0.9)
    uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    step = np.array([0.004, 0.004, 0.3, 0.3])
    from paper_1605_04718_amd.api import Grid, Problem
    p = Problem([Grid(n=32, u0=u0, v0=v0, y=y, sigma=sigma)], TAU, steps, 1e-12, precision=1,
                lo=LO, hi=HI, step=step, max_batch=64, **NORMAL)
    p.surrogate_create(64, 2, 8, seed=5)
    params = p.surrogate_params(0)
    params[-1] = (torch.zeros_like(params[-1][0]), torch.zeros_like(params[-1][1]))
    p.surrogate_params(1, params)
    p.surrogate_set_scaling(torch.ones(64, device="cuda"), torch.ones(64, device="cuda"), 0.1)
    C = 48
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (C, 1))
    phi0[:, 0] += np.linspace(-0.004, 0.004, C)
    th0 = torch.tensor(inputs.to_natural(phi0), device="cuda")
    ll0, _, _ = p.log_likelihood(th0)
    ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=29, da=True)
    ch.loglik_sur = p.surrogate_loglik(torch.tensor(phi0, device="cuda"))
    lls0 = ch.loglik_sur.cpu().numpy().copy()
    p.mcmc_step(ch, 1, mode=DA)
    torch.cuda.synchronize()
    ll0 = ll0.cpu().numpy()
    got_phi, acc1 = ch.phi.cpu().numpy(), ch.n_accept1.cpu().numpy()

    def ll(q):
        return float(oracle.loglik_batch(inputs.to_natural(q), u0, v0, y, sigma, TAU, steps,
                                         rtol=1e-12)[0][0])

    compared = rejected1 = 0
    for c in range(C):
        prop = osamp.propose(phi0[c], 29, c, 0, step, 0b1111)
        if osamp.in_support(prop, LO, HI, ORACLE_NORMAL):
            lu1 = math.log(oracle.uniform1(29, c, 0, osamp.PURPOSE_STAGE1))
            if lu1 < osamp.log_prior_ratio(phi0[c], prop, ORACLE_NORMAL):
                la2 = ll0[c] - ll(prop)
                if abs(math.log(oracle.uniform1(29, c, 0, osamp.PURPOSE_ACCEPT)) - la2) < 1e-6:
                    continue
        res = osamp.da_step(phi0[c], ll0[c], lls0[c], 29, c, 0, LO, HI, step, 0b1111, ll,
                            lambda q: lls0[c], prior=ORACLE_NORMAL)
        assert bool(acc1[c]) == res[3], c
        assert np.allclose(got_phi[c], res[0], rtol=1e-12, atol=1e-13), c
        rejected1 += not res[3]
        compared += 1
    assert compared > C - 4 and rejected1 > 0
    p.close()
