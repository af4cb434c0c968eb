"""GPU Metropolis kernels (Algorithm 1) vs the oracle sampler, through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from oracle import sampler as osamp
from gpu_common import THETA_TRUE, TAU, make_problem, need_gpu
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu

LO = np.array([0.0, 0.0, math.log(50.0), math.log(5.0)])
HI = np.array([1.0, 1.0, math.log(500.0), math.log(50.0)])
STEP = 0.02 * (HI - LO)


def chains_at(phi, ll, seed=11, trace_steps=0):
    import torch
    from paper_1605_04718_amd.api import ChainState
    return ChainState.create(torch.tensor(phi, dtype=torch.float64, device="cuda"),
                             torch.tensor(ll, dtype=torch.float64, device="cuda"), seed=seed,
                             trace_steps=trace_steps)


def test_proposals_match_oracle_stream():
    import torch
    need_gpu()
    C = 300
    p, _, _ = make_problem(16 * 2, 1, lo=LO, hi=HI, step=5 * STEP, max_batch=C)
    phi = inputs.box_draws(C, LO, HI, seed=8)
    ch = chains_at(phi, np.zeros(C), seed=123)
    ch.step = 987654321
    prop, inside = p.propose(ch)
    torch.cuda.synchronize()
    prop, inside = prop.cpu().numpy(), inside.cpu().numpy()
    for c in range(C):
        want = osamp.propose(phi[c], 123, c, 987654321, 5 * STEP, 0b1111)
        # Box-Muller through each side's log/cos/sin: agreement to a few ulp
        assert np.allclose(prop[c], want, rtol=1e-14, atol=1e-14)
        assert bool(inside[c]) == osamp.in_box(want, LO, HI)
    assert 0 < inside.sum() < C
    p.close()


def test_correlated_proposals_match_oracle_stream():
    """The proposal with a lower-triangular factor L (phi' = phi + L z)."""
    import torch
    from paper_1605_04718_amd.api import Grid, Problem
    need_gpu()
    C = 200
    L = np.array([[0.02, 0, 0, 0], [-0.01, 0.015, 0, 0], [0.003, 0.004, 0.05, 0],
                  [0.03, -0.02, 0.01, 0.04]])
    u0, v0 = inputs.initial_fields(32, 0.1, 0.9)
    p = Problem([Grid(n=32, u0=u0, v0=v0)], TAU, 1, 1e-7, lo=LO, hi=HI, free_mask=0b1011,
                max_batch=C, prop_chol=L)
    phi = inputs.box_draws(C, LO, HI, seed=9)
    ch = chains_at(phi, np.zeros(C), seed=77)
    ch.step = 12345
    prop, inside = p.propose(ch)
    torch.cuda.synchronize()
    prop, inside = prop.cpu().numpy(), inside.cpu().numpy()
    for c in range(C):
        want = osamp.propose(phi[c], 77, c, 12345, None, 0b1011, chol=L)
        assert np.allclose(prop[c], want, rtol=1e-14, atol=1e-14)
        assert prop[c][2] == phi[c][2]          # fixed coordinate untouched
        assert bool(inside[c]) == osamp.in_box(want, LO, HI)
    p.close()


def test_accept_decisions_match_oracle_bitwise():
    import torch
    need_gpu()
    C = 500
    p, _, _ = make_problem(32, 1, lo=LO, hi=HI, step=STEP, max_batch=C)
    rng = np.random.default_rng(4)
    phi = inputs.box_draws(C, LO, HI, seed=9)
    ll = rng.uniform(0, 5, C)
    ll[:10] = np.inf
    ch = chains_at(phi, ll, seed=77)
    ch.step = 42
    prop, inside = p.propose(ch)
    ll_prop = torch.tensor(rng.uniform(0, 5, C), dtype=torch.float64, device="cuda")
    ll_prop[10:20] = math.inf
    p.accept(ch, prop, inside, ll_prop)
    torch.cuda.synchronize()
    assert ch.step == 43
    prop_h, inside_h, llp = prop.cpu().numpy(), inside.cpu().numpy(), ll_prop.cpu().numpy()
    got_phi, got_ll = ch.phi.cpu().numpy(), ch.loglik.cpu().numpy()
    n_acc = ch.n_accept.cpu().numpy()
    for c in range(C):
        acc = False
        if inside_h[c]:
            u = oracle.uniform1(77, c, 42, osamp.PURPOSE_ACCEPT)
            acc = math.log(u) < ll[c] - llp[c]
        assert bool(n_acc[c]) == acc
        if acc:
            assert np.array_equal(got_phi[c], prop_h[c]) and got_ll[c] == llp[c]
        else:
            assert np.array_equal(got_phi[c], phi[c]) and (got_ll[c] == ll[c] or
                                                          (np.isinf(ll[c]) and np.isinf(got_ll[c])))
    p.close()


def test_gaussian_toy_chain_matches_oracle_chain():
    """Non-intrusive use: the GPU sampler on an external Phi follows the
    oracle's chain step for step."""
    import torch
    need_gpu()
    C, S = 64, 150
    mu = np.array([0.3, 0.6, 5.0, 2.5])
    sd = np.array([0.05, 0.08, 0.3, 0.2])
    lo, hi = np.array([0.0, 0.0, 3.0, 1.0]), np.array([1.0, 1.0, 7.0, 4.0])
    step = 1.2 * sd

    def phi_np(q):
        return 0.5 * (((np.atleast_2d(q) - mu) / sd) ** 2).sum(1)

    p, _, _ = make_problem(32, 1, lo=lo, hi=hi, step=step, max_batch=C)
    start = np.tile(mu, (C, 1))
    ch = chains_at(start, phi_np(start), seed=5)
    mu_t = torch.tensor(mu, device="cuda")
    sd_t = torch.tensor(sd, device="cuda")
    phis, lls = start.copy(), phi_np(start)
    for s in range(S):
        prop, inside = p.propose(ch)
        llp = 0.5 * (((prop - mu_t) / sd_t) ** 2).sum(1)
        p.accept(ch, prop, inside, llp.contiguous())
        phis, lls, _, _ = osamp.rwm_batch_step(phis, lls, 5, s, lo, hi, step, 0b1111, phi_np)
    torch.cuda.synchronize()
    assert np.allclose(ch.phi.cpu().numpy(), phis, rtol=1e-12, atol=1e-12)
    assert np.array_equal(ch.n_accept.cpu().numpy() > 0, np.any(phis != start, axis=1))
    p.close()


def _pde_chain_setup():
    n, steps, C = 32, 12, 6
    u0, v0 = inputs.initial_fields(n, 0.1, 0.9)
    uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    step = np.array([0.004, 0.004, 0.01, 0.01])
    p, _, _ = make_problem(n, steps, precision=1, y=y, sigma=sigma, u0=u0, v0=v0, lo=LO, hi=HI,
                           step=step, max_batch=C)
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (C, 1))
    phi0[:, 0] += np.linspace(-0.01, 0.01, C)

    def ll_fn(q):
        return oracle.loglik_batch(inputs.to_natural(q), u0, v0, y, sigma, TAU, steps, rtol=1e-12)[0]

    return p, phi0, ll_fn, step


def test_mcmc_step_on_pde_matches_oracle_chain():
    import torch
    need_gpu()
    S = 4
    p, phi0, ll_fn, step = _pde_chain_setup()
    ll0 = ll_fn(phi0)
    ch = chains_at(phi0, ll0, seed=31, trace_steps=S)
    p.solver_timing(enable=True, reset=True)
    p.mcmc_step(ch, S)  # null stream: direct launches
    torch.cuda.synchronize()
    ms, launches = p.solver_timing(enable=False)
    assert launches == S and ms > 0
    phis, lls = phi0.copy(), ll0.copy()
    trace = []
    for s in range(S):
        phis, lls, acc, _ = osamp.rwm_batch_step(phis, lls, 31, s, LO, HI, step, 0b1111, ll_fn)
        trace.append(phis.copy())
    assert np.allclose(ch.phi.cpu().numpy(), phis, rtol=1e-12, atol=1e-13)
    assert np.allclose(ch.loglik.cpu().numpy(), lls, rtol=1e-8)
    assert np.allclose(ch.trace.cpu().numpy(), np.stack(trace), rtol=1e-12, atol=1e-13)
    assert ch.step == S
    p.close()


def test_trace_rows_across_calls():
    """One call of S steps and S calls of one step fill the same trace rows."""
    import torch
    need_gpu()
    S = 3
    p, phi0, ll_fn, step = _pde_chain_setup()
    ll0 = ll_fn(phi0)
    a = chains_at(phi0, ll0, seed=5, trace_steps=S)
    p.mcmc_step(a, S)
    b = chains_at(phi0, ll0, seed=5, trace_steps=S)
    for _ in range(S):
        p.mcmc_step(b, 1)
    torch.cuda.synchronize()
    assert torch.equal(a.trace, b.trace) and torch.equal(a.phi, b.phi)
    assert torch.equal(b.trace[-1], b.phi)
    # a trace that ran out of rows is left alone (no write past its end)
    c = chains_at(phi0, ll0, seed=5, trace_steps=1)
    p.mcmc_step(c, 2)
    torch.cuda.synchronize()
    assert torch.equal(c.trace[0], a.trace[0])
    p.close()


def test_zz_graph_replay_matches_direct_launches():
    """mcmc_step_batch on a created stream replays a captured graph; the
    chain must equal the one from direct launches bit for bit."""
    import torch
    need_gpu()
    S = 4
    p, phi0, ll_fn, step = _pde_chain_setup()
    ll0 = ll_fn(phi0)
    ch2 = chains_at(phi0, ll0, seed=31, trace_steps=S)
    p.mcmc_step(ch2, S)  # direct launches on the null stream
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    ch = chains_at(phi0, ll0, seed=31, trace_steps=S)
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        p.mcmc_step(ch, S)
    side.synchronize()
    assert torch.equal(ch.phi, ch2.phi) and torch.equal(ch.loglik, ch2.loglik)
    assert torch.equal(ch.trace, ch2.trace)
    p.close()


def test_chain_counters_count_completed_steps_and_status_bits():
    """mcmc_step_batch's per-chain counters against the same proposals solved
    through forward_solve_steady_batch: solves, completed IMEX steps (a solve
    that stops at the CG cap in step s completed s) and one count per status
    bit.  With a CG cap of 3 iterations the proposals fail part way; with the
    default cap they complete."""
    import torch
    need_gpu()
    C, steps = 256, 60
    u0, v0 = inputs.initial_fields(32, 0.1, 0.9)
    uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    phi = inputs.box_draws(C, LO, HI, seed=31)
    for maxit in (3, 0):
        p, _, _ = make_problem(32, steps, y=y, sigma=sigma, u0=u0, v0=v0, lo=LO, hi=HI,
                               step=5 * STEP, max_batch=C, maxit=maxit)
        ch = chains_at(phi, np.full(C, np.inf), seed=17)
        prop, inside = p.propose(ch)
        th = torch.tensor(inputs.to_natural(prop.cpu().numpy()), device="cuda")
        _, _, st, _, nsteps = p.forward_solve_steady(th)
        p.mcmc_step(ch, 1)
        torch.cuda.synchronize()
        inside, st, nsteps = inside.cpu().numpy() != 0, st.cpu().numpy(), nsteps.cpu().numpy()
        failed = inside & (st != 0)
        if maxit == 3:
            assert failed.sum() > inside.sum() // 2
        else:
            assert failed.sum() < inside.sum() // 10
        assert np.all(nsteps[inside & (st == 0)] == steps)
        assert np.all(nsteps[failed] < steps)
        assert np.array_equal(ch.n_solves.cpu().numpy(), inside.astype(np.int64))
        assert np.array_equal(ch.imex_steps.cpu().numpy(), np.where(inside, nsteps, 0))
        fb = ch.fail_bits.cpu().numpy()
        for k in range(8):
            assert np.array_equal(fb[:, k], (inside & ((st >> k) & 1 == 1)).astype(np.int64)), k
        p.close()
