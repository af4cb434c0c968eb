"""The solve queue of a Metropolis step is ordered by per-chain cost
estimates kept in the problem handle.  The order decides only which
workgroup takes which item when, never what an item computes: the same
chains stepped on two problems whose estimates differ give identical
results, bit for bit."""
import math

import numpy as np
import pytest

from gpu_common import THETA_TRUE, make_problem, need_gpu
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu

LO = np.array([0.0, 0.0, math.log(50.0), math.log(5.0)])
HI = np.array([1.0, 1.0, math.log(500.0), math.log(50.0)])


def test_results_do_not_depend_on_the_queue_order():
    import torch
    import oracle
    from paper_1605_04718_amd.api import ChainState
    need_gpu()
    n, steps, C, S = 32, 40, 96, 3
    u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
    uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, 2.5e-4, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    kw = dict(y=y, sigma=sigma, u0=u0, v0=v0, lo=LO, hi=HI, step=0.05 * (HI - LO), max_batch=C)
    p1, _, _ = make_problem(n, steps, **kw)
    p2, _, _ = make_problem(n, steps, **kw)
    # p2's cost memory comes from other chains (other states, other seed)
    other = inputs.box_draws(C, LO, HI, seed=99)
    ll_o, _, _ = p2.log_likelihood(torch.tensor(inputs.to_natural(other), device="cuda"))
    warm = ChainState.create(torch.tensor(other, device="cuda"), ll_o.clone(), seed=5)
    p2.mcmc_step(warm, 4)
    phi = inputs.box_draws(C, LO, HI, seed=31)
    th = torch.tensor(inputs.to_natural(phi), device="cuda")
    ll1, _, _ = p1.log_likelihood(th)
    ll2, _, _ = p2.log_likelihood(th)
    torch.cuda.synchronize()
    assert torch.equal(ll1, ll2)
    a = ChainState.create(torch.tensor(phi, device="cuda"), ll1.clone(), seed=7, trace_steps=S)
    b = ChainState.create(torch.tensor(phi, device="cuda"), ll2.clone(), seed=7, trace_steps=S)
    for _ in range(S):
        p1.mcmc_step(a, 1)
        p2.mcmc_step(b, 1)
    torch.cuda.synchronize()
    assert torch.equal(a.trace, b.trace) and torch.equal(a.loglik, b.loglik)
    assert torch.equal(a.n_accept, b.n_accept) and torch.equal(a.cg_iters, b.cg_iters)
    assert int(a.n_accept.sum()) > 0
    p1.close()
    p2.close()


def test_delayed_acceptance_results_do_not_depend_on_the_queue_order():
    """The same with delayed acceptance, where only the first-stage accepts
    are solved: a constant-output surrogate makes stage 1 a uniform draw, so
    about half of the items are solved in each step."""
    import torch
    import oracle
    from paper_1605_04718_amd.api import DA, ChainState
    need_gpu()
    n, steps, C, S = 32, 40, 96, 3
    u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
    uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, 2.5e-4, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    kw = dict(y=y, sigma=sigma, u0=u0, v0=v0, lo=LO, hi=HI, step=0.05 * (HI - LO), max_batch=C)
    probs = []
    for k in range(2):
        p, _, _ = make_problem(n, steps, **kw)
        p.surrogate_create(64, 2, 8, seed=5)
        params = p.surrogate_params(0)
        params[-1] = (torch.zeros_like(params[-1][0]), torch.zeros_like(params[-1][1]))
        p.surrogate_params(1, params)
        p.surrogate_set_scaling(torch.ones(64, device="cuda"), torch.ones(64, device="cuda"), 0.1)
        probs.append(p)
    p1, p2 = probs
    other = inputs.box_draws(C, LO, HI, seed=98)
    ll_o, _, _ = p2.log_likelihood(torch.tensor(inputs.to_natural(other), device="cuda"))
    warm = ChainState.create(torch.tensor(other, device="cuda"), ll_o.clone(), seed=6, da=True)
    warm.loglik_sur = p2.surrogate_loglik(torch.tensor(other, device="cuda"))
    p2.mcmc_step(warm, 4, mode=DA)
    phi = inputs.box_draws(C, LO, HI, seed=32)
    th = torch.tensor(inputs.to_natural(phi), device="cuda")
    chains = []
    for p in (p1, p2):
        ll, _, _ = p.log_likelihood(th)
        ch = ChainState.create(torch.tensor(phi, device="cuda"), ll.clone(), seed=8, da=True,
                               trace_steps=S)
        ch.loglik_sur = p.surrogate_loglik(torch.tensor(phi, device="cuda"))
        chains.append(ch)
    a, b = chains
    for _ in range(S):
        p1.mcmc_step(a, 1, mode=DA)
        p2.mcmc_step(b, 1, mode=DA)
    torch.cuda.synchronize()
    assert torch.equal(a.trace, b.trace) and torch.equal(a.loglik, b.loglik)
    assert torch.equal(a.n_accept1, b.n_accept1) and torch.equal(a.n_solves, b.n_solves)
    assert torch.equal(a.cg_iters, b.cg_iters)
    assert 0 < int(a.n_solves.sum()) < C * S
    p1.close()
    p2.close()
