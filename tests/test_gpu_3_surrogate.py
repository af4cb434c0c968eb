"""Surrogate MLP (BF16 MFMA kernels) and delayed acceptance vs the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle
from oracle import mlp as omlp
from oracle import sampler as osamp
from gpu_common import THETA_TRUE, TAU, make_problem, need_gpu, rel_l2
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu

LO = np.array([0.0, 0.0, math.log(50.0), math.log(5.0)])
HI = np.array([1.0, 1.0, math.log(500.0), math.log(50.0)])


def small_problem(width=128, depth=2, out_side=8, n=32, steps=4, y=True, precision=0, step=None):
    u0, v0 = inputs.initial_fields(n, 0.1, 0.9)
    yy, sigma = None, 0.05
    if y:
        uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, steps, rtol=1e-12)
        yy, sigma = inputs.noisy_data(uo, 0.01)
    p, _, _ = make_problem(n, steps, precision=precision, y=yy, sigma=sigma, u0=u0, v0=v0, lo=LO,
                           hi=HI, step=step if step is not None else 0.02 * (HI - LO),
                           max_batch=256)
    p.surrogate_create(width, depth, out_side, seed=5)
    return p, u0, v0, yy, sigma


def host_params(p, dir=0):
    return [(W.double().cpu().numpy(), b.double().cpu().numpy()) for W, b in p.surrogate_params(dir)]


def test_forward_matches_oracle_with_the_same_weights():
    import torch
    need_gpu()
    p, *_ = small_problem()
    phi = inputs.box_draws(100, LO, HI, seed=12)  # ragged: padded to 128 rows inside
    out = p.surrogate_forward(torch.tensor(phi, device="cuda"), raw=True)
    torch.cuda.synchronize()
    params = host_params(p)
    want, _ = omlp.forward(params, omlp.scale_inputs(phi, LO, HI))
    assert out.shape == (100, 64)
    # BF16 weights and activations, FP32 accumulation
    assert rel_l2(out.cpu().numpy(), want) < 3e-2
    p.close()


def test_gradients_loss_and_adam_step_match_oracle():
    import torch
    need_gpu()
    p, *_ = small_problem()
    rng = np.random.default_rng(3)
    B = 192
    phi = inputs.box_draws(B, LO, HI, seed=13)
    target = rng.standard_normal((B, 64)).astype(np.float32)
    before = host_params(p)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    p.surrogate_train_step(torch.tensor(phi, device="cuda"), torch.tensor(target, device="cuda"),
                           1e-3, loss)
    torch.cuda.synchronize()
    grads = host_params(p, dir=2)
    after = host_params(p)
    y, cache = omlp.forward(before, omlp.scale_inputs(phi, LO, HI))
    want_loss, dy = omlp.mse(y, target.astype(np.float64))
    want_grads = omlp.backward(before, cache, dy)
    assert loss.item() == pytest.approx(want_loss, rel=2e-2)
    for (gW, gb), (wW, wb) in zip(grads, want_grads):
        assert rel_l2(gW, wW) < 5e-2 and rel_l2(gb, wb) < 5e-2
    # Adam (FP32 on the GPU) applied to the GPU's own gradients
    st = {}
    want_after = omlp.adam_step(before, grads, st, lr=1e-3)
    for (aW, ab), (wW, wb) in zip(after, want_after):
        assert np.abs(aW - wW).max() < 2e-6 and np.abs(ab - wb).max() < 2e-6
    p.close()


def test_training_reduces_the_loss_on_a_smooth_target():
    import torch
    need_gpu()
    p, *_ = small_problem(width=512, depth=4, out_side=8)
    rng = np.random.default_rng(4)
    B = 256
    phi_all = inputs.box_draws(2048, LO, HI, seed=14)
    x = omlp.scale_inputs(phi_all, LO, HI)
    freq = rng.standard_normal((4, 64))
    target_all = np.sin(x @ freq).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses = []
    for s in range(200):
        i = (s * B) % 2048
        p.surrogate_train_step(torch.tensor(phi_all[i:i + B], device="cuda"),
                               torch.tensor(target_all[i:i + B], device="cuda"), 1e-3, loss)
        losses.append(loss.item())
    torch.cuda.synchronize()
    assert np.mean(losses[-20:]) < 0.5 * np.mean(losses[:5])
    p.close()


def test_downsample_and_surrogate_misfit_match_oracle():
    import torch
    need_gpu()
    p, u0, v0, y, sigma = small_problem()
    rng = np.random.default_rng(5)
    u = torch.tensor(rng.standard_normal((3, 32, 32)).astype(np.float32), device="cuda")
    ds = p.downsample(u)
    mean = torch.tensor(rng.uniform(0.5, 1.5, 64).astype(np.float32), device="cuda")
    sd = torch.tensor(rng.uniform(0.1, 0.3, 64).astype(np.float32), device="cuda")
    p.surrogate_set_scaling(mean, sd, 0.07)
    phi = inputs.box_draws(10, LO, HI, seed=15)
    ll = p.surrogate_loglik(torch.tensor(phi, device="cuda"))
    torch.cuda.synchronize()
    want_ds = omlp.block_mean(u.double().cpu().numpy(), 8).reshape(3, 64)
    assert np.allclose(ds.cpu().numpy(), want_ds, rtol=1e-6, atol=1e-6)
    params = host_params(p)
    ybar = omlp.block_mean(y, 8).reshape(64)
    want = omlp.surrogate_misfit(params, phi, LO, HI, mean.double().cpu().numpy(),
                                 sd.double().cpu().numpy(), ybar, 0.07)
    assert np.allclose(ll.cpu().numpy(), want, rtol=3e-2)
    p.close()


def test_da_with_constant_surrogate_is_the_plain_chain():
    """Zero output layer -> Phi~ constant -> stage 1 always accepts and the
    delayed-acceptance chain equals the plain chain bit for bit."""
    import torch
    from paper_1605_04718_amd.api import DA, PLAIN, ChainState
    need_gpu()
    step = np.array([0.004, 0.004, 0.01, 0.01])
    p, u0, v0, y, sigma = small_problem(step=step, precision=1, steps=6)
    params = p.surrogate_params(0)
    params[-1] = (torch.zeros_like(params[-1][0]), torch.zeros_like(params[-1][1]))
    p.surrogate_params(1, params)
    p.surrogate_set_scaling(torch.ones(64, device="cuda"), torch.ones(64, device="cuda"), 0.1)
    C, S = 8, 5
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (C, 1))
    phi0[:, 1] += np.linspace(-0.01, 0.01, C)
    th0 = torch.tensor(inputs.to_natural(phi0), device="cuda")
    ll0, _, _ = p.log_likelihood(th0)
    runs = []
    for mode in (PLAIN, DA):
        ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=17,
                               trace_steps=S, da=True)
        ch.loglik_sur = p.surrogate_loglik(torch.tensor(phi0, device="cuda"))
        p.mcmc_step(ch, S, mode=mode)
        torch.cuda.synchronize()
        runs.append(ch)
    assert torch.equal(runs[0].trace, runs[1].trace)
    assert torch.equal(runs[1].n_accept1, runs[1].n_solves)  # stage 1 accepted every in-box proposal
    p.close()


def test_da_step_matches_oracle_decisions():
    """DA decisions vs the oracle's DA step on the same states, with the
    oracle evaluating the network in FP64 from the GPU's weights; decisions
    whose margin is below the BF16 error of Phi~ are not compared."""
    import torch
    from paper_1605_04718_amd.api import DA, ChainState
    need_gpu()
    step = np.array([0.01, 0.01, 0.02, 0.02])
    p, u0, v0, y, sigma = small_problem(step=step, precision=1, steps=6)
    p.surrogate_set_scaling(torch.full((64,), 1.0, device="cuda"),
                            torch.full((64,), 0.05, device="cuda"), 0.2)
    C = 64
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (C, 1))
    phi0[:, 0] += np.linspace(-0.02, 0.02, C)
    th0 = torch.tensor(inputs.to_natural(phi0), device="cuda")
    ll0, _, _ = p.log_likelihood(th0)
    ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=23, da=True)
    ch.loglik_sur = p.surrogate_loglik(torch.tensor(phi0, device="cuda"))
    lls0 = ch.loglik_sur.cpu().numpy().copy()
    p.mcmc_step(ch, 1, mode=DA)
    torch.cuda.synchronize()
    params = host_params(p)
    ybar = omlp.block_mean(y, 8).reshape(64)

    def sur(q):
        return float(omlp.surrogate_misfit(params, q, LO, HI, np.ones(64), np.full(64, 0.05), ybar,
                                           0.2)[0])

    def ll(q):
        return float(oracle.loglik_batch(inputs.to_natural(q), u0, v0, y, sigma, TAU, 6,
                                         rtol=1e-12)[0][0])

    got_phi = ch.phi.cpu().numpy()
    acc1 = ch.n_accept1.cpu().numpy()
    compared = 0
    for c in range(C):
        prop = osamp.propose(phi0[c], 23, c, 0, step, 0b1111)
        if not osamp.in_box(prop, LO, HI):
            continue
        s0, s1 = sur(phi0[c]), sur(prop)
        tol = 0.05 * (abs(s0) + abs(s1) + 1.0)  # BF16 error bound of Phi~ differences
        if abs(math.log(oracle.uniform1(23, c, 0, osamp.PURPOSE_STAGE1)) - (s0 - s1)) < tol:
            continue
        if math.log(oracle.uniform1(23, c, 0, osamp.PURPOSE_STAGE1)) < s0 - s1:
            la2 = (ll0[c].item() - ll(prop)) - (s0 - s1)
            if abs(math.log(oracle.uniform1(23, c, 0, osamp.PURPOSE_ACCEPT)) - la2) < tol:
                continue
        res = osamp.da_step(phi0[c], ll0[c].item(), lls0[c], 23, c, 0, LO, HI, step, 0b1111, ll, sur)
        assert bool(acc1[c]) == res[3]
        if res[3]:
            assert np.allclose(got_phi[c], res[0], rtol=1e-12, atol=1e-13)
        compared += 1
    assert compared > C // 2
    p.close()


def test_full_size_network_gradients_and_three_adam_steps_match_oracle():
    """The surrogate at its full size (4 -> 4 x 512 -> 32^2 outputs, GELU)
    and a batch of 1024: every hidden GEMM has K = 512 and the output layer
    N = 1024, so the K loop runs several 128-wide steps with the next step's
    tiles loaded during the current one.  Three consecutive training steps:
    loss and all gradients against the FP64 oracle at the GPU's weights
    before each step, and the weights after each step against the oracle's
    Adam, whose moment state carries over the three steps (bias correction
    at t = 1, 2, 3)."""
    import torch
    need_gpu()
    p, *_ = small_problem(width=512, depth=4, out_side=32, n=128, steps=1, y=False)
    rng = np.random.default_rng(7)
    B = 1024
    phi_all = inputs.box_draws(3 * B, LO, HI, seed=16)
    x = omlp.scale_inputs(phi_all, LO, HI)
    target_all = np.tanh(x @ rng.standard_normal((4, 1024))).astype(np.float32)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    st = {}
    assert [W.shape for W, _ in host_params(p)] == [(512, 4), (512, 512), (512, 512), (512, 512),
                                                    (1024, 512)]
    for t in range(3):
        phi = phi_all[t * B:(t + 1) * B]
        target = target_all[t * B:(t + 1) * B]
        before = host_params(p)
        print(f"full-size surrogate: training step {t + 1} of 3, batch {B}", flush=True)
        p.surrogate_train_step(torch.tensor(phi, device="cuda"),
                               torch.tensor(target, device="cuda"), 1e-3, loss)
        torch.cuda.synchronize()
        grads = host_params(p, dir=2)
        after = host_params(p)
        y, cache = omlp.forward(before, omlp.scale_inputs(phi, LO, HI))
        want_loss, dy = omlp.mse(y, target.astype(np.float64))
        want_grads = omlp.backward(before, cache, dy)
        assert loss.item() == pytest.approx(want_loss, rel=2e-2), (t, loss.item(), want_loss)
        for li, ((gW, gb), (wW, wb)) in enumerate(zip(grads, want_grads)):
            assert rel_l2(gW, wW) < 5e-2 and rel_l2(gb, wb) < 5e-2, (t, li, rel_l2(gW, wW),
                                                                     rel_l2(gb, wb))
        want_after = omlp.adam_step(before, grads, st, lr=1e-3)
        assert st["t"] == t + 1
        for (aW, ab), (wW, wb) in zip(after, want_after):
            assert np.abs(aW - wW).max() < 2e-6 and np.abs(ab - wb).max() < 2e-6, t
    p.close()


def _oracle_sur(p, y, mean, sd, sigma1, out_side=8):
    params = host_params(p)
    ybar = omlp.block_mean(y, out_side).reshape(-1)

    def sur(q):
        return float(omlp.surrogate_misfit(params, q, LO, HI, mean, sd, ybar, sigma1)[0])
    return sur


def test_surrogate_chain_with_constant_surrogate_replays_with_the_oracle():
    """Delayed acceptance with a four-substep surrogate chain, a constant
    Phi~ (zero output layer) and a normal prior on ln gamma: each substep's
    decision then rests on the prior ratio and the support alone (FP64 on
    both sides), so the GPU trace must follow the oracle's surrogate-chain
    step exactly, the oracle taking its own FP64 misfits of the proposals."""
    import torch
    from paper_1605_04718_amd.api import DA, ChainState, Grid, Problem
    need_gpu()
    n, steps, S, C, m = 32, 6, 4, 16, 4
    u0, v0 = inputs.initial_fields(n, 0.1, 0.9)
    uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    step = np.array([0.004, 0.004, 0.05, 0.01])
    prior = osamp.Prior(kinds=(0, 0, 1, 0), mean=(0, 0, math.log(200.0), 0), sd=(1, 1, 0.1, 1))
    p = Problem([Grid(n=n, u0=u0, v0=v0, y=y, sigma=sigma)], TAU, steps, 1e-12, precision=1,
                lo=LO, hi=HI, step=step, max_batch=64, prior_kind=prior.kinds,
                prior_mean=prior.mean, prior_sd=prior.sd)
    p.surrogate_create(128, 2, 8, seed=5)
    params = p.surrogate_params(0)
    params[-1] = (torch.zeros_like(params[-1][0]), torch.zeros_like(params[-1][1]))
    p.surrogate_params(1, params)
    p.surrogate_set_scaling(torch.ones(64, device="cuda"), torch.ones(64, device="cuda"), 0.1)
    p.set_da_substeps(m)
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (C, 1))
    phi0[:, 1] += np.linspace(-0.01, 0.01, C)
    ll0, _, _ = p.log_likelihood(torch.tensor(inputs.to_natural(phi0), device="cuda"))
    ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=29,
                           trace_steps=S, da=True)
    ch.loglik_sur = p.surrogate_loglik(torch.tensor(phi0, device="cuda"))
    sur0 = float(ch.loglik_sur[0].item())
    p.mcmc_step(ch, S, mode=DA)
    torch.cuda.synchronize()
    trace = ch.trace.cpu().numpy()
    acc1 = ch.n_accept1.cpu().numpy()

    def ll(q):
        return float(oracle.loglik_batch(inputs.to_natural(np.atleast_2d(q)), u0, v0, y, sigma,
                                         TAU, steps, rtol=1e-12)[0][0])

    ll0 = ll0.cpu().numpy()
    replayed = 0
    for c in range(C):
        cur, l, ls = phi0[c].copy(), float(ll0[c]), sur0
        moved = 0
        for s in range(S):
            cur, l, ls, m1, _, _ = osamp.da_chain_step(cur, l, ls, 29, c, s, m, LO, HI, step,
                                                       0b1111, ll, lambda q: sur0, prior=prior)
            moved += m1
            assert np.allclose(trace[s, c], cur, rtol=1e-12, atol=1e-13), (c, s, trace[s, c], cur)
        assert acc1[c] == moved
        replayed += 1
    assert replayed == C
    assert acc1.sum() > 0
    p.close()


def test_surrogate_chain_decisions_match_the_oracle():
    """A trained-looking (random-weight) surrogate and three substeps: each
    chain's surrogate chain is replayed with the oracle network evaluated in
    FP64 from the GPU's weights; chains where any decision lies within the
    BF16 error of Phi~ of its threshold are not compared."""
    import torch
    from paper_1605_04718_amd.api import DA, ChainState
    need_gpu()
    step = np.array([0.01, 0.01, 0.02, 0.02])
    m = 3
    p, u0, v0, y, sigma = small_problem(step=step, precision=1, steps=6)
    mean, sd, sigma1 = np.ones(64), np.full(64, 0.05), 0.2
    p.surrogate_set_scaling(torch.tensor(mean, dtype=torch.float32, device="cuda"),
                            torch.tensor(sd, dtype=torch.float32, device="cuda"), sigma1)
    p.set_da_substeps(m)
    C = 64
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (C, 1))
    phi0[:, 0] += np.linspace(-0.02, 0.02, C)
    ll0, _, _ = p.log_likelihood(torch.tensor(inputs.to_natural(phi0), device="cuda"))
    ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=31, da=True)
    ch.loglik_sur = p.surrogate_loglik(torch.tensor(phi0, device="cuda"))
    lls0 = ch.loglik_sur.cpu().numpy().copy()
    p.mcmc_step(ch, 1, mode=DA)
    torch.cuda.synchronize()
    sur = _oracle_sur(p, y, mean, sd, sigma1)

    def ll(q):
        return float(oracle.loglik_batch(inputs.to_natural(np.atleast_2d(q)), u0, v0, y, sigma,
                                         TAU, 6, rtol=1e-12)[0][0])

    got_phi = ch.phi.cpu().numpy()
    acc1 = ch.n_accept1.cpu().numpy()
    acc = ch.n_accept.cpu().numpy()
    ll0 = ll0.cpu().numpy()
    compared = 0
    for c in range(C):
        # the surrogate chain with margins: skip the chain if any decision is close
        z, lz, close, moves = phi0[c].copy(), sur(phi0[c]), False, 0
        for j in range(m):
            if j == 0:
                dz = oracle.normals4(31, c, 0, osamp.PURPOSE_PROPOSAL)
                u = oracle.uniform1(31, c, 0, osamp.PURPOSE_STAGE1)
            else:
                dz = oracle.normals4_at(31, c, 0, osamp.PURPOSE_SUB_PROPOSAL, 2 * j)
                u = oracle.uniform_at(31, c, 0, osamp.PURPOSE_SUB_ACCEPT, j)
            prop = osamp.rw_move(z, dz, step, 0b1111)
            if not osamp.in_box(prop, LO, HI):
                continue
            lp = sur(prop)
            tol = 0.05 * (abs(lz) + abs(lp) + 1.0)
            if abs(math.log(u) - (lz - lp)) < tol:
                close = True
                break
            if math.log(u) < lz - lp:
                z, lz, moves = prop, lp, moves + 1
        if close:
            continue
        if moves:
            la2 = (ll0[c] - ll(z)) - (sur(phi0[c]) - lz)
            if abs(math.log(oracle.uniform1(31, c, 0, osamp.PURPOSE_ACCEPT)) - la2) < \
                    0.05 * (abs(sur(phi0[c])) + abs(lz) + 1.0):
                continue
        res = osamp.da_chain_step(phi0[c], float(ll0[c]), float(lls0[c]), 31, c, 0, m, LO, HI,
                                  step, 0b1111, ll, sur)
        assert bool(acc1[c]) == res[3], c
        assert bool(acc[c]) == res[4], c
        assert np.allclose(got_phi[c], res[0], rtol=1e-12, atol=1e-13), c
        compared += 1
    assert compared > C // 3
    p.close()


def test_one_step_calls_replay_graphs_and_match_direct_launches():
    """With one Metropolis step per call on a created stream, the first call
    of a layout runs directly, the second captures, the rest replay; plain
    steps, one-proposal delayed acceptance and a three-substep surrogate
    chain must give the chains of direct launches on the null stream bit
    for bit."""
    import torch
    from paper_1605_04718_amd.api import DA, PLAIN, ChainState
    need_gpu()
    step = np.array([0.01, 0.01, 0.02, 0.02])
    p, u0, v0, y, sigma = small_problem(step=step, precision=1, steps=6)
    p.surrogate_set_scaling(torch.ones(64, device="cuda"), torch.full((64,), 0.05, device="cuda"),
                            0.2)
    C, S = 48, 5
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (C, 1))
    phi0[:, 0] += np.linspace(-0.02, 0.02, C)
    ll0, _, _ = p.log_likelihood(torch.tensor(inputs.to_natural(phi0), device="cuda"))
    lls0 = p.surrogate_loglik(torch.tensor(phi0, device="cuda"))
    torch.cuda.synchronize()

    def chains(da):
        ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=41,
                               trace_steps=S, da=da)
        if da:
            ch.loglik_sur = lls0.clone()
        return ch

    side = torch.cuda.Stream()
    for m, mode in ((1, PLAIN), (1, DA), (3, DA)):
        p.set_da_substeps(m)
        ref = chains(mode == DA)
        p.mcmc_step(ref, S, mode=mode)   # null stream: direct launches
        torch.cuda.synchronize()
        ch = chains(mode == DA)
        assert p.captured_graphs() == 0
        with torch.cuda.stream(side):
            for k in range(S):
                p.mcmc_step(ch, 1, mode=mode)
                side.synchronize()
                assert p.captured_graphs() == (0 if k == 0 else 1), (m, mode, k)
        assert torch.equal(ch.phi, ref.phi) and torch.equal(ch.loglik, ref.loglik), (m, mode)
        assert torch.equal(ch.trace, ref.trace) and torch.equal(ch.n_solves, ref.n_solves)
        if mode == DA:
            assert torch.equal(ch.loglik_sur, ref.loglik_sur)
    p.close()
