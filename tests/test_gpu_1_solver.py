"""GPU forward solve and misfit vs the FP64 oracle (through the C ABI)."""
import math

import numpy as np
import pytest

import oracle
from gpu_common import THETA_TRUE, TAU, make_problem, need_gpu, rel_l2, theta_batch
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu


def run_gpu(p, thetas):
    import torch
    th = torch.tensor(np.asarray(thetas), dtype=torch.float64, device="cuda")
    u, v, st, it = p.forward_solve(th)
    torch.cuda.synchronize()
    return u.double().cpu().numpy(), v.double().cpu().numpy(), st.cpu().numpy(), it.cpu().numpy()


def oracle_fields(thetas, u0, v0, n_steps, rtol=1e-12, growth=0, rate=0.0):
    out = []
    for th in thetas:
        u, v, it, st = oracle.forward_solve(th, u0, v0, TAU, n_steps, growth=growth, rate=rate,
                                            rtol=rtol)
        out.append((u, v, it, st))
    return out


@pytest.mark.parametrize("n,steps", [(32, 40), (64, 12)])
def test_fp64_resident_matches_oracle(n, steps):
    need_gpu()
    thetas = np.vstack([THETA_TRUE, theta_batch(3)])
    p, u0, v0 = make_problem(n, steps, precision=1)
    ug, vg, st, it = run_gpu(p, thetas)
    for k, (uo, vo, ito, sto) in enumerate(oracle_fields(thetas, u0, v0, steps)):
        assert st[k] == 0 and sto == 0
        assert rel_l2(ug[k], uo) < 1e-10 and rel_l2(vg[k], vo) < 1e-10, (k, rel_l2(ug[k], uo))
        # CG on the same systems; the GPU starts each solve from the
        # minimal-residual predictor, so it never needs more than one extra
        # iteration per solve and usually needs fewer
        assert np.all(it[k] <= ito + steps), (it[k], ito)
    p.close()


@pytest.mark.parametrize("n,steps", [(32, 30), (64, 20), (128, 10)])
def test_fp32_resident_matches_oracle(n, steps):
    need_gpu()
    thetas = np.vstack([THETA_TRUE, theta_batch(3, seed=5)])
    p, u0, v0 = make_problem(n, steps, precision=0, maxit=3000)
    ug, vg, st, it = run_gpu(p, thetas)
    for k, (uo, vo, ito, sto) in enumerate(oracle_fields(thetas, u0, v0, steps)):
        assert st[k] == 0
        # FP32 fields, FP64 dots; short horizon: the 1e-5 relative L2 bar
        assert rel_l2(ug[k], uo) < 1e-5 and rel_l2(vg[k], vo) < 1e-5, (k, rel_l2(ug[k], uo))
    p.close()


def test_fp64_streamed_128_matches_oracle():
    need_gpu()
    thetas = np.vstack([THETA_TRUE, theta_batch(1, seed=9)])
    p, u0, v0 = make_problem(128, 4, precision=1, maxit=3000)
    ug, vg, st, it = run_gpu(p, thetas)
    for k, (uo, vo, ito, sto) in enumerate(oracle_fields(thetas, u0, v0, 4)):
        assert st[k] == 0
        assert rel_l2(ug[k], uo) < 1e-10 and rel_l2(vg[k], vo) < 1e-10
    p.close()


def test_fp32_streamed_256_matches_oracle():
    need_gpu()
    thetas = np.vstack([THETA_TRUE])
    p, u0, v0 = make_problem(256, 3, precision=0, maxit=3000)
    p.set_tile(0, 128)  # the single-workgroup streamed tile (the default is cooperative)
    ug, vg, st, it = run_gpu(p, thetas)
    uo, vo, ito, sto = oracle_fields(thetas, u0, v0, 3)[0]
    assert st[0] == 0
    assert rel_l2(ug[0], uo) < 1e-5 and rel_l2(vg[0], vo) < 1e-5
    p.close()


@pytest.mark.parametrize("precision,tol", [(1, 1e-10), (0, 1e-5)])
def test_growing_domain_matches_oracle(precision, tol):
    need_gpu()
    n, steps, rate = 32, 30, 0.4
    thetas = np.vstack([THETA_TRUE, theta_batch(2, seed=3)])
    p, u0, v0 = make_problem(n, steps, precision=precision, growth=1, rate=rate)
    ug, vg, st, it = run_gpu(p, thetas)
    for k, (uo, vo, ito, sto) in enumerate(oracle_fields(thetas, u0, v0, steps, growth=1, rate=rate)):
        assert st[k] == 0
        assert rel_l2(ug[k], uo) < tol and rel_l2(vg[k], vo) < tol
    p.close()


def test_loglik_fused_misfit_and_field_misfit():
    import torch
    need_gpu()
    n, steps = 32, 25
    u0, v0 = inputs.initial_fields(n, 0.1, 0.9)
    uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    thetas = np.vstack([THETA_TRUE, theta_batch(4, seed=17)])
    p, _, _ = make_problem(n, steps, precision=1, y=y, sigma=sigma, u0=u0, v0=v0)
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    phi, st, it = p.log_likelihood(th)
    u, v, st2, it2 = p.forward_solve(th)
    phi_f = p.field_misfit(u)
    torch.cuda.synchronize()
    phi, u, phi_f = phi.cpu().numpy(), u.cpu().numpy(), phi_f.cpu().numpy()
    want, sto, _ = oracle.loglik_batch(thetas, u0, v0, y, sigma, TAU, steps, rtol=1e-12)
    for k in range(len(thetas)):
        # the misfit reduction alone (same field): FP64 rounding only
        assert phi[k] == pytest.approx(oracle.misfit(y, u[k], sigma), rel=1e-12)
        assert phi_f[k] == pytest.approx(oracle.misfit(y, u[k], sigma), rel=1e-12)
        # the whole chain: FP64 fields agree to ~1e-11, Phi to the same order
        assert phi[k] == pytest.approx(want[k], rel=1e-8, abs=1e-8)
    p.close()


def test_failure_flags_and_robust_phi():
    import torch
    need_gpu()
    n, steps = 32, 6
    u0, v0 = inputs.initial_fields(n, 0.1, 0.9)
    y = np.ones((n, n))
    # gamma tau u v > 1 + gamma tau -> sigma_u < 0: indefinite operator
    p, _, _ = make_problem(n, steps, precision=0, y=y, u0=u0, v0=v0)
    th = torch.tensor([[0.1, 0.9, 1e6, 10.0], list(THETA_TRUE)], dtype=torch.float64, device="cuda")
    phi, st, _ = p.log_likelihood(th)
    torch.cuda.synchronize()
    _, sto, _ = oracle.loglik_batch(th.cpu().numpy(), u0, v0, y, 0.05, TAU, steps, rtol=1e-7)
    assert st[0].item() & oracle.BREAKDOWN and sto[0] & oracle.BREAKDOWN
    assert math.isinf(phi[0].item()) and st[1].item() == 0 and math.isfinite(phi[1].item())
    p.close()
    # iteration cap
    p, _, _ = make_problem(n, steps, precision=0, y=y, u0=u0, v0=v0, maxit=1)
    phi, st, it = p.log_likelihood(th[1:])
    torch.cuda.synchronize()
    assert st[0].item() & oracle.NOT_CONVERGED and math.isinf(phi[0].item())
    p.close()
    # non-finite initial field
    u0b = u0.copy()
    u0b[3, 4] = np.nan
    p, _, _ = make_problem(n, steps, precision=0, y=y, u0=u0b, v0=v0)
    phi, st, it = p.log_likelihood(th[1:])
    torch.cuda.synchronize()
    assert st[0].item() & oracle.NONFINITE and math.isinf(phi[0].item())
    p.close()


def test_queue_ragged_batches_and_determinism():
    """More items than resident workgroups, a ragged count, n = 0, repeated theta."""
    import torch
    need_gpu()
    n, steps = 32, 8
    p, u0, v0 = make_problem(n, steps, precision=0, max_batch=3001)
    th = np.tile(np.asarray(THETA_TRUE), (3001, 1))
    th[1::2] = theta_batch(1500, seed=2)
    ug, vg, st, it = run_gpu(p, th)
    assert np.all(st == 0)
    # identical inputs give bit-identical outputs, whichever workgroup ran them
    assert np.all(ug[0::2] == ug[0])
    for k in (1, 777, 2999):
        uo, vo, _, _ = oracle.forward_solve(th[k], u0, v0, TAU, steps, rtol=1e-12)
        assert rel_l2(ug[k], uo) < 1e-5
    e = torch.zeros((0, 4), dtype=torch.float64, device="cuda")
    u, v, st0, _ = p.forward_solve(e)
    torch.cuda.synchronize()
    assert u.shape[0] == 0
    p.close()
