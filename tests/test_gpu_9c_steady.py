"""Steady-state stopping (Sec. 3.1.2) on the GPU solves against the oracle,
through the C ABI: resident (FP64, FP32), streamed (FP64) and cooperative
(FP32 256^2) tiles."""
import numpy as np
import pytest

import oracle
from gpu_common import TAU, need_gpu, rel_l2
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu

THETAS = np.array([(0.1, 0.9, 200.0, 1.0), (0.1, 0.9, 200.0, 10.0), (0.2, 0.7, 100.0, 2.0)])


def run(n, precision, tol, cap, thetas, rtol=None):
    import torch
    from paper_1605_04718_amd.api import Grid, Problem
    u0, v0 = inputs.initial_fields(n, 0.1, 0.9)
    rtol = rtol or (1e-12 if precision else 1e-7)
    p = Problem([Grid(n=n, u0=u0, v0=v0)], TAU, cap, rtol, precision=precision,
                max_batch=len(thetas), steady_tol=tol)
    th = torch.tensor(thetas, dtype=torch.float64, device="cuda")
    u, v, st, it, steps = p.forward_solve_steady(th)
    torch.cuda.synchronize()
    out = (u.double().cpu().numpy(), v.double().cpu().numpy(), st.cpu().numpy(),
           steps.cpu().numpy())
    p.close()
    return u0, v0, out


@pytest.mark.parametrize("n,precision,cap,tol,fields_tol", [
    (32, 1, 3000, 0.1, 1e-9),
    (64, 0, 3000, 0.1, 1e-5),
    (128, 1, 400, 0.1, 1e-9),  # FP64 at 128^2: the streamed tile
])
def test_stopping_step_and_fields_match_oracle(n, precision, cap, tol, fields_tol):
    need_gpu()
    thetas = THETAS if n <= 64 else THETAS[1:2]
    u0, v0, (u, v, st, steps) = run(n, precision, tol, cap, thetas)
    for k, th in enumerate(thetas):
        uo, vo, so, _, sto = oracle.forward_solve_steady(th, u0, v0, TAU, cap, tol, rtol=1e-12)
        assert sto == 0 and st[k] == 0, (k, st[k], sto)
        if precision == 1:
            assert steps[k] == so, (k, steps[k], so)
        else:
            # FP32 increments: the norm may cross the threshold one step apart
            assert abs(int(steps[k]) - so) <= 1, (k, steps[k], so)
            if steps[k] != so:
                continue
        assert rel_l2(u[k].reshape(n, n), uo) < fields_tol and rel_l2(v[k].reshape(n, n), vo) < fields_tol


def test_cooperative_tile_stops_with_the_oracle():
    need_gpu()
    n, cap, tol = 256, 200, 0.1
    thetas = THETAS[1:2]
    u0, v0, (u, v, st, steps) = run(n, 0, tol, cap, thetas)
    uo, vo, so, _, sto = oracle.forward_solve_steady(thetas[0], u0, v0, TAU, cap, tol, rtol=1e-12)
    assert sto == 0 and st[0] == 0 and abs(int(steps[0]) - so) <= 1, (steps[0], so)
    if steps[0] == so:
        assert rel_l2(u[0].reshape(n, n), uo) < 1e-5


def test_cap_reached_is_flagged_and_rejected():
    import torch
    from paper_1605_04718_amd.api import Grid, Problem
    need_gpu()
    n, cap = 32, 20
    u0, v0 = inputs.initial_fields(n, 0.1, 0.9)
    uo, _, _, _ = oracle.forward_solve((0.1, 0.9, 200.0, 10.0), u0, v0, TAU, cap, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    p = Problem([Grid(n=n, u0=u0, v0=v0, y=y, sigma=sigma)], TAU, cap, 1e-12, precision=1,
                max_batch=4, steady_tol=1e-9)
    th = torch.tensor(THETAS, dtype=torch.float64, device="cuda")
    _, _, st, _, steps = p.forward_solve_steady(th)
    phi, st2, _ = p.log_likelihood(th)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 32) and np.all(steps.cpu().numpy() == cap)
    assert np.all(np.isinf(phi.cpu().numpy())) and np.all(st2.cpu().numpy() == 32)
    p.close()


def test_fixed_horizon_reports_n_steps():
    need_gpu()
    _, _, (_, _, st, steps) = run(32, 1, 0.0, 15, THETAS)
    assert np.all(st == 0) and np.all(steps == 15)
