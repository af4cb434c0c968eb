"""Cooperative 256 x 256 FP32 tile (four workgroups per item, 64-row strips,
edge rows and CG sums exchanged through global memory) vs the FP64 oracle,
through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_common import THETA_TRUE, TAU, make_problem, need_gpu, rel_l2, theta_batch
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu

COOP_CPT = 16       # cells per thread of the cooperative tile at 256^2
STREAMED_CPT = 128  # the single-workgroup streamed tile


def run(p, thetas):
    import torch
    th = torch.tensor(np.asarray(thetas), dtype=torch.float64, device="cuda")
    u, v, st, it = p.forward_solve(th)
    torch.cuda.synchronize()
    return u.double().cpu().numpy(), v.double().cpu().numpy(), st.cpu().numpy(), it.cpu().numpy()


def test_coop_256_fields_and_misfit_match_oracle():
    """Several CG iterations per solve, the predictor from the second step
    on, and the group-summed misfit."""
    import torch
    need_gpu()
    steps = 6
    n = 256
    u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
    uo_true, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo_true, 0.01)
    thetas = np.vstack([THETA_TRUE, theta_batch(2, seed=41)])
    p, _, _ = make_problem(n, steps, precision=0, maxit=4000, y=y, sigma=sigma, u0=u0, v0=v0)
    p.set_tile(0, COOP_CPT)
    print(f"coop 256: {len(thetas)} items, {steps} steps", flush=True)
    ug, vg, st, it = run(p, thetas)
    phi, st2, _ = p.log_likelihood(torch.tensor(thetas, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    phi = phi.cpu().numpy()
    want, sto, _ = oracle.loglik_batch(thetas, u0, v0, y, sigma, TAU, steps, rtol=1e-12)
    for k, th in enumerate(thetas):
        uo, vo, ito, so = oracle.forward_solve(th, u0, v0, TAU, steps, rtol=1e-12)
        assert st[k] == 0 and so == 0 and int(st2[k]) == 0
        assert rel_l2(ug[k], uo) < 1e-5 and rel_l2(vg[k], vo) < 1e-5, (k, rel_l2(ug[k], uo),
                                                                        rel_l2(vg[k], vo))
        assert np.all(it[k] > 0)
        # misfit: sum of n^2 squared residuals of size ~sigma; the field
        # error (<= 1e-5 relative) moves it by far less than 1e-3 relative
        assert abs(phi[k] - want[k]) <= 1e-3 * abs(want[k]) + 1e-6, (phi[k], want[k])
    p.close()


def test_coop_256_growing_domain_matches_oracle():
    need_gpu()
    steps, rate = 5, 0.4
    thetas = np.vstack([THETA_TRUE, theta_batch(1, seed=43)])
    p, u0, v0 = make_problem(256, steps, precision=0, maxit=4000, growth=1, rate=rate)
    p.set_tile(0, COOP_CPT)
    print(f"coop 256 growing: {len(thetas)} items, {steps} steps", flush=True)
    ug, vg, st, it = run(p, thetas)
    for k, th in enumerate(thetas):
        uo, vo, ito, so = oracle.forward_solve(th, u0, v0, TAU, steps, growth=1, rate=rate,
                                               rtol=1e-12)
        assert st[k] == 0 and so == 0
        assert rel_l2(ug[k], uo) < 1e-5 and rel_l2(vg[k], vo) < 1e-5, (k, rel_l2(ug[k], uo))
    p.close()


def test_coop_256_more_items_than_groups():
    """Each group takes several items in turn; sampled items against the
    oracle, every item against the streamed single-workgroup tile."""
    need_gpu()
    steps, m = 2, 150
    thetas = theta_batch(m, seed=47)
    p, u0, v0 = make_problem(256, steps, precision=0, maxit=4000, max_batch=m)
    p.set_tile(0, COOP_CPT)
    print(f"coop 256: {m} items, {steps} steps", flush=True)
    ug, vg, st, _ = run(p, thetas)
    assert np.all(st == 0)
    for k in (0, 1, 70, m - 1):
        uo, vo, _, so = oracle.forward_solve(thetas[k], u0, v0, TAU, steps, rtol=1e-12)
        assert so == 0
        assert rel_l2(ug[k], uo) < 1e-5 and rel_l2(vg[k], vo) < 1e-5, (k, rel_l2(ug[k], uo))
    p.set_tile(0, STREAMED_CPT)
    print(f"streamed 256: {m} items, {steps} steps", flush=True)
    us, vs, ss, _ = run(p, thetas)
    assert np.all(ss == 0)
    for k in range(m):
        assert rel_l2(ug[k], us[k]) < 2e-5 and rel_l2(vg[k], vs[k]) < 2e-5, k
    p.close()


def test_coop_256_long_cg_runs_give_identical_bits_in_every_group():
    """Regression test for the group exchange: 32 copies of one stiff
    parameter vector (d = 30.5, gamma = 336: tens of CG iterations per step,
    so long runs of one-value exchanges) solved twice at rtol 1e-9.  Every
    group sums the same values in the same order, so all 64 results must be
    the same bits, every item must solve, and no group may give up a wait.
    A poll that took a stale partial sum (a slot whose 8-bit tag aliased an
    exchange 256 sequence numbers back) broke exactly this: the members of a
    group then diverged, giving wrong fields or a group time-out."""
    import torch
    need_gpu()
    steps, m = 2000, 32
    theta = np.tile([[0.0089, 0.979, 335.7, 30.5]], (m, 1))
    p, _, _ = make_problem(256, steps, precision=0, rtol=1e-9, maxit=4000, max_batch=m)
    p.set_tile(0, COOP_CPT)
    print(f"coop 256 stiff copies: {m} items, {steps} steps, twice", flush=True)
    u1, v1, st1, it1 = run(p, theta)
    u2, v2, st2, it2 = run(p, theta)
    assert np.all(st1 == 0) and np.all(st2 == 0), (st1, st2)
    assert p.check_solves() == 0
    assert it1[0, 1] > 20 * steps  # the long-CG regime this test is for
    for u, v, it in ((u1, v1, it1), (u2, v2, it2)):
        assert np.array_equal(u, np.broadcast_to(u1[0], u.shape))
        assert np.array_equal(v, np.broadcast_to(v1[0], v.shape))
        assert np.array_equal(it, np.broadcast_to(it1[0], it.shape))
    p.close()


def test_set_tile_rejects_unsupported():
    from paper_1605_04718_amd._lib import RDError
    need_gpu()
    p, _, _ = make_problem(256, 1, precision=1)
    with pytest.raises(RDError):
        p.set_tile(0, COOP_CPT)  # the cooperative tile is FP32 only
    with pytest.raises(RDError):
        p.set_tile(1, STREAMED_CPT)
    p.close()


def test_group_timeout_has_its_own_status_and_a_call_error():
    """Forced from the host: member 1 of every group sleeps 2 ms before the
    group's first exchange while the others wait at most 20 us, so every
    bounded wait gives up and every kernel still runs to its end.  Every
    256^2 item then carries RD_ST_GROUP_TIMEOUT (not the CG-cap bit), the
    count turns into RD_ETIMEOUT at rd_check_solves, and with the defaults
    restored the same batch solves."""
    from paper_1605_04718_amd._lib import RD_ETIMEOUT, ST_GROUP_TIMEOUT, RDError
    need_gpu()
    steps, m = 3, 12
    thetas = theta_batch(m, seed=53)
    p, _, _ = make_problem(256, steps, precision=0, maxit=4000, max_batch=m)
    p.set_tile(0, COOP_CPT)
    assert p.check_solves() == 0
    p.set_coop_wait(wait_ticks=2000, stall_ticks=200000)
    print(f"coop 256 forced group timeout: {m} items, {steps} steps", flush=True)
    _, _, st, _ = run(p, thetas)
    assert np.all(st == ST_GROUP_TIMEOUT), st
    with pytest.raises(RDError) as e:
        p.check_solves()
    assert e.value.code == RD_ETIMEOUT
    assert p.group_timeouts() == 0  # the failing check reset the count
    p.set_coop_wait(0, 0)
    print(f"coop 256 after restoring the wait: {m} items", flush=True)
    _, _, st, _ = run(p, thetas)
    assert np.all(st == 0), st
    assert p.check_solves() == 0
    p.close()


def test_group_timeout_in_the_fused_mixed_launch():
    """The same forced give-up inside one launch over 256^2 and 64^2 items:
    the 256^2 items carry RD_ST_GROUP_TIMEOUT, the 64^2 items (served by the
    same workgroups afterwards) solve normally."""
    import torch
    from paper_1605_04718_amd._lib import ST_GROUP_TIMEOUT
    from paper_1605_04718_amd.api import Grid, Problem
    need_gpu()
    steps = 3
    grids = []
    for n in (64, 256):
        u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
        grids.append(Grid(n=n, u0=u0, v0=v0, y=None, sigma=1.0))
    p = Problem(grids, TAU, steps, 1e-7, precision=0, cg_maxit=4000, max_batch=16)
    p.set_mixed_threads(1024)
    ids = np.array([0, 1] * 8, dtype=np.int32)
    thetas = theta_batch(len(ids), seed=59)
    th = torch.tensor(thetas, device="cuda")
    gid = torch.tensor(ids, device="cuda")
    p.set_coop_wait(wait_ticks=2000, stall_ticks=200000)
    print("fused mixed launch, forced group timeout: 8 x 64^2 + 8 x 256^2", flush=True)
    _, _, st, _ = p.forward_solve(th, grid_id=gid)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert np.all(st[ids == 1] == ST_GROUP_TIMEOUT), st
    assert np.all(st[ids == 0] == 0), st
    assert p.group_timeouts() > 0
    p.set_coop_wait(0, 0)
    _, _, st, _ = p.forward_solve(th, grid_id=gid)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    assert p.check_solves() == 0
    p.close()
