"""Uneven batches: several grid classes (sizes, stationary and growing
domains) served by one persistent launch, against the FP64 oracle and
against the single-class kernels."""
import numpy as np
import pytest

import oracle
from gpu_common import THETA_TRUE, TAU, need_gpu, rel_l2, theta_batch
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu

RATE = 0.01
# (n, growth) of the classes: 64, 128 and 256 cells per side, each
# stationary and growing as rho = exp(0.01 t)
CLASSES = [(64, 0), (64, 1), (128, 0), (128, 1), (256, 0), (256, 1)]


def classes_problem(n_steps, precision=0, data=False, max_batch=64):
    from paper_1605_04718_amd.api import Grid, Problem
    grids, fields = [], []
    for n, growth in CLASSES:
        u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
        y, sigma = None, 1.0
        if data:
            uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, n_steps, growth=growth,
                                               rate=RATE, rtol=1e-12)
            y, sigma = inputs.noisy_data(uo, 0.01)
        grids.append(Grid(n=n, u0=u0, v0=v0, y=y, sigma=sigma, growth=growth,
                          growth_rate=RATE if growth else 0.0))
        fields.append((u0, v0, y, sigma))
    p = Problem(grids, TAU, n_steps, 1e-12 if precision else 1e-7, precision=precision,
                max_batch=max_batch)
    return p, fields


def batch_ids(m, seed=5):
    """A shuffled batch covering every class (4:2:1 by size, as in the uneven workload)."""
    rng = np.random.default_rng(seed)
    ids = []
    for cls, (n, growth) in enumerate(CLASSES):
        ids += [cls] * {64: 4, 128: 2, 256: 1}[n]
    ids = np.array(ids * (m // len(ids) + 1))[:m]
    rng.shuffle(ids)
    return ids.astype(np.int32)


@pytest.mark.parametrize("threads", [1024, 512])
def test_mixed_batch_matches_oracle_per_class(threads):
    """1024 threads: one launch, 256^2 items by the cooperative role first;
    512: a cooperative launch, then the mixed launch for the other classes."""
    import torch
    need_gpu()
    steps = 5
    p, fields = classes_problem(steps)
    p.set_mixed_threads(threads)
    assert p.mixed_threads() == threads
    ids = batch_ids(14)
    thetas = np.vstack([THETA_TRUE, theta_batch(len(ids) - 1, seed=31)])
    th = torch.tensor(thetas, device="cuda")
    gid = torch.tensor(ids, device="cuda")
    u, v, st, it = p.forward_solve(th, grid_id=gid)
    torch.cuda.synchronize()
    u, v, st = u.double().cpu().numpy(), v.double().cpu().numpy(), st.cpu().numpy()
    assert u.shape == (len(ids), 256 * 256)
    for c, cls in enumerate(ids):
        n, growth = CLASSES[cls]
        u0, v0, _, _ = fields[cls]
        uo, vo, _, sto = oracle.forward_solve(thetas[c], u0, v0, TAU, steps, growth=growth,
                                              rate=RATE if growth else 0.0, rtol=1e-12)
        assert st[c] == 0 and sto == 0
        ug = u[c, :n * n].reshape(n, n)
        vg = v[c, :n * n].reshape(n, n)
        assert rel_l2(ug, uo) < 1e-5 and rel_l2(vg, vo) < 1e-5, (c, n, growth, rel_l2(ug, uo))
    p.close()


def test_mixed_batch_equals_single_class_launches():
    """The same items solved class by class (separate single-class problems)
    agree with the mixed launch to the FP32 solve accuracy (the strip
    layouts, and so the summation orders, may differ)."""
    import torch
    from paper_1605_04718_amd.api import Grid, Problem
    need_gpu()
    steps = 4
    p, fields = classes_problem(steps)
    ids = batch_ids(14, seed=8)
    thetas = theta_batch(len(ids), seed=32)
    u, _, st, _ = p.forward_solve(torch.tensor(thetas, device="cuda"),
                                  grid_id=torch.tensor(ids, device="cuda"))
    torch.cuda.synchronize()
    u = u.double().cpu().numpy()
    for cls, (n, growth) in enumerate(CLASSES):
        sel = np.nonzero(ids == cls)[0]
        if len(sel) == 0:
            continue
        u0, v0, _, _ = fields[cls]
        q = Problem([Grid(n=n, u0=u0, v0=v0, growth=growth, growth_rate=RATE if growth else 0.0)],
                    TAU, steps, 1e-7, max_batch=64)
        us, _, sts, _ = q.forward_solve(torch.tensor(thetas[sel], device="cuda"))
        torch.cuda.synchronize()
        us = us.double().cpu().numpy()
        for k, c in enumerate(sel):
            assert st[c] == 0 and int(sts[k]) == 0
            got = u[c, :n * n].reshape(n, n)
            assert rel_l2(got, us[k]) < 2e-6, (n, growth, rel_l2(got, us[k]))
        q.close()
    p.close()


def test_mixed_loglik_fused_misfit_and_bad_grid_ids():
    import torch
    need_gpu()
    steps = 3
    p, fields = classes_problem(steps, data=True)
    ids = batch_ids(10, seed=9)
    ids[3] = len(CLASSES)      # out of range: not solved
    ids[7] = -1
    thetas = theta_batch(len(ids), seed=33)
    phi, st, _ = p.log_likelihood(torch.tensor(thetas, device="cuda"),
                                  grid_id=torch.tensor(ids, device="cuda"))
    torch.cuda.synchronize()
    phi, st = phi.cpu().numpy(), st.cpu().numpy()
    for c, cls in enumerate(ids):
        if cls < 0 or cls >= len(CLASSES):
            assert st[c] == 16 and np.isinf(phi[c])
            continue
        n, growth = CLASSES[cls]
        u0, v0, y, sigma = fields[cls]
        want, sto, _ = oracle.loglik_batch(thetas[c:c + 1], u0, v0, y, sigma, TAU, steps,
                                           growth=growth, rate=RATE if growth else 0.0,
                                           rtol=1e-12)
        assert st[c] == 0 and sto[0] == 0
        assert abs(phi[c] - want[0]) <= 1e-4 * abs(want[0]) + 1e-6, (c, phi[c], want[0])
    p.close()


def test_mixed_fp64_matches_oracle():
    import torch
    need_gpu()
    steps = 3
    p, fields = classes_problem(steps, precision=1)
    ids = batch_ids(7, seed=10)
    thetas = theta_batch(len(ids), seed=34)
    u, _, st, _ = p.forward_solve(torch.tensor(thetas, device="cuda"),
                                  grid_id=torch.tensor(ids, device="cuda"))
    torch.cuda.synchronize()
    u, st = u.cpu().numpy(), st.cpu().numpy()
    for c, cls in enumerate(ids):
        n, growth = CLASSES[cls]
        u0, v0, _, _ = fields[cls]
        uo, _, _, _ = oracle.forward_solve(thetas[c], u0, v0, TAU, steps, growth=growth,
                                           rate=RATE if growth else 0.0, rtol=1e-12)
        assert st[c] == 0
        assert rel_l2(u[c, :n * n].reshape(n, n), uo) < 1e-10
    p.close()


def test_mixed_autotune_and_graph_step():
    """Autotuned workgroup size, then Metropolis steps over a mixed batch
    through the captured-graph path equal the same steps launched directly."""
    import torch
    from paper_1605_04718_amd.api import ChainState
    need_gpu()
    steps = 3
    p, fields = classes_problem(steps, data=True)
    p.autotune()
    assert p.mixed_threads() in (512, 1024)
    ids = torch.tensor(batch_ids(12, seed=11), device="cuda")
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (12, 1))
    phi0[:, 0] += np.linspace(-0.01, 0.01, 12)
    th0 = torch.tensor(inputs.to_natural(phi0), device="cuda")
    ll0, st0, _ = p.log_likelihood(th0, grid_id=ids)
    torch.cuda.synchronize()
    assert int(st0.abs().sum()) == 0
    runs = []
    for graphs in (False, True):
        ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=3,
                               trace_steps=3, grid_id=ids)
        torch.cuda.synchronize()
        if graphs:  # a created stream: the step is captured and replayed
            side = torch.cuda.Stream()
            with torch.cuda.stream(side):
                p.mcmc_step(ch, 3)
            side.synchronize()
        else:       # the null stream: direct launches
            p.mcmc_step(ch, 3)
        torch.cuda.synchronize()
        runs.append(ch)
    assert torch.equal(runs[0].trace, runs[1].trace)
    assert torch.equal(runs[0].loglik, runs[1].loglik)
    p.close()


def test_changing_the_launch_shape_drops_captured_steps():
    """A Metropolis step captured as a graph with 1024-thread workgroups is
    not replayed after the workgroup size (or a tile) changes: the setters
    drop every captured step, the next step on the stream is captured anew,
    and chains stepped through both shapes agree bit for bit with chains
    stepped directly with the same shapes."""
    import torch
    from paper_1605_04718_amd.api import ChainState
    need_gpu()
    steps = 3
    p, fields = classes_problem(steps, data=True)
    ids = torch.tensor(batch_ids(12, seed=13), device="cuda")
    phi0 = np.tile(inputs.to_sampling(THETA_TRUE)[0], (12, 1))
    phi0[:, 1] += np.linspace(-0.01, 0.01, 12)
    ll0, st0, _ = p.log_likelihood(torch.tensor(inputs.to_natural(phi0), device="cuda"),
                                   grid_id=ids)
    torch.cuda.synchronize()
    side = torch.cuda.Stream()
    ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=5,
                           trace_steps=4, grid_id=ids)
    p.set_mixed_threads(1024)
    assert p.captured_graphs() == 0
    with torch.cuda.stream(side):
        p.mcmc_step(ch, 2)       # the first step runs directly, the second is captured
    side.synchronize()
    assert p.captured_graphs() == 1
    p.set_mixed_threads(512)
    assert p.captured_graphs() == 0
    with torch.cuda.stream(side):
        p.mcmc_step(ch, 2)
    side.synchronize()
    assert p.captured_graphs() == 1
    p.set_tile(0, 16)
    assert p.captured_graphs() == 0
    # the same steps launched directly (null stream) with the same shapes
    ref = ChainState.create(torch.tensor(phi0, device="cuda"), ll0.clone(), seed=5,
                            trace_steps=4, grid_id=ids)
    p.set_mixed_threads(1024)
    p.mcmc_step(ref, 2)
    p.set_mixed_threads(512)
    p.mcmc_step(ref, 2)
    torch.cuda.synchronize()
    assert torch.equal(ch.trace, ref.trace)
    assert torch.equal(ch.loglik, ref.loglik)
    p.close()
