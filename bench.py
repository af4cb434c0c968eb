"""Benchmark: batched Metropolis on the 128x128 Schnakenberg problem, plain
and with a surrogate first stage (delayed acceptance).

One step = one Metropolis step (Algorithm 1) of every chain: proposal, fused
IMEX/CG forward solve + Gaussian misfit of every in-box proposal,
accept/reject.  Workload (the batched plain-sampler configuration): 4096
chains, 128 x 128 cells, FP32 fields with FP64 reductions, four free
parameters (a, b, ln gamma, ln d) with a uniform prior box a, b in [0, 1],
gamma in [50, 500], d in [5, 50] (log-uniform), proposal s.d. 2 % of each
box side, T = 2, synthetic data from theta = (0.1, 0.9, 200, 10) with 1 %
Gaussian noise, chains started from prior draws.  The time step is 2.5e-4
(8000 steps): at dt = 1e-3 the Picard-linearised IMEX step is unstable for
the homogeneous mode at this theta (gamma dt above
|f_u + g_v| / ((a+b)(2b-a)) = 0.118).

The delayed-acceptance leg trains the surrogate (BF16 MFMA MLP 4-512x4-1024)
on a bounded number of the library's own prior solves first, then runs the
same number of steps from the same chain states: every proposal is screened
by the surrogate and only stage-1 passes are solved.

The uneven leg (the `mixed` block, skipped with --no-mixed) runs 4095
chains split 4:2:1 over 64^2, 128^2 and 256^2 grids, half on growing
domains, in one launch per step.

Prints one JSON line: value = PDE cell-steps per second of the plain
sampler (solves actually performed), the roofline of the fused solve
kernel, the FP64 CPU oracle baseline, the delayed-acceptance figures
beside the plain ones, and the uneven leg.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_CELLS = 128
TAU = 2.5e-4
T_FINAL = 2.0
THETA_TRUE = (0.1, 0.9, 200.0, 10.0)
LO = (0.0, 0.0, math.log(50.0), math.log(5.0))
HI = (1.0, 1.0, math.log(500.0), math.log(50.0))
CG_RTOL = 1e-7
CG_MAXIT = 400
# The uneven workload's largest class (256^2) needs up to ~350 CG iterations
# per step in its first steps (d = 50); CG iteration counts grow about
# linearly with n, so its cap is four times the 128^2 one.
CG_MAXIT_MIXED = 1600
PEAK_FP32 = 157.3e12   # MI355X vector FP32 (packed); FLOP/s
PEAK_FP64 = 78.6e12    # MI355X vector FP64; FLOP/s
# Algorithmic FP operations of the fused solve (per cell, per species; a
# fused multiply-add counts 2):
#   one CG iteration: q = A p (5-point differences 7, c t + sigma p 3), the
#   two dot products of CG (4) and its three vector updates (6) -> 20; the
#   kernel's extra work (re-forming the diagonal, the third dot product that
#   saves a reduction) is not counted
#   one step's set-up: residual of the high part (14: differences 7,
#   diagonal 2, residual 2, right-hand side 1, its norm 2), of the low part
#   (14) and the compensated fold of the increment (10) -> 38 (the optional
#   predictor sweep is not counted)
FLOP_CG_ITER = 20.0
FLOP_SETUP = 38.0
# HBM bytes of the fused solve kernel from two rocprofv3 PMC passes over the
# timed step of `bench.py --steps 1 --warmup 0 --no-da --no-cpu-baseline
# --no-mixed` (3831 solves): FETCH_SIZE 3 501 785 479 KiB x 2.00 +
# WRITE_SIZE 7 460 049 918 KiB x 1.00 (factors from a 256 MiB copy), per
# solve-step.  Valid only for the kernel version and tile it was measured on
# (the one-pass residual of hi and lo; the queue order does not change what
# a solve reads or writes).
MEASURED_TRAFFIC = {"k_solve_resident<128,16,float>": 483253.3208332028}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(u0, v0, y, sigma, n_steps_sample, threads):
    """The FP64 oracle on a bounded sample of the same workload: `threads`
    solves (one per core, OpenMP) of the first n_steps_sample time steps."""
    import oracle
    os.environ.setdefault("OMP_NUM_THREADS", str(threads))
    rng = np.random.default_rng(6)
    phi = np.array(LO) + (np.array(HI) - np.array(LO)) * rng.uniform(size=(threads, 4))
    theta = np.concatenate([phi[:, :2], np.exp(phi[:, 2:])], axis=1)
    theta[0] = THETA_TRUE
    t0 = time.time()
    _, st, it = oracle.loglik_batch(theta, u0, v0, y, sigma, TAU, n_steps_sample, rtol=CG_RTOL,
                                    maxit=CG_MAXIT)
    dt = time.time() - t0
    cell_steps = threads * N_CELLS * N_CELLS * n_steps_sample
    return dict(value=cell_steps / dt, unit="cell-steps/s", cores=threads, kind="oracle",
                sample=f"{threads} prior draws (one per thread), first {n_steps_sample} of "
                       f"{int(round(T_FINAL / TAU))} IMEX steps at {N_CELLS}x{N_CELLS}, FP64, "
                       f"rtol {CG_RTOL}, start vector = previous level; {dt:.1f} s wall; mean "
                       f"CG iters/step u {it[:, 0].mean() / n_steps_sample:.1f} "
                       f"v {it[:, 1].mean() / n_steps_sample:.1f} (the early steps, where the "
                       f"fields move fastest, cost more iterations than the run average)")


def run_leg(p, ch, mode, warmup, steps, stream, name):
    """Warm-up then timed Metropolis steps; returns the leg's counters."""
    import torch
    with torch.cuda.stream(stream):
        for k in range(warmup):
            t = time.time()
            p.mcmc_step(ch, 1, mode=mode)
            stream.synchronize()
            log(f"{name} warmup step {k}: {time.time() - t:.2f} s")
        solves0 = int(ch.n_solves.sum())
        iters0 = ch.cg_iters.sum(0).cpu().numpy().astype(np.float64)
        acc0 = int(ch.n_accept.sum())
        acc10 = int(ch.n_accept1.sum())
        p.solver_timing(enable=True, reset=True)
        torch.cuda.synchronize()
        t0 = time.time()
        for k in range(steps):
            p.mcmc_step(ch, 1, mode=mode)
            stream.synchronize()
            log(f"{name} timed step {k}: {time.time() - t0:.2f} s elapsed")
        torch.cuda.synchronize()
        wall = time.time() - t0
    kern_ms, launches = p.solver_timing(enable=False)
    return dict(wall=wall, kern_ms=kern_ms, launches=launches,
                solves=int(ch.n_solves.sum()) - solves0,
                iters=ch.cg_iters.sum(0).cpu().numpy().astype(np.float64) - iters0,
                accepted=int(ch.n_accept.sum()) - acc0,
                accepted1=int(ch.n_accept1.sum()) - acc10)


def ess_block(trace, wall):
    from paper_1605_04718_amd import stats
    summ = stats.summary(trace)
    ess = [v["ess_bulk"] for v in summ.values()]
    rh = [v["rhat"] for v in summ.values()]
    ok = all(math.isfinite(e) for e in ess)
    return {"min_bulk_ess": min(ess) if ok else None,
            "max_rhat": max(rh) if all(math.isfinite(r) for r in rh) else None,
            "ess_per_sec": (min(ess) / wall) if ok and wall > 0 else None,
            "draws_per_chain": int(trace.shape[0])}


def laplace_hessian(Problem, Grid, inputs, u0, v0, y, sigma, rtol, h=3e-4):
    """Central-difference Hessian of Phi at the data-generating parameters
    (33 misfits in one batched launch): the Laplace approximation the
    stationary leg sizes its proposal and warm start with."""
    import itertools
    import torch
    n_steps = int(round(T_FINAL / TAU))
    p = Problem([Grid(n=N_CELLS, u0=u0, v0=v0, y=y, sigma=sigma)], TAU, n_steps, rtol,
                cg_maxit=2000, lo=LO, hi=HI, max_batch=64)
    c = inputs.to_sampling(THETA_TRUE)[0]
    pts = [c.copy()]
    for i in range(4):
        for s in (1, -1):
            q = c.copy()
            q[i] += s * h
            pts.append(q)
    pairs = list(itertools.combinations(range(4), 2))
    for i, j in pairs:
        for si, sj in ((1, 1), (1, -1), (-1, 1), (-1, -1)):
            q = c.copy()
            q[i] += si * h
            q[j] += sj * h
            pts.append(q)
    ll, st, _ = p.log_likelihood(torch.tensor(inputs.to_natural(np.array(pts)), device="cuda"))
    torch.cuda.synchronize()
    ll = ll.cpu().numpy()
    p.close()
    H = np.zeros((4, 4))
    for i in range(4):
        H[i, i] = (ll[1 + 2 * i] - 2 * ll[0] + ll[2 + 2 * i]) / h ** 2
    for k, (i, j) in enumerate(pairs):
        fpp, fpm, fmp, fmm = ll[9 + 4 * k: 13 + 4 * k]
        H[i, j] = H[j, i] = (fpp - fpm - fmp + fmm) / (4 * h * h)
    return c, H, float(ll[0])


def stationary_leg(args, u0, v0, y, sigma, log):
    """Plain vs delayed acceptance near stationarity: proposal and warm start
    from the Laplace approximation, CG tolerance tight enough to resolve the
    posterior, surrogate trained on draws around it."""
    import torch
    from paper_1605_04718_amd import inputs, surrogate
    from paper_1605_04718_amd.api import DA, PLAIN, ChainState, Grid, Problem
    n_steps = int(round(T_FINAL / TAU))
    C, S, rtol = args.st_chains, args.st_steps, args.st_rtol
    c, H, phi_c = laplace_hessian(Problem, Grid, inputs, u0, v0, y, sigma, rtol)
    ev = np.linalg.eigvalsh(H)
    if not ev.min() > 0:
        raise RuntimeError(f"Laplace Hessian not positive definite: {ev}")
    cov = np.linalg.inv(H)
    msd = np.sqrt(np.diag(cov))
    Lc = np.linalg.cholesky(cov)
    Lp = np.linalg.cholesky((2.38 ** 2 / 4.0) * cov)   # optimal random-walk scale, d = 4
    rng = np.random.default_rng(7)
    phi0 = c + rng.standard_normal((C, 4)) @ Lc.T
    log(f"stationary: Laplace marginal s.d. {msd}, Phi(theta_true) {phi_c:.1f}")
    p = Problem([Grid(n=N_CELLS, u0=u0, v0=v0, y=y, sigma=sigma)], TAU, n_steps, rtol,
                cg_maxit=2000, lo=LO, hi=HI, max_batch=max(C, 4096), prop_chol=Lp)
    p.autotune()
    phi0_t = torch.tensor(phi0, dtype=torch.float64, device="cuda")
    ll0, st0, _ = p.log_likelihood(torch.tensor(inputs.to_natural(phi0), device="cuda"))
    torch.cuda.synchronize()
    stream = torch.cuda.Stream()
    ch = ChainState.create(phi0_t.clone(), ll0.clone(), seed=inputs.SEED_SAMPLER + 10,
                           trace_steps=S)
    plain = run_leg(p, ch, PLAIN, 0, S, stream, "stationary plain")
    tr_p = ch.trace.cpu().numpy()
    # local surrogate: inputs mapped over +-8 posterior s.d., trained on draws
    # spread three times wider than the Laplace approximation
    p.surrogate_create(512, 4, 32, seed=inputs.SEED_SURROGATE_INIT)
    p.surrogate_set_input_box(c - 8 * msd, c + 8 * msd)
    draws = c + 3.0 * np.random.default_rng(8).standard_normal((args.st_sur_solves, 4)) @ Lc.T
    draws = np.clip(draws, c - 8 * msd, c + 8 * msd)
    t0 = time.time()
    rep = surrogate.fit(p, sigma, LO, HI, len(draws), args.st_sur_epochs, log=log, phi=draws)
    fit_s = time.time() - t0
    lls0 = p.surrogate_loglik(phi0_t)
    torch.cuda.synchronize()
    chd = ChainState.create(phi0_t.clone(), ll0.clone(), seed=inputs.SEED_SAMPLER + 10,
                            trace_steps=S, da=True)
    chd.loglik_sur = lls0.clone()
    da = run_leg(p, chd, DA, 0, S, stream, "stationary da")
    tr_d = chd.trace.cpu().numpy()
    pmh = None
    if args.st_pmh > 0:
        # Algorithm 2 from the same warm start: N proposals per chain and
        # step (around an auxiliary point), N draws; as many draws per chain
        # as the other samplers' steps
        N = args.st_pmh
        K = max(1, S // N)
        chp = ChainState.create(phi0_t.clone(), ll0.clone(), seed=inputs.SEED_SAMPLER + 10,
                                trace_steps=K * N)
        solves0 = int(chp.n_solves.sum())
        torch.cuda.synchronize()
        t = time.time()
        with torch.cuda.stream(stream):
            for k in range(K):
                p.pmh_step(chp, N)
                stream.synchronize()
                log(f"stationary pmh step {k} ({N} proposals per chain): {time.time() - t:.1f} s")
        pmh = {"wall": time.time() - t, "solves": int(chp.n_solves.sum()) - solves0,
               "moved": int(chp.n_accept.sum()), "draws": K * N, "steps": K, "n_prop": N}
        tr_m = chp.trace.cpu().numpy()
    p.close()
    burn = S // 2
    from paper_1605_04718_amd import stats
    sp, sd_ = stats.summary(tr_p[burn:]), stats.summary(tr_d[burn:])
    agree = {}
    names = list(sp.keys())
    for i, k in enumerate(names):
        se = math.hypot(sp[k]["mcse_mean"], sd_[k]["mcse_mean"])
        row = {"mean_plain": sp[k]["mean"], "mean_da": sd_[k]["mean"],
               "mean_diff_in_mcse": abs(sp[k]["mean"] - sd_[k]["mean"]) / se if se > 0 else None}
        xp, xd = tr_p[burn:, :, i].T, tr_d[burn:, :, i].T
        for q, nm in ((0.025, "q025"), (0.975, "q975")):
            qp, qd = float(np.quantile(xp, q)), float(np.quantile(xd, q))
            sq = math.hypot(stats.mcse_quantile(xp, q), stats.mcse_quantile(xd, q))
            row[f"{nm}_plain"], row[f"{nm}_da"] = qp, qd
            row[f"{nm}_diff_in_mcse"] = abs(qp - qd) / sq if sq > 0 else None
        agree[k] = row
    ep, ed = ess_block(tr_p[burn:], plain["wall"]), ess_block(tr_d[burn:], da["wall"])
    pmh_block = None
    if pmh is not None:
        mb = pmh["draws"] // 2
        sm = stats.summary(tr_m[mb:])
        for i, k in enumerate(names):
            se = math.hypot(sp[k]["mcse_mean"], sm[k]["mcse_mean"])
            agree[k]["mean_pmh"] = sm[k]["mean"]
            agree[k]["mean_diff_pmh_in_mcse"] = (abs(sp[k]["mean"] - sm[k]["mean"]) / se
                                                  if se > 0 else None)
        em = ess_block(tr_m[mb:], pmh["wall"])
        pmh_block = {"wall_s": pmh["wall"], "n_prop": pmh["n_prop"], "steps": pmh["steps"],
                     "draws_per_chain": pmh["draws"], "solves": pmh["solves"],
                     "moved_fraction": pmh["moved"] / (C * pmh["draws"]), **em,
                     "ess_per_solve": (em["min_bulk_ess"] / pmh["solves"]
                                       if em["min_bulk_ess"] else None)}
    return {
        "workload": f"{C} chains x {S} steps (second half kept), 128x128, T=2, CG rtol {rtol}, "
                    "correlated random walk with the Laplace covariance x 2.38^2/4, warm start "
                    "from the Laplace approximation at the data-generating parameters",
        "laplace_marginal_sd": msd.tolist(),
        "plain": {"wall_s": plain["wall"], "accept_rate": plain["accepted"] / (C * S),
                  "solves": plain["solves"], **ep,
                  "ess_per_solve": (ep["min_bulk_ess"] / plain["solves"]
                                    if ep["min_bulk_ess"] else None)},
        "da": {"wall_s": da["wall"], "accept_rate": da["accepted"] / (C * S),
               "stage1_accept_rate": da["accepted1"] / (C * S), "solves": da["solves"],
               "surrogate_held_out": rep["held_out"], "surrogate_fit_s": fit_s, **ed,
               "ess_per_solve": (ed["min_bulk_ess"] / da["solves"]
                                 if ed["min_bulk_ess"] else None)},
        "ess_per_sec_speedup": (ed["ess_per_sec"] / ep["ess_per_sec"]
                                if ed["ess_per_sec"] and ep["ess_per_sec"] else None),
        "da_ess_per_sec_incl_surrogate_fit": (ed["min_bulk_ess"] / (da["wall"] + fit_s)
                                              if ed["min_bulk_ess"] else None),
        "posterior_mean_agreement": agree,
        "pmh": pmh_block,
    }


def mixed_leg(args, log):
    """The uneven workload: chains split 4:2:1 over 64^2, 128^2 and 256^2
    grids, half on stationary and half on growing domains (rho = e^{0.01 t}),
    six datasets; per step one launch (1024-thread workgroups: groups of four
    solve the 256^2 items, then join the other classes) or two (512: a
    cooperative launch, then the mixed one), replayed from a captured graph;
    wall-clock cell-steps/s of the solves performed."""
    import torch
    from paper_1605_04718_amd import inputs
    from paper_1605_04718_amd.api import ChainState, Grid, Problem
    n_steps = int(round(T_FINAL / TAU))
    classes = [(64, 0), (64, 1), (128, 0), (128, 1), (256, 0), (256, 1)]
    counts = {n: max(2, int(round(c * args.mixed_scale)))
              for n, c in ((64, 2340), (128, 1170), (256, 585))}
    grids = []
    for n, growth in classes:
        u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
        grids.append((n, growth, u0, v0))
    # data: each class's own noise-free field at theta_true from the library
    gen = Problem([Grid(n=n, u0=u0, v0=v0, growth=g, growth_rate=0.01 if g else 0.0)
                   for n, g, u0, v0 in grids], TAU, n_steps, CG_RTOL, cg_maxit=CG_MAXIT_MIXED,
                  max_batch=len(classes))
    th = torch.tensor([THETA_TRUE] * len(classes), dtype=torch.float64, device="cuda")
    gid = torch.arange(len(classes), dtype=torch.int32, device="cuda")
    log("mixed: data solves (one per class)")
    ut, _, st, _ = gen.forward_solve(th, grid_id=gid)
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    gen.close()
    gl = []
    for k, (n, g, u0, v0) in enumerate(grids):
        y, sigma = inputs.noisy_data(ut[k, :n * n].double().cpu().numpy().reshape(n, n), 0.01,
                                     seed=100 + k)
        gl.append(Grid(n=n, u0=u0, v0=v0, y=y, sigma=sigma, growth=g,
                       growth_rate=0.01 if g else 0.0))
    ids = []
    for k, (n, g, _, _) in enumerate(grids):
        ids += [k] * (counts[n] // 2 + (counts[n] % 2 if g == 0 else 0))
    C = len(ids)
    ids = torch.tensor(np.array(ids, dtype=np.int32), device="cuda")
    step = tuple(0.02 * (h - l) for l, h in zip(LO, HI))
    p = Problem(gl, TAU, n_steps, CG_RTOL, cg_maxit=CG_MAXIT_MIXED, lo=LO, hi=HI, step=step,
                max_batch=C)
    p.autotune()
    T = p.mixed_threads()
    log(f"mixed: autotuned workgroup {T} threads; initial misfits of {C} chains")
    phi0 = inputs.box_draws(C, LO, HI, seed=inputs.SEED_CHAIN_INIT)
    ll0, st0, _ = p.log_likelihood(torch.tensor(inputs.to_natural(phi0), device="cuda"),
                                   grid_id=ids)
    torch.cuda.synchronize()
    st0 = st0.cpu().numpy()
    idn0 = ids.cpu().numpy()
    failed0 = {f"{n}{'g' if g else 's'}": int((st0[idn0 == k] != 0).sum())
               for k, (n, g, _, _) in enumerate(grids)}
    log(f"mixed: initial misfits done; failed solves per class {failed0}")
    ch = ChainState.create(torch.tensor(phi0, device="cuda"), ll0, seed=inputs.SEED_SAMPLER,
                           grid_id=ids)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        # warm-up: the first step of a new layout runs directly, the second is
        # captured; the timed steps are graph replays
        t = time.time()
        p.mcmc_step(ch, 2)
        stream.synchronize()
        log(f"mixed warmup (2 steps, the second captured): {time.time() - t:.1f} s")
        per_class0 = ch.n_solves.cpu().numpy().copy()
        t0 = time.time()
        for k in range(args.mixed_steps):
            p.mcmc_step(ch, 1)
            stream.synchronize()
            log(f"mixed timed step {k}: {time.time() - t0:.1f} s elapsed")
        wall = time.time() - t0
    solves = ch.n_solves.cpu().numpy() - per_class0
    idn = ids.cpu().numpy()
    cell_steps = 0.0
    per = {}
    for k, (n, g, _, _) in enumerate(grids):
        sk = int(solves[idn == k].sum())
        per[f"{n}{'g' if g else 's'}"] = sk
        cell_steps += sk * n * n * n_steps
    p.close()
    log(f"mixed: {C} chains, workgroup {T} threads, {args.mixed_steps} steps in {wall:.2f} s")
    return {"workload": f"{C} chains: {counts[64]} x 64^2, {counts[128]} x 128^2, "
                        f"{counts[256]} x 256^2 (the 4:2:1 mix at {args.mixed_scale:g} of 4095 "
                        "chains), half stationary and half growing (rho = exp(0.01 t)), 6 datasets, "
                        "T=2, " + ("one launch per step (256^2 items by groups of four "
                                   "workgroups, then the other classes)" if T == 1024 else
                                   "per step a cooperative launch for the 256^2 items and a "
                                   "persistent launch for the rest") +
                        ", replayed from a captured graph",
            "cell_steps_per_s": cell_steps / wall, "ms_per_step": 1e3 * wall / args.mixed_steps,
            "steps": args.mixed_steps,
            "mixed_threads": T, "solves_per_class": per, "cg_maxit": CG_MAXIT_MIXED,
            "initial_failed_solves_per_class": failed0}


def precision_256_leg(args, log):
    """FP32 against FP64 at 256^2: 16 prior draws solved to T = 2 on the
    stationary domain by the FP32 path (cooperative tile, rtol 1e-7) and by
    the FP64 path (streamed tile, rtol 1e-10); relative L2 of the final u
    and v fields.  The FP64 reference runs in chunks of steps, each
    restarting from the previous chunk's FP64 fields (exact on a stationary
    domain: a step depends only on the current fields), as two 8-class
    problems per chunk (one class per draw)."""
    import torch
    from paper_1605_04718_amd import inputs
    from paper_1605_04718_amd.api import Grid, Problem
    n, m = 256, 16
    n_steps = int(round(T_FINAL / TAU))
    chunk = args.p256_chunk
    u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
    phi = inputs.box_draws(m, LO, HI, seed=inputs.SEED_DATASET)
    th = torch.tensor(inputs.to_natural(phi), dtype=torch.float64, device="cuda")
    p32 = Problem([Grid(n=n, u0=u0, v0=v0)], TAU, n_steps, CG_RTOL, cg_maxit=CG_MAXIT_MIXED,
                  max_batch=m)
    torch.cuda.synchronize()
    t = time.time()
    u32, v32, st32, _ = p32.forward_solve(th)
    torch.cuda.synchronize()
    t32 = time.time() - t
    u32 = u32.double().cpu().numpy().reshape(m, -1)
    v32 = v32.double().cpu().numpy().reshape(m, -1)
    st32 = st32.cpu().numpy()
    p32.close()
    log(f"precision 256: FP32 path {t32:.1f} s")
    U = [u0.ravel().copy() for _ in range(m)]
    V = [v0.ravel().copy() for _ in range(m)]
    st64 = np.zeros(m, dtype=np.int64)
    t = time.time()
    for c0 in range(0, n_steps, chunk):
        steps = min(chunk, n_steps - c0)
        for h0 in range(0, m, 8):
            ks = list(range(h0, min(h0 + 8, m)))
            grids = [Grid(n=n, u0=U[k].reshape(n, n), v0=V[k].reshape(n, n)) for k in ks]
            p = Problem(grids, TAU, steps, 1e-10, precision=1, max_batch=len(ks))
            gid = torch.arange(len(ks), dtype=torch.int32, device="cuda")
            u, v, st, _ = p.forward_solve(th[ks[0]:ks[-1] + 1].contiguous(), grid_id=gid)
            torch.cuda.synchronize()
            u = u.cpu().numpy().reshape(len(ks), -1)
            v = v.cpu().numpy().reshape(len(ks), -1)
            st = st.cpu().numpy()
            for j, k in enumerate(ks):
                U[k], V[k] = u[j, :n * n].copy(), v[j, :n * n].copy()
                st64[k] |= int(st[j])
            p.close()
            log(f"precision 256: FP64 reference draws {ks[0]}-{ks[-1]}, {c0 + steps}/{n_steps} "
                f"steps, {time.time() - t:.1f} s")
    t64 = time.time() - t
    ok = [k for k in range(m) if st32[k] == 0 and st64[k] == 0]

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))

    eu = [rel(u32[k, :n * n], U[k]) for k in ok]
    ev = [rel(v32[k, :n * n], V[k]) for k in ok]
    return {
        "workload": f"{m} prior draws, 256x256, stationary, T=2 ({n_steps} steps of 2.5e-4): "
                    "FP32 path (compensated fields, cooperative tile, CG rtol 1e-7) against FP64 "
                    f"(streamed tile, CG rtol 1e-10, {chunk}-step chunks)",
        "solved_both": len(ok), "failed_fp32": int((st32 != 0).sum()),
        "failed_fp64": int((st64 != 0).sum()),
        "rel_l2_u": {"median": float(np.median(eu)), "max": float(np.max(eu)),
                     "per_draw": eu},
        "rel_l2_v": {"median": float(np.median(ev)), "max": float(np.max(ev)),
                     "per_draw": ev},
        "fp32_seconds": t32, "fp64_seconds": t64,
    }


def growth1d_leg(args, log):
    """Example 1's one-dimensional growing domain: n = 100 cells, tau = 1e-4,
    the fused float64 solve + misfit of g1d_log_likelihood_batch for
    `--g1d-items` prior draws of the three growth coefficients over
    `--g1d-steps` IMEX steps (the paper's horizon T = 600 is 6e6 steps; the
    timed horizon is shorter and the full-horizon time is extrapolated).
    Data: the exponential-growth solution of the same horizon plus 5 %
    noise.  FLOPs are the kernel's issued float64 operations (a reciprocal
    counted as one): per padded row and reduction level 14, per row and
    step 13 more for assembly and the final solve; 128 rows x 2 systems,
    6 exchange levels at n = 100 (the seventh is a lane-local 2 x 2 solve)."""
    import torch
    from paper_1605_04718_amd import inputs
    from paper_1605_04718_amd.api import Growth1D
    n, tau, steps, m = 100, 1e-4, args.g1d_steps, args.g1d_items
    theta = (0.1, 0.9, 1000.0, 10.0)
    u0, v0 = inputs.initial_fields_1d(n)
    gdata = Growth1D(n, steps, tau, theta, u0, v0, law=Growth1D.EXP, max_batch=1)
    ud, vd, _ = gdata.forward(None, m=1)
    gdata.close()
    y, sigma = inputs.noisy_data(np.stack([ud[0].cpu().numpy(), vd[0].cpu().numpy()]), 0.05,
                                 seed=inputs.SEED_DATA_NOISE)
    rho_T = math.exp(0.001 * steps * tau)
    g = Growth1D(n, steps, tau, theta, u0, v0, rho_T=rho_T, y=y, obs=3, sigma=sigma,
                 max_batch=m)
    beta = torch.tensor(inputs.box_draws(m, (-0.2, -0.2, -0.2), (0.4, 0.2, 0.2),
                                         seed=inputs.SEED_DATASET), device="cuda")
    phi, st = g.log_likelihood(beta[:64].contiguous())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    phi, st = g.log_likelihood(beta)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    g.close()
    levels = 6 if n > 64 else math.ceil(math.log2(n))
    flops = m * steps * 2 * 128 * (14 * levels + 13)
    achieved = flops / (ms * 1e-3)
    full_steps = int(round(600 / tau))
    log(f"growth1d: {m} items x {steps} steps in {ms:.1f} ms")
    return {
        "workload": f"Example 1, n={n}, tau={tau}, {m} items x {steps} steps (fused solve + misfit)",
        "ms": ms, "item_steps_per_s": m * steps / (ms * 1e-3),
        "cell_steps_per_s": m * steps * n / (ms * 1e-3),
        "solved": int((st == 0).sum().item()),
        "full_horizon_seconds_per_batch": ms * 1e-3 * full_steps / steps,
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64, "traffic": None,
                     "kernel": "k_g1d_solve", "flops_per_launch": flops},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=8)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=2000)
    ap.add_argument("--no-da", action="store_true", help="skip the delayed-acceptance leg")
    ap.add_argument("--sur-solves", type=int, default=16384,
                    help="prior solves the surrogate is trained on in the DA leg")
    ap.add_argument("--sur-epochs", type=int, default=40)
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the uneven 64/128/256 workload (the `mixed` block)")
    ap.add_argument("--mixed", action="store_true",
                    help="(default) run the uneven workload; kept for older command lines")
    ap.add_argument("--mixed-steps", type=int, default=1,
                    help="timed steps of the uneven workload")
    ap.add_argument("--mixed-scale", type=float, default=1.0,
                    help="fraction of the 4095 chains of the uneven workload")
    ap.add_argument("--precision-256", action="store_true",
                    help="also compare the FP32 and FP64 paths at 256^2 (16 prior draws, T = 2)")
    ap.add_argument("--p256-chunk", type=int, default=1000,
                    help="steps per FP64 reference call of --precision-256")
    ap.add_argument("--stationary", action="store_true",
                    help="also run plain vs delayed acceptance near stationarity (ESS/s)")
    ap.add_argument("--st-chains", type=int, default=1024)
    ap.add_argument("--st-steps", type=int, default=40)
    ap.add_argument("--st-rtol", type=float, default=1e-9)
    ap.add_argument("--st-sur-solves", type=int, default=8192)
    ap.add_argument("--st-sur-epochs", type=int, default=60)
    ap.add_argument("--growth1d", action="store_true",
                    help="also time Example 1's 1-D growing-domain likelihood")
    ap.add_argument("--growth1d-only", action="store_true",
                    help="run only the 1-D leg and print its JSON object")
    ap.add_argument("--g1d-items", type=int, default=4096)
    ap.add_argument("--g1d-steps", type=int, default=20000)
    ap.add_argument("--st-pmh", type=int, default=0, metavar="N",
                    help="also run Algorithm 2 (N proposals per chain and step) near stationarity")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="first copy MIB MiB device-to-device (a known-size kernel that scales "
                         "hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU: the chains are independent and shard across GPUs "
              f"without communication, so --gpus {args.gpus} is not measured here.",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1605_04718_amd import inputs
    from paper_1605_04718_amd.api import DA, PLAIN, ChainState, Grid, Problem

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
    if args.growth1d_only:
        torch.cuda.set_device(0)
        print(json.dumps({"growth1d": growth1d_leg(args, log)}), flush=True)
        return
    if args.copy_calibration:
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {nbytes} bytes read and written once")
        del src, dst
    n_steps = int(round(T_FINAL / TAU))
    C = args.chains
    step = tuple(0.02 * (h - l) for l, h in zip(LO, HI))

    # synthetic data: noise-free field at theta_true from the library + 1 % noise
    u0, v0 = inputs.initial_fields(N_CELLS, THETA_TRUE[0], THETA_TRUE[1])
    gen = Problem([Grid(n=N_CELLS, u0=u0, v0=v0)], TAU, n_steps, CG_RTOL, cg_maxit=CG_MAXIT,
                  max_batch=1)
    u_true, _, st, _ = gen.forward_solve(torch.tensor([THETA_TRUE], dtype=torch.float64, device=dev))
    torch.cuda.synchronize()
    assert int(st[0]) == 0
    y, sigma = inputs.noisy_data(u_true[0].double().cpu().numpy(), 0.01)
    gen.close()

    p = Problem([Grid(n=N_CELLS, u0=u0, v0=v0, y=y, sigma=sigma)], TAU, n_steps, CG_RTOL,
                cg_maxit=CG_MAXIT, lo=LO, hi=HI, step=step, max_batch=C)
    cpt = p.autotune()[0]
    log(f"autotuned tile: {cpt} cells per thread ({N_CELLS * N_CELLS // cpt} threads)")
    phi0 = inputs.box_draws(C, LO, HI, seed=inputs.SEED_CHAIN_INIT)
    phi0_t = torch.tensor(phi0, dtype=torch.float64, device=dev)
    th0 = torch.tensor(inputs.to_natural(phi0), dtype=torch.float64, device=dev)
    ll0, _, _ = p.log_likelihood(th0)
    total = args.warmup + args.steps
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    log(f"setup done: {C} chains, {N_CELLS}^2, {n_steps} IMEX steps per solve")

    ch = ChainState.create(phi0_t.clone(), ll0.clone(), seed=inputs.SEED_SAMPLER,
                           trace_steps=total)
    plain = run_leg(p, ch, PLAIN, args.warmup, args.steps, stream, "plain")
    plain_trace = ch.trace.cpu().numpy()

    cells = N_CELLS * N_CELLS
    wall = plain["wall"]
    solves = plain["solves"]
    iters = plain["iters"]
    value = solves * cells * n_steps / wall
    k_u = iters[0] / max(solves * n_steps, 1)
    k_v = iters[1] / max(solves * n_steps, 1)
    kern_ms = plain["kern_ms"]
    flops = cells * (2 * n_steps * solves * FLOP_SETUP + (iters[0] + iters[1]) * FLOP_CG_ITER)
    achieved = flops / (kern_ms / 1e3) if kern_ms > 0 else 0.0
    ess_plain = ess_block(plain_trace, wall)
    kernel = f"k_solve_resident<128,{cpt},float>"
    launches = max(plain["launches"], 1)
    traffic_per_launch = (MEASURED_TRAFFIC[kernel] * solves * n_steps / launches
                          if kernel in MEASURED_TRAFFIC else None)
    line = {
        "metric": "PDE cell-steps/sec (plain batched Metropolis, 128x128); ESS/sec and the "
                  "surrogate delayed-acceptance figures reported beside it",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fields (compensated hi+lo) and CG vectors; f64 dots, misfit, accept",
        "data": "synthetic",
        "config": {"workload": "batched plain sampler: 4096 chains, 128x128, T=2 (dt 2.5e-4, 8000 "
                               "IMEX steps), 4 params, step 2% of prior range, chains from prior "
                               "draws",
                   "chains": C, "grid": N_CELLS, "imex_steps": n_steps, "dt": TAU,
                   "cg_rtol": CG_RTOL, "cg_maxit": CG_MAXIT, "parallelism": "chains on one GPU"},
        "solves": solves,
        "accept_rate": plain["accepted"] / max(C * args.steps, 1),
        "mh_steps_per_s": C * args.steps / wall,
        "cg_iters_per_step": {"u": k_u, "v": k_v},
        "cell_cg_iters_per_s": cells * (iters[0] + iters[1]) / wall,
        "ess": {"plain": ess_plain,
                "note": "bulk-ESS (min over a, b, ln gamma, ln d) and split-R-hat of the "
                        f"{total}-step traces of chains started from prior draws: a transient, "
                        "not a stationary estimate; ESS/s = min ESS / timed wall time"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
                     "traffic": traffic_per_launch,
                     "traffic_unit": "bytes per launch (PMC FETCH_SIZE + WRITE_SIZE, scaled by "
                                     "the measured per-solve-step figure of this kernel)",
                     "kernel": kernel,
                     "kernel_ms_per_launch": kern_ms / max(plain["launches"], 1),
                     "launches": plain["launches"],
                     "flops_per_launch": flops / max(plain["launches"], 1)},
    }

    if not args.no_da:
        from paper_1605_04718_amd import surrogate
        p.surrogate_create(512, 4, 32, seed=inputs.SEED_SURROGATE_INIT)
        t0 = time.time()
        rep = surrogate.fit(p, sigma, LO, HI, args.sur_solves, args.sur_epochs, log=log)
        fit_s = time.time() - t0
        rep.pop("loss_history", None)
        lls0 = p.surrogate_loglik(phi0_t)
        torch.cuda.synchronize()
        chd = ChainState.create(phi0_t.clone(), ll0.clone(), seed=inputs.SEED_SAMPLER,
                                trace_steps=total, da=True)
        chd.loglik_sur = lls0.clone()
        da = run_leg(p, chd, DA, args.warmup, args.steps, stream, "da")
        da_trace = chd.trace.cpu().numpy()
        dwall = da["wall"]
        line["da"] = {
            "cell_steps_per_s": da["solves"] * cells * n_steps / dwall,
            "ms_per_step": 1e3 * dwall / args.steps,
            "mh_steps_per_s": C * args.steps / dwall,
            "mh_steps_speedup_vs_plain": (C * args.steps / dwall) / (C * args.steps / wall),
            "solves": da["solves"],
            "solves_per_chain_step": da["solves"] / (C * args.steps),
            "plain_solves_per_chain_step": solves / (C * args.steps),
            "stage1_accept_rate": da["accepted1"] / max(C * args.steps, 1),
            "accept_rate": da["accepted"] / max(C * args.steps, 1),
            "surrogate": {k: rep[k] for k in ("solves", "dropped", "outliers", "dataset_seconds",
                                              "train_samples", "epochs", "train_seconds",
                                              "train_tflops", "final_train_mse", "held_out",
                                              "sigma1")},
            "surrogate_fit_seconds": fit_s,
        }
        line["ess"]["da"] = ess_block(da_trace, dwall)

    if not args.no_mixed:
        line["mixed"] = mixed_leg(args, log)
    if args.precision_256:
        line["precision_256"] = precision_256_leg(args, log)
    if args.stationary:
        line["stationary"] = stationary_leg(args, u0, v0, y, sigma, log)
    if args.growth1d:
        line["growth1d"] = growth1d_leg(args, log)

    if not args.no_cpu_baseline:
        threads = os.cpu_count() or 1
        threads = min(threads, 16)
        log(f"cpu baseline: oracle on {threads} threads")
        line["cpu_baseline"] = cpu_baseline(u0, v0, y, sigma, args.cpu_sample_steps, threads)
    print(json.dumps(line), flush=True)
    p.close()


if __name__ == "__main__":
    main()
