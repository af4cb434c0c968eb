"""Benchmark: batched plain Metropolis sampler on the 128x128 Schnakenberg problem.

One step = one Metropolis step (Algorithm 1) of every chain: proposal,
fused IMEX/CG forward solve + Gaussian misfit of every in-box proposal,
accept/reject.  Workload (the batched-plain-sampler configuration): 4096
chains, 128 x 128 cells, FP32 fields with FP64 reductions, four free
parameters (a, b, ln gamma, ln d) with a uniform prior box a, b in [0, 1],
gamma in [50, 500], d in [5, 50] (log-uniform), proposal s.d. 2 % of each
box side, T = 2, synthetic data from theta = (0.1, 0.9, 200, 10) with 1 %
Gaussian noise.  The time step is 2.5e-4 (8000 steps): at dt = 1e-3 the
Picard-linearised IMEX step is unstable for the homogeneous mode at this
theta (gamma dt above |f_u + g_v| / ((a+b)(2b-a)) = 0.118).

Prints one JSON line (metric: PDE cell-steps per second, plus ESS/s, the
roofline of the fused solve kernel and the FP64 CPU oracle baseline).
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
PEAK_FP32 = 157.3e12   # MI355X vector FP32 (packed); FLOP/s
# Algorithmic FP operations of the fused solve (per cell, per species):
#   one CG iteration: stencil q = sigma p + c sum(p - p_nb) (10), p.q (2),
#   r -= alpha q (2), r.r (2), x += alpha p (2), p = r + beta p (2) -> 20
#   one step's set-up: reaction diagonal (4), residual r0 (10), b and the two
#   norms (6) -> 20
FLOP_CG_ITER = 20.0
FLOP_SETUP = 20.0


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
                       f"rtol {CG_RTOL}; {dt:.1f} s wall; mean CG iters/step "
                       f"u {it[:, 0].mean() / n_steps_sample:.1f} v {it[:, 1].mean() / n_steps_sample:.1f}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--chains", type=int, default=4096)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-steps", type=int, default=2000)
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
    from paper_1605_04718_amd import inputs, stats
    from paper_1605_04718_amd.api import ChainState, Grid, Problem

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.device("cuda:0")
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
    th0 = torch.tensor(inputs.to_natural(phi0), dtype=torch.float64, device=dev)
    ll0, _, _ = p.log_likelihood(th0)
    total = args.warmup + args.steps
    ch = ChainState.create(torch.tensor(phi0, dtype=torch.float64, device=dev), ll0,
                           seed=inputs.SEED_SAMPLER, trace_steps=total)
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    log(f"setup done: {C} chains, {N_CELLS}^2, {n_steps} IMEX steps per solve")

    with torch.cuda.stream(stream):
        for k in range(args.warmup):
            t = time.time()
            p.mcmc_step(ch, 1)
            stream.synchronize()
            log(f"warmup step {k}: {time.time() - t:.2f} s")
        solves0 = int(ch.n_solves.sum())
        iters0 = ch.cg_iters.sum(0).cpu().numpy().astype(np.float64)
        acc0 = int(ch.n_accept.sum())
        p.solver_timing(enable=True, reset=True)
        torch.cuda.synchronize()
        t0 = time.time()
        for k in range(args.steps):
            p.mcmc_step(ch, 1)
            stream.synchronize()
            log(f"timed step {k}: {time.time() - t0:.2f} s elapsed")
        torch.cuda.synchronize()
        wall = time.time() - t0
    kern_ms, launches = p.solver_timing(enable=False)
    solves = int(ch.n_solves.sum()) - solves0
    iters = ch.cg_iters.sum(0).cpu().numpy().astype(np.float64) - iters0
    accepted = int(ch.n_accept.sum()) - acc0
    cells = N_CELLS * N_CELLS
    cell_steps = solves * cells * n_steps
    value = cell_steps / wall
    k_u = iters[0] / max(solves * n_steps, 1)
    k_v = iters[1] / max(solves * n_steps, 1)
    flops = cells * (2 * n_steps * solves * FLOP_SETUP + (iters[0] + iters[1]) * FLOP_CG_ITER)
    achieved = flops / (kern_ms / 1e3) if kern_ms > 0 else 0.0
    trace = ch.trace.cpu().numpy()
    summ = stats.summary(trace)
    ess_vals = [v["ess_bulk"] for v in summ.values()]
    ess_min = min(ess_vals) if all(math.isfinite(e) for e in ess_vals) else float("nan")
    line = {
        "metric": "PDE cell-steps/sec (plain batched Metropolis, 128x128); ESS/sec reported beside it",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 fields/CG vectors, f64 dots/misfit/accept",
        "data": "synthetic",
        "config": {"workload": "batched plain sampler: 4096 chains, 128x128, T=2 (dt 2.5e-4, 8000 "
                               "IMEX steps), 4 params, step 2% of prior range",
                   "chains": C, "grid": N_CELLS, "imex_steps": n_steps, "dt": TAU,
                   "cg_rtol": CG_RTOL, "cg_maxit": CG_MAXIT, "parallelism": "chains on one GPU"},
        "solves": solves,
        "accept_rate": accepted / max(C * args.steps, 1),
        "cg_iters_per_step": {"u": k_u, "v": k_v},
        "cell_cg_iters_per_s": cells * (iters[0] + iters[1]) / wall,
        "ess_per_sec": ess_min / wall if math.isfinite(ess_min) else None,
        "ess_note": f"min bulk-ESS over (a, b, ln gamma, ln d) of the {total}-step trace of "
                    f"{C} chains started from prior draws, over the timed wall time; "
                    f"min bulk-ESS = {ess_min:.1f}",
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32, "traffic": None,
                     "kernel": f"k_solve_resident<128,{cpt},float>",
                     "kernel_ms_per_launch": kern_ms / max(launches, 1),
                     "launches": launches},
    }
    if not args.no_cpu_baseline:
        threads = os.cpu_count() or 1
        threads = min(threads, 16)
        log(f"cpu baseline: oracle on {threads} threads")
        line["cpu_baseline"] = cpu_baseline(u0, v0, y, sigma, args.cpu_sample_steps, threads)
    print(json.dumps(line), flush=True)
    p.close()


if __name__ == "__main__":
    main()
