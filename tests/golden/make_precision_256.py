"""Writes tests/golden/precision_256.npz: FP64 oracle fields of 16 prior draws
on the 256 x 256 stationary unit square at T = 2 (dt 2.5e-4, 8000 IMEX
steps), the reference against which the FP32 path's error is stated at
256 x 256.  Per draw: u and v at CG rtol 1e-10 (float32), the oracle's own
difference between rtol 1e-7 (the FP32 workload's tolerance) and 1e-10,
which bounds what a solve stopped at rtol 1e-7 can agree to whatever its
arithmetic, and the amplification of a relative 6e-8 perturbation of the
initial fields (the size of an FP32 rounding) over the trajectory.

The draws are uniform on the prior box of the 4-parameter workload
(a, b in [0, 1], ln gamma in [ln 50, ln 500], ln d in [ln 5, ln 50]),
seed 6 of the shared input generators.

Calls only the oracle and the shared input generators:

    python tests/golden/make_precision_256.py   (about an hour on 6 cores)
"""
import math
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N, TAU, STEPS, M = 256, 2.5e-4, 8000, 16
RTOL, RTOL_FP32, EPS = 1e-10, 1e-7, 6e-8
THETA_TRUE = (0.1, 0.9, 200.0, 10.0)
LO = (0.0, 0.0, math.log(50.0), math.log(5.0))
HI = (1.0, 1.0, math.log(500.0), math.log(50.0))
MAXIT = 10 * N * N


def thetas(m=M):
    from paper_1605_04718_amd import inputs
    return inputs.to_natural(inputs.box_draws(m, LO, HI, seed=inputs.SEED_DATASET))


def solve(args):
    import oracle
    from paper_1605_04718_amd import inputs
    k, variant, steps = args
    th = thetas()[k]
    u0, v0 = inputs.initial_fields(N, THETA_TRUE[0], THETA_TRUE[1])
    t = time.time()
    if variant == 1:
        rng = np.random.default_rng(300 + k)
        u0 = u0 * (1.0 + EPS * rng.uniform(-1.0, 1.0, u0.shape))
        v0 = v0 * (1.0 + EPS * rng.uniform(-1.0, 1.0, v0.shape))
    rtol = RTOL_FP32 if variant == 2 else RTOL
    u, v, it, st = oracle.forward_solve(th, u0, v0, TAU, steps, rtol=rtol, maxit=MAXIT)
    print(f"draw {k} variant {variant}: {time.time() - t:.0f} s, status {st}, "
          f"iterations/step {it / steps}", flush=True)
    return u, v, it, st


def main():
    steps = int(os.environ.get("GOLDEN_STEPS", STEPS))
    m = int(os.environ.get("GOLDEN_M", M))
    jobs = [(k, v, steps) for v in (0, 2, 1) for k in range(m)]
    with Pool(int(os.environ.get("GOLDEN_PROCS", 6))) as pool:
        res = dict(zip([(k, v) for k, v, _ in jobs], pool.map(solve, jobs, chunksize=1)))
    u = np.stack([res[(k, 0)][0] for k in range(m)]).astype(np.float32)
    v = np.stack([res[(k, 0)][1] for k in range(m)]).astype(np.float32)
    status = np.array([res[(k, 0)][3] for k in range(m)])
    iters = np.stack([res[(k, 0)][2] for k in range(m)])

    def rel(k, j):
        if res[(k, j)][3] or res[(k, 0)][3]:
            return float("nan")
        du = np.linalg.norm(res[(k, j)][0] - res[(k, 0)][0]) / np.linalg.norm(res[(k, 0)][0])
        dv = np.linalg.norm(res[(k, j)][1] - res[(k, 0)][1]) / np.linalg.norm(res[(k, 0)][1])
        return max(du, dv)

    amp = np.array([rel(k, 1) / EPS for k in range(m)])
    cg_sens = np.array([rel(k, 2) for k in range(m)])
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "precision_256.npz")
    if steps != STEPS or m != M:
        path = path.replace(".npz", "_trial.npz")
    np.savez_compressed(path, theta=thetas(m), u=u, v=v, status=status, iters=iters,
                        amplification=amp, cg_sensitivity=cg_sens, n=N, tau=TAU, steps=steps,
                        rtol=RTOL, rtol_fp32=RTOL_FP32, eps=EPS)
    print(path, "status", status, "amplification", amp, "cg sensitivity", cg_sens)


if __name__ == "__main__":
    main()
