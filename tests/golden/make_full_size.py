"""Writes tests/golden/full_size_128.npz: FP64 oracle fields of the 128 x 128
workload at T = 2 (dt 2.5e-4, 8000 IMEX steps, CG rtol 1e-12) for three
parameter vectors, plus two sensitivities of each trajectory from which the
GPU tests derive their FP32 tolerance: to a relative 6e-8 perturbation of
the initial fields (the size of an FP32 rounding), and to the CG tolerance
of the FP32 workload (the oracle at rtol 1e-7 against rtol 1e-12): a solve
stopped at rtol 1e-7 is only defined to within that difference.

Calls only the oracle and the shared input generators:

    python tests/golden/make_full_size.py     (about a minute on 8 cores)
"""
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

N, TAU, STEPS, RTOL, EPS, RTOL_FP32 = 128, 2.5e-4, 8000, 1e-12, 6e-8, 1e-7
THETAS = np.array([
    [0.1, 0.9, 200.0, 10.0],                # the data-generating parameters: Turing pattern
    [0.135, 0.721, 167.619, 10.214],        # a pattern-forming prior draw
    [0.813, 0.913, 202.118, 26.82],         # a prior draw outside the Turing space: decays
])


def solve(args):
    import oracle
    from paper_1605_04718_amd import inputs
    k, perturb = args
    u0, v0 = inputs.initial_fields(N, 0.1, 0.9)
    if perturb == 2:
        return oracle.forward_solve(THETAS[k], u0, v0, TAU, STEPS, rtol=RTOL_FP32)
    if perturb:
        rng = np.random.default_rng(100 + k)
        u0 = u0 * (1.0 + EPS * rng.uniform(-1.0, 1.0, u0.shape))
        v0 = v0 * (1.0 + EPS * rng.uniform(-1.0, 1.0, v0.shape))
    u, v, it, st = oracle.forward_solve(THETAS[k], u0, v0, TAU, STEPS, rtol=RTOL)
    return u, v, it, st


def main():
    jobs = [(k, pert) for k in range(len(THETAS)) for pert in (0, 1, 2)]
    with Pool(min(len(jobs), os.cpu_count() or 1)) as pool:
        res = pool.map(solve, jobs)
    u = np.stack([res[3 * k][0] for k in range(len(THETAS))])
    v = np.stack([res[3 * k][1] for k in range(len(THETAS))])
    status = np.array([res[3 * k][3] for k in range(len(THETAS))])

    def rel(k, j):
        du = np.linalg.norm(res[3 * k + j][0] - u[k]) / np.linalg.norm(u[k])
        dv = np.linalg.norm(res[3 * k + j][1] - v[k]) / np.linalg.norm(v[k])
        return max(du, dv)

    amp = [rel(k, 1) / EPS for k in range(len(THETAS))]
    cg_sens = [rel(k, 2) for k in range(len(THETAS))]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "full_size_128.npz")
    np.savez_compressed(out, theta=THETAS, u=u, v=v, status=status, amplification=np.array(amp),
                        cg_sensitivity=np.array(cg_sens), n=N, tau=TAU, steps=STEPS, rtol=RTOL,
                        eps=EPS, rtol_fp32=RTOL_FP32)
    print(out, "amplification", amp, "cg sensitivity", cg_sens, "status", status)


if __name__ == "__main__":
    main()
