"""Surrogate pipeline for the first stage of delayed acceptance.

The network (the library's BF16 MFMA MLP) maps sampling coordinates
phi = (a, b, ln gamma, ln d) to the block-mean-downsampled u field at T.  It
is trained on forward solves that the library itself produces from prior
draws, and it is used only to screen proposals: the full solve makes the
final decision (Christen and Fox, J. Comput. Graph. Stat. 14(4), 2005), so
the sampled posterior does not depend on how good the surrogate is.

Every solve, downsampling, forward and backward pass and Adam step runs in
the library's kernels; this module only draws inputs, batches and shuffles.

Command line (one surrogate training run on the 128 x 128 workload):

    python -m paper_1605_04718_amd.surrogate --solves 200000 --epochs 40
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time
from dataclasses import dataclass

import numpy as np
import torch

from . import inputs


def to_natural_t(phi: torch.Tensor) -> torch.Tensor:
    """(a, b, ln gamma, ln d) -> (a, b, gamma, d) on the device."""
    th = phi.clone()
    th[:, 2:] = torch.exp(phi[:, 2:])
    return th


@dataclass
class Dataset:
    phi: torch.Tensor      # [m, 4] float64 sampling coordinates
    u_ds: torch.Tensor     # [m, S*S] float32 block means of u at T
    solve_seconds: float
    dropped: int           # prior draws whose solve failed (not in the dataset)
    outliers: int          # draws with |u| above the cut (not in the dataset)


def make_dataset(p, m, lo, hi, seed=inputs.SEED_DATASET, batch=4096, max_abs=10.0,
                 log=None, phi=None) -> Dataset:
    """m prior draws (uniform on the box [lo, hi] in sampling coordinates),
    each solved to T on grid class 0 and downsampled to the surrogate's
    output size.  Failed solves are dropped, and so are fields with a block
    mean above max_abs in magnitude: at the largest gamma of the box the
    time step leaves the stable range of the linearised scheme for some
    (a, b), and the resulting large spurious fields would dominate a
    squared-error fit while lying far from any posterior mass.  `phi`
    ([m, 4]) replaces the prior draws, e.g. draws around the posterior."""
    dev = torch.device("cuda")
    batch = min(batch, p.max_batch)
    if phi is None:
        phi = inputs.box_draws(m, lo, hi, seed=seed)
    phi_all = torch.as_tensor(np.asarray(phi), dtype=torch.float64).to(dev)
    m = phi_all.shape[0]
    S = p.sur_shape[2]
    keep_phi, keep_u = [], []
    dropped = outliers = 0
    torch.cuda.synchronize()
    t0 = time.time()
    for i in range(0, m, batch):
        ph = phi_all[i:i + batch]
        u, _, st, _ = p.forward_solve(to_natural_t(ph), fields=True)
        ds = p.downsample(u)
        ok = st == 0
        dropped += int((~ok).sum())
        big = ok & ~(ds.abs().amax(dim=1) <= max_abs)
        outliers += int(big.sum())
        ok = ok & ~big
        keep_phi.append(ph[ok])
        keep_u.append(ds[ok])
        del u
        if log:
            torch.cuda.synchronize()
            log(f"dataset: {min(i + batch, m)}/{m} solves, {time.time() - t0:.1f} s")
    torch.cuda.synchronize()
    secs = time.time() - t0
    return Dataset(torch.cat(keep_phi), torch.cat(keep_u).reshape(-1, S * S), secs, dropped,
                   outliers)


def split(ds: Dataset, held_out: float = 0.05):
    """Deterministic train / held-out split (the draws are already i.i.d.)."""
    m = ds.phi.shape[0]
    k = int(round(m * (1.0 - held_out)))
    return (ds.phi[:k], ds.u_ds[:k]), (ds.phi[k:], ds.u_ds[k:])


def standardisation(u_train: torch.Tensor, floor: float = 1e-6):
    """Per-pixel mean and s.d. of the training targets (s.d. floored)."""
    mean = u_train.mean(dim=0)
    sd = u_train.std(dim=0).clamp_min(floor)
    return mean.float().contiguous(), sd.float().contiguous()


def train(p, phi, target_std, epochs, batch=1024, lr=1e-3, seed=0, log=None):
    """Adam on the mean squared error of standardised targets; returns the
    mean training loss of each epoch and the seconds spent in training."""
    dev = phi.device
    m = phi.shape[0]
    g = torch.Generator(device=dev)
    g.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    history = []
    steps = 0
    torch.cuda.synchronize()
    t0 = time.time()
    for ep in range(epochs):
        perm = torch.randperm(m, device=dev, generator=g)
        acc = torch.zeros(1, dtype=torch.float64, device=dev)
        nb = 0
        for i in range(0, m - batch + 1, batch):
            idx = perm[i:i + batch]
            p.surrogate_train_step(phi[idx].contiguous(), target_std[idx].contiguous(), lr, loss)
            acc += loss
            nb += 1
            steps += 1
        history.append(float(acc.item()) / max(nb, 1))
        if log and (ep % max(1, epochs // 10) == 0 or ep == epochs - 1):
            log(f"epoch {ep}: mse {history[-1]:.4e} ({time.time() - t0:.1f} s)")
    torch.cuda.synchronize()
    return history, time.time() - t0, steps


def predict(p, phi, batch=4096):
    """De-standardised predictions [n, S*S] (float32)."""
    outs = [p.surrogate_forward(phi[i:i + batch].contiguous(), raw=False)
            for i in range(0, phi.shape[0], batch)]
    return torch.cat(outs)


def held_out_error(p, phi, u_true):
    """Relative L2 errors of the surrogate against full solves: over the
    whole held-out set, and the median of the per-sample errors; plus the
    per-pixel RMS error (the surrogate's noise level)."""
    pred = predict(p, phi).double()
    t = u_true.double()
    diff = pred - t
    total = float(diff.norm() / t.norm())
    per = (diff.norm(dim=1) / t.norm(dim=1)).cpu().numpy()
    rms = float(diff.pow(2).mean().sqrt())
    return {"rel_l2": total, "rel_l2_median": float(np.median(per)),
            "rel_l2_p90": float(np.quantile(per, 0.9)), "rms_per_pixel": rms}


def baseline_error(u_train, u_true):
    """The same errors for the constant predictor (training mean): what the
    method has without a network."""
    mean = u_train.double().mean(dim=0, keepdim=True)
    t = u_true.double()
    diff = mean - t
    return float(diff.norm() / t.norm())


def first_stage_sigma(sigma, block, rms):
    """Per-pixel noise s.d. of the first stage: the block mean of `block`
    noisy data values has variance sigma^2 / block; the surrogate adds its
    own error, taken as independent Gaussian with the held-out RMS."""
    return math.sqrt(sigma * sigma / block + rms * rms)


def fit(p, sigma, lo, hi, solves, epochs, batch=1024, lr=1e-3, held_out=0.05, log=None,
        phi=None):
    """Dataset -> split -> standardisation -> training -> held-out error ->
    first-stage scaling installed in p.  Returns a report dict."""
    ds = make_dataset(p, solves, lo, hi, log=log, phi=phi)
    (ph_tr, u_tr), (ph_te, u_te) = split(ds, held_out)
    mean, sd = standardisation(u_tr)
    target = ((u_tr - mean) / sd).float().contiguous()
    history, train_s, steps = train(p, ph_tr, target, epochs, batch=batch, lr=lr, log=log)
    p.surrogate_set_scaling(mean, sd, 1.0)
    err = held_out_error(p, ph_te, u_te)
    err["constant_predictor_rel_l2"] = baseline_error(u_tr, u_te)
    N = p.grids[0].n
    S = p.sur_shape[2]
    sig1 = first_stage_sigma(sigma, (N // S) ** 2, err["rms_per_pixel"])
    p.surrogate_set_scaling(mean, sd, sig1)
    width, depth, _ = p.sur_shape
    sizes = [4] + [width] * depth + [S * S]
    macs = sum(a * b for a, b in zip(sizes[:-1], sizes[1:]))
    # forward 2 flops per MAC, backward 4 (input and weight gradients)
    train_flops = 6.0 * macs * batch * steps
    return {
        "solves": solves, "dropped": ds.dropped, "outliers": ds.outliers,
        "dataset_seconds": ds.solve_seconds,
        "train_samples": int(ph_tr.shape[0]), "held_out_samples": int(ph_te.shape[0]),
        "epochs": epochs, "batch": batch, "lr": lr, "train_steps": steps,
        "train_seconds": train_s, "train_tflops": train_flops / train_s / 1e12 if train_s else None,
        "final_train_mse": history[-1] if history else None, "loss_history": history,
        "held_out": err, "sigma1": sig1,
        "scaling_mean": mean, "scaling_sd": sd,   # device tensors (not for JSON)
    }


def _main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--solves", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--out", default="")
    args = ap.parse_args(argv)
    from .api import Grid, Problem
    theta_true = (0.1, 0.9, 200.0, 10.0)
    tau, T = 2.5e-4, 2.0
    lo = (0.0, 0.0, math.log(50.0), math.log(5.0))
    hi = (1.0, 1.0, math.log(500.0), math.log(50.0))

    def log(msg):
        print(f"[surrogate] {msg}", file=sys.stderr, flush=True)

    n_steps = int(round(T / tau))
    u0, v0 = inputs.initial_fields(args.n, theta_true[0], theta_true[1])
    gen = Problem([Grid(n=args.n, u0=u0, v0=v0)], tau, n_steps, 1e-7, cg_maxit=400, max_batch=1)
    ut, _, st, _ = gen.forward_solve(torch.tensor([theta_true], dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    y, sigma = inputs.noisy_data(ut[0].double().cpu().numpy(), 0.01)
    gen.close()
    p = Problem([Grid(n=args.n, u0=u0, v0=v0, y=y, sigma=sigma)], tau, n_steps, 1e-7,
                cg_maxit=400, lo=lo, hi=hi, max_batch=4096)
    p.autotune()
    p.surrogate_create(512, 4, 32, seed=inputs.SEED_SURROGATE_INIT)
    rep = fit(p, sigma, lo, hi, args.solves, args.epochs, batch=args.batch, lr=args.lr, log=log)
    rep.pop("scaling_mean")
    rep.pop("scaling_sd")
    rep["grid"] = args.n
    rep["workload"] = (f"{args.solves} prior draws solved at {args.n}x{args.n} to T = 2 "
                       f"(dt 2.5e-4) -> 32x32 block means; MLP 4-512x4-1024 GELU, BF16 MFMA")
    line = json.dumps(rep)
    print(line)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")
    p.close()


if __name__ == "__main__":
    _main()
