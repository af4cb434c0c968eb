"""Python binding of the C ABI (argument marshalling only).

Device arrays are torch tensors on the current HIP device; the library
enqueues its kernels on torch's current stream.  Nothing here computes a
step of the method.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _lib
from ._lib import RD_ETIMEOUT, RD_OK, Chains, GridDesc, ProblemDesc, check, lib

PLAIN, DA = _lib.MODE_PLAIN, _lib.MODE_DA
FP32, FP64 = _lib.PRECISION_FP32, _lib.PRECISION_FP64


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device arrays must be HIP tensors")
    if not t.is_contiguous():
        raise ValueError("device arrays must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


@dataclass
class Grid:
    """One grid class: size n, growth law, initial fields and data (host float64)."""
    n: int
    u0: np.ndarray
    v0: np.ndarray
    y: np.ndarray | None = None
    sigma: float = 1.0
    growth: int = 0
    growth_rate: float = 0.0


class Problem:
    """Owns an rd_problem handle (init_problem / destroy_problem)."""

    def __init__(self, grids, dt, n_steps, cg_rtol, *, precision=FP32, cg_maxit=0,
                 free_mask=0b1111, lo=(0, 0, 0, 0), hi=(1, 1, 1, 1), step=(0, 0, 0, 0),
                 max_batch=4096, prop_chol=None, prior_kind=(0, 0, 0, 0),
                 prior_mean=(0.0, 0.0, 0.0, 0.0), prior_sd=(1.0, 1.0, 1.0, 1.0),
                 turing_support=False, steady_tol=0.0):
        """prop_chol: optional lower-triangular 4 x 4 factor L of a correlated
        random-walk step (phi' = phi + L z); step is then unused.
        prior_kind[i]: 0 uniform on [lo[i], hi[i]], 1 normal N(prior_mean[i],
        prior_sd[i]^2) in sampling coordinate i (log-normal in gamma, d);
        turing_support: restrict the support to the Turing space.
        steady_tol > 0: stop each solve at the first step whose time
        derivative has an L2 norm below steady_tol (n_steps is the cap)."""
        if isinstance(grids, Grid):
            grids = [grids]
        self.grids = list(grids)
        self.precision = precision
        self.max_batch = max_batch
        self.n_steps = n_steps
        self.dt = dt
        keep = []
        gd = (GridDesc * len(self.grids))()
        for k, g in enumerate(self.grids):
            u0 = np.ascontiguousarray(g.u0, dtype=np.float64).reshape(-1)
            v0 = np.ascontiguousarray(g.v0, dtype=np.float64).reshape(-1)
            if u0.size != g.n * g.n or v0.size != g.n * g.n:
                raise ValueError("u0/v0 must have n*n entries")
            keep += [u0, v0]
            gd[k].n = g.n
            gd[k].growth = g.growth
            gd[k].growth_rate = g.growth_rate
            gd[k].u0 = u0.ctypes.data_as(_lib.c_dp)
            gd[k].v0 = v0.ctypes.data_as(_lib.c_dp)
            if g.y is not None:
                y = np.ascontiguousarray(g.y, dtype=np.float64).reshape(-1)
                if y.size != g.n * g.n:
                    raise ValueError("y must have n*n entries")
                keep.append(y)
                gd[k].y = y.ctypes.data_as(_lib.c_dp)
            gd[k].sigma = g.sigma
        d = ProblemDesc()
        d.n_grids = len(self.grids)
        d.grids = gd
        d.dt = dt
        d.n_steps = n_steps
        d.cg_rtol = cg_rtol
        d.cg_maxit = cg_maxit
        d.precision = precision
        d.free_mask = free_mask
        for i in range(4):
            d.lo[i], d.hi[i], d.step[i] = lo[i], hi[i], step[i]
        d.max_batch = max_batch
        for i in range(4):
            d.prior_kind[i] = int(prior_kind[i])
            d.prior_mean[i] = float(prior_mean[i])
            d.prior_sd[i] = float(prior_sd[i])
        d.turing_support = int(bool(turing_support))
        d.steady_tol = float(steady_tol)
        if prop_chol is not None:
            L = np.asarray(prop_chol, dtype=np.float64).reshape(4, 4)
            for i in range(4):
                for j in range(4):
                    d.prop_chol[4 * i + j] = L[i, j]
        h = ctypes.c_void_p()
        torch.cuda.init()
        check(lib().init_problem(ctypes.byref(d), ctypes.byref(h)), "init_problem")
        self.h = h
        del keep

    def close(self):
        if getattr(self, "h", None):
            lib().destroy_problem(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def field_dtype(self):
        return torch.float32 if self.precision == FP32 else torch.float64

    # -- forward map and likelihood -------------------------------------
    def forward_solve(self, theta, grid_id=None, fields=True, stream=None):
        """theta: HIP float64 [n, 4] (a, b, gamma, d).  Returns (u, v, status, iters).

        With one grid class u, v are [n, N, N]; with several they are
        [n, M*M] (M the largest size) and item c of size N is
        u[c, :N*N].view(N, N)."""
        n = theta.shape[0]
        M = max(g.n for g in self.grids)
        shape = (n, M, M) if len(self.grids) == 1 else (n, M * M)
        dev = theta.device
        u = torch.empty(shape, dtype=self.field_dtype, device=dev) if fields else None
        v = torch.empty(shape, dtype=self.field_dtype, device=dev) if fields else None
        st = torch.empty(n, dtype=torch.int32, device=dev)
        it = torch.empty((n, 2), dtype=torch.int32, device=dev)
        check(lib().forward_solve_batch(self.h, n, _ptr(theta), _ptr(grid_id), _ptr(u), _ptr(v),
                                        _ptr(st), _ptr(it), _stream(stream)), "forward_solve_batch")
        return u, v, st, it

    def forward_solve_steady(self, theta, grid_id=None, stream=None):
        """forward_solve plus the IMEX steps each item took: (u, v, status,
        iters, steps int32 [n])."""
        n = theta.shape[0]
        M = max(g.n for g in self.grids)
        shape = (n, M, M) if len(self.grids) == 1 else (n, M * M)
        dev = theta.device
        u = torch.empty(shape, dtype=self.field_dtype, device=dev)
        v = torch.empty(shape, dtype=self.field_dtype, device=dev)
        st = torch.empty(n, dtype=torch.int32, device=dev)
        it = torch.empty((n, 2), dtype=torch.int32, device=dev)
        steps = torch.empty(n, dtype=torch.int32, device=dev)
        check(lib().forward_solve_steady_batch(self.h, n, _ptr(theta), _ptr(grid_id), _ptr(u),
                                               _ptr(v), _ptr(st), _ptr(it), _ptr(steps),
                                               _stream(stream)), "forward_solve_steady_batch")
        return u, v, st, it, steps

    def log_likelihood(self, theta, grid_id=None, stream=None):
        """Returns (phi float64 [n], status int32 [n], iters int32 [n, 2])."""
        n = theta.shape[0]
        dev = theta.device
        phi = torch.empty(n, dtype=torch.float64, device=dev)
        st = torch.empty(n, dtype=torch.int32, device=dev)
        it = torch.empty((n, 2), dtype=torch.int32, device=dev)
        check(lib().log_likelihood_batch(self.h, n, _ptr(theta), _ptr(grid_id), _ptr(phi),
                                         _ptr(st), _ptr(it), _stream(stream)),
              "log_likelihood_batch")
        return phi, st, it

    def field_misfit(self, u, stream=None):
        n = u.shape[0]
        phi = torch.empty(n, dtype=torch.float64, device=u.device)
        check(lib().field_misfit_batch(self.h, n, _ptr(u), None, _ptr(phi), _stream(stream)),
              "field_misfit_batch")
        return phi

    # -- sampler ----------------------------------------------------------
    def mcmc_step(self, chains: "ChainState", n_steps=1, mode=PLAIN, stream=None):
        c = chains.struct()
        check(lib().mcmc_step_batch(self.h, ctypes.byref(c), n_steps, mode, _stream(stream)),
              "mcmc_step_batch")
        chains.step = int(c.step)

    def propose(self, chains: "ChainState", stream=None):
        n = chains.n
        dev = chains.phi.device
        prop = torch.empty((n, 4), dtype=torch.float64, device=dev)
        inside = torch.empty(n, dtype=torch.int32, device=dev)
        c = chains.struct()
        check(lib().propose_batch(self.h, ctypes.byref(c), _ptr(prop), _ptr(inside),
                                  _stream(stream)), "propose_batch")
        return prop, inside

    def accept(self, chains: "ChainState", prop, inside, loglik_prop, stream=None):
        c = chains.struct()
        check(lib().accept_batch(self.h, ctypes.byref(c), _ptr(prop), _ptr(inside),
                                 _ptr(loglik_prop), _stream(stream)), "accept_batch")
        chains.step = int(c.step)

    # -- parallel Metropolis-Hastings (Algorithm 2) ------------------------
    def pmh_step(self, chains: "ChainState", n_prop, n_iter=1, stream=None):
        """n_iter steps of Algorithm 2 (N = n_prop proposals per chain, N
        draws each) with Phi from the library's solve."""
        c = chains.struct()
        check(lib().pmh_step_batch(self.h, ctypes.byref(c), int(n_prop), int(n_iter),
                                   _stream(stream)), "pmh_step_batch")
        chains.step = int(c.step)

    def pmh_propose(self, chains: "ChainState", n_prop, stream=None):
        """The N proposals of every chain: ([n * N, 4] float64, [n * N] int32)."""
        n = chains.n
        dev = chains.phi.device
        prop = torch.empty((n * n_prop, 4), dtype=torch.float64, device=dev)
        inside = torch.empty(n * n_prop, dtype=torch.int32, device=dev)
        c = chains.struct()
        check(lib().pmh_propose_batch(self.h, ctypes.byref(c), int(n_prop), _ptr(prop),
                                      _ptr(inside), _stream(stream)), "pmh_propose_batch")
        return prop, inside

    def pmh_resample(self, chains: "ChainState", n_prop, prop, inside, loglik_prop, stream=None):
        c = chains.struct()
        check(lib().pmh_resample_batch(self.h, ctypes.byref(c), int(n_prop), _ptr(prop),
                                       _ptr(inside), _ptr(loglik_prop), _stream(stream)),
              "pmh_resample_batch")
        chains.step = int(c.step)

    # -- surrogate (first stage of delayed acceptance) -------------------
    def surrogate_create(self, width=512, depth=4, out_side=32, seed=5):
        check(lib().surrogate_create(self.h, width, depth, out_side, seed), "surrogate_create")
        self.sur_shape = (width, depth, out_side)

    def downsample(self, u, stream=None):
        n = u.shape[0]
        S = self.sur_shape[2]
        out = torch.empty((n, S * S), dtype=torch.float32, device=u.device)
        check(lib().downsample_batch(self.h, n, _ptr(u), _ptr(out), _stream(stream)),
              "downsample_batch")
        return out

    def surrogate_set_input_box(self, lo, hi):
        lo_a = (ctypes.c_double * 4)(*[float(x) for x in lo])
        hi_a = (ctypes.c_double * 4)(*[float(x) for x in hi])
        check(lib().surrogate_set_input_box(self.h, lo_a, hi_a), "surrogate_set_input_box")

    def surrogate_set_scaling(self, mean, sd, sigma1, stream=None):
        check(lib().surrogate_set_scaling(self.h, _ptr(mean), _ptr(sd), float(sigma1),
                                          _stream(stream)), "surrogate_set_scaling")

    def surrogate_train_step(self, phi, target, lr, loss_out=None, stream=None):
        check(lib().surrogate_train_step(self.h, phi.shape[0], _ptr(phi), _ptr(target), float(lr),
                                         _ptr(loss_out), _stream(stream)), "surrogate_train_step")

    def surrogate_forward(self, phi, raw=True, stream=None):
        n = phi.shape[0]
        S = self.sur_shape[2]
        out = torch.empty((n, S * S), dtype=torch.float32, device=phi.device)
        check(lib().surrogate_forward(self.h, n, _ptr(phi), _ptr(out), int(raw), _stream(stream)),
              "surrogate_forward")
        return out

    def surrogate_loglik(self, phi, stream=None):
        out = torch.empty(phi.shape[0], dtype=torch.float64, device=phi.device)
        check(lib().surrogate_loglik_batch(self.h, phi.shape[0], _ptr(phi), _ptr(out),
                                           _stream(stream)), "surrogate_loglik_batch")
        return out

    def surrogate_layer_shapes(self):
        w, d, S = self.sur_shape
        sizes = [4] + [w] * d + [S * S]
        return list(zip(sizes[1:], sizes[:-1]))

    def surrogate_params(self, dir=0, params=None, stream=None):
        """dir 0: read [(W, b)]; 1: write `params`; 2: read last gradients."""
        out = []
        for layer, (fo, fi) in enumerate(self.surrogate_layer_shapes()):
            if dir == 1:
                W, b = (t.float().contiguous() for t in params[layer])
            else:
                W = torch.empty((fo, fi), dtype=torch.float32, device="cuda")
                b = torch.empty(fo, dtype=torch.float32, device="cuda")
            check(lib().surrogate_params(self.h, layer, _ptr(W), _ptr(b), dir, _stream(stream)),
                  "surrogate_params")
            out.append((W, b))
        return out

    # -- utilities --------------------------------------------------------
    def autotune(self):
        out = (ctypes.c_int32 * len(self.grids))()
        check(lib().rd_autotune(self.h, ctypes.cast(out, ctypes.c_void_p)), "rd_autotune")
        return list(out)

    def set_tile(self, grid, cpt):
        """Select grid class `grid`'s tile by cells per thread."""
        check(lib().rd_set_tile(self.h, int(grid), int(cpt)), "rd_set_tile")

    def set_mixed_threads(self, threads):
        """Workgroup size (512 or 1024) of the launch for batches mixing classes."""
        check(lib().rd_set_mixed_threads(self.h, int(threads)), "rd_set_mixed_threads")

    def set_da_substeps(self, substeps):
        """First stage of delayed acceptance: that many Metropolis steps on
        the surrogate posterior (1: one screened proposal)."""
        check(lib().rd_set_da_substeps(self.h, int(substeps)), "rd_set_da_substeps")

    def captured_graphs(self):
        """Metropolis steps currently held as captured HIP graphs."""
        t = ctypes.c_int32()
        check(lib().rd_captured_graphs(self.h, ctypes.byref(t)), "rd_captured_graphs")
        return t.value

    def mixed_threads(self):
        """Workgroup size of the launch that serves batches mixing grid classes."""
        t = ctypes.c_int32()
        check(lib().rd_mixed_threads(self.h, ctypes.byref(t)), "rd_mixed_threads")
        return t.value

    def check_solves(self, reset=True):
        """Synchronises and raises RDError (RD_ETIMEOUT) when a cooperative
        group wait gave up since the last check; returns the count (0)."""
        n = ctypes.c_int64()
        check(lib().rd_check_solves(self.h, ctypes.byref(n), int(reset)), "rd_check_solves")
        return n.value

    def group_timeouts(self, reset=True):
        """Members whose cooperative group wait gave up (no exception)."""
        n = ctypes.c_int64()
        code = lib().rd_check_solves(self.h, ctypes.byref(n), int(reset))
        if code not in (RD_OK, RD_ETIMEOUT):
            check(code, "rd_check_solves")
        return n.value

    def set_coop_wait(self, wait_ticks=0, stall_ticks=0):
        """Test hook: bound of a cooperative group wait and a first-exchange
        delay of member 1 of every group (100 MHz ticks; 0, 0 restores)."""
        check(lib().rd_set_coop_wait(self.h, int(wait_ticks), int(stall_ticks)),
              "rd_set_coop_wait")

    def solver_timing(self, enable=True, reset=False):
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        check(lib().rd_solver_timing(self.h, int(enable), ctypes.byref(ms), ctypes.byref(n),
                                     int(reset)), "rd_solver_timing")
        return ms.value, n.value


class Growth1D:
    """Owns a g1d_problem handle: the one-dimensional growing domain of
    Example 1 (g1d_init / g1d_destroy).  Host arrays are float64 numpy
    arrays; y is [2, n] (rows u, v) or None."""

    POLY, EXP, LOGISTIC = _lib.G1D_LAW_POLY, _lib.G1D_LAW_EXP, _lib.G1D_LAW_LOGISTIC

    def __init__(self, n, n_steps, tau, theta, u0, v0, *, law=0, rho_T=1.0, y=None, obs=1,
                 sigma=1.0, max_batch=1024, lo=(-10.0,) * 3, hi=(10.0,) * 3, step=(0.0,) * 3,
                 prior_kind=(0, 0, 0), prior_mean=(0.0,) * 3, prior_sd=(1.0,) * 3):
        self._keep = [np.ascontiguousarray(u0, dtype=np.float64),
                      np.ascontiguousarray(v0, dtype=np.float64)]
        d = _lib.G1dDesc()
        d.n, d.n_steps, d.tau, d.law, d.rho_T = n, n_steps, tau, law, rho_T
        d.theta[:] = [float(x) for x in theta]
        d.u0 = self._keep[0].ctypes.data_as(_lib.c_dp)
        d.v0 = self._keep[1].ctypes.data_as(_lib.c_dp)
        if y is not None:
            self._keep.append(np.ascontiguousarray(np.asarray(y, dtype=np.float64).reshape(2, n)))
            d.y = self._keep[-1].ctypes.data_as(_lib.c_dp)
        d.obs, d.sigma, d.max_batch = obs, sigma, max_batch
        d.lo[:], d.hi[:], d.step[:] = ([float(x) for x in lo], [float(x) for x in hi],
                                       [float(x) for x in step])
        d.prior_kind[:] = [int(x) for x in prior_kind]
        d.prior_mean[:] = [float(x) for x in prior_mean]
        d.prior_sd[:] = [float(x) for x in prior_sd]
        h = ctypes.c_void_p()
        check(lib().g1d_init(ctypes.byref(d), ctypes.byref(h)), "g1d_init")
        self.h, self.n, self.law = h, n, law

    def close(self):
        if getattr(self, "h", None):
            lib().g1d_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def forward(self, beta=None, m=None, stream=None):
        """beta: HIP float64 [m, 3] (polynomial law) or None with m items of
        a data law.  Returns (u, v, status) with u, v float64 [m, n]."""
        m = beta.shape[0] if beta is not None else (m or 1)
        dev = beta.device if beta is not None else torch.device("cuda")
        u = torch.empty((m, self.n), dtype=torch.float64, device=dev)
        v = torch.empty((m, self.n), dtype=torch.float64, device=dev)
        st = torch.empty(m, dtype=torch.int32, device=dev)
        check(lib().g1d_forward_batch(self.h, m, _ptr(beta), _ptr(u), _ptr(v), _ptr(st),
                                      _stream(stream)), "g1d_forward_batch")
        return u, v, st

    def log_likelihood(self, beta, stream=None):
        """Returns (phi float64 [m], status int32 [m])."""
        m = beta.shape[0]
        phi = torch.empty(m, dtype=torch.float64, device=beta.device)
        st = torch.empty(m, dtype=torch.int32, device=beta.device)
        check(lib().g1d_log_likelihood_batch(self.h, m, _ptr(beta), _ptr(phi), _ptr(st),
                                             _stream(stream)), "g1d_log_likelihood_batch")
        return phi, st

    def mcmc_step(self, chains: "ChainState", n_steps=1, stream=None):
        """Metropolis steps over beta; chains.phi is [C, 4] with beta in the
        first three columns."""
        c = chains.struct()
        check(lib().g1d_mcmc_step_batch(self.h, ctypes.byref(c), n_steps, _stream(stream)),
              "g1d_mcmc_step_batch")
        chains.step = int(c.step)


@dataclass
class ChainState:
    """Device state of a batch of chains (the rd_chains struct's arrays)."""
    phi: torch.Tensor
    loglik: torch.Tensor
    seed: int = 4
    step: int = 0
    loglik_sur: torch.Tensor | None = None
    grid_id: torch.Tensor | None = None
    n_accept: torch.Tensor | None = None
    n_accept1: torch.Tensor | None = None
    n_solves: torch.Tensor | None = None
    cg_iters: torch.Tensor | None = None
    trace: torch.Tensor | None = None
    trace_step0: int = 0
    imex_steps: torch.Tensor | None = None   # [n] IMEX steps completed by the solves
    fail_bits: torch.Tensor | None = None    # [n][8] solves with status bit k set

    @property
    def n(self):
        return self.phi.shape[0]

    @classmethod
    def create(cls, phi, loglik, seed=4, step=0, trace_steps=0, da=False, grid_id=None):
        dev = phi.device
        n = phi.shape[0]
        z = lambda: torch.zeros(n, dtype=torch.int64, device=dev)  # noqa: E731
        return cls(phi=phi.contiguous(), loglik=loglik.contiguous(), seed=seed, step=step,
                   loglik_sur=torch.zeros(n, dtype=torch.float64, device=dev) if da else None,
                   grid_id=grid_id, n_accept=z(), n_accept1=z(), n_solves=z(),
                   cg_iters=torch.zeros((n, 2), dtype=torch.int64, device=dev),
                   trace=(torch.zeros((trace_steps, n, 4), dtype=torch.float64, device=dev)
                          if trace_steps else None), trace_step0=step,
                   imex_steps=z(), fail_bits=torch.zeros((n, 8), dtype=torch.int64, device=dev))

    def struct(self) -> Chains:
        c = Chains()
        c.n_chains = self.n
        c.phi = _ptr(self.phi)
        c.loglik = _ptr(self.loglik)
        c.loglik_sur = _ptr(self.loglik_sur)
        c.grid_id = _ptr(self.grid_id)
        c.n_accept = _ptr(self.n_accept)
        c.n_accept1 = _ptr(self.n_accept1)
        c.n_solves = _ptr(self.n_solves)
        c.cg_iters = _ptr(self.cg_iters)
        c.trace = _ptr(self.trace)
        c.trace_rows = self.trace.shape[0] if self.trace is not None else 0
        c.trace_step0 = self.trace_step0
        c.seed = self.seed
        c.step = self.step
        c.imex_steps = _ptr(self.imex_steps)
        c.fail_bits = _ptr(self.fail_bits)
        return c

    def save(self, path, stream=None):
        """Write the chain state to `path` (rd_chains_save)."""
        c = self.struct()
        check(lib().rd_chains_save(ctypes.byref(c), os.fsencode(path), _stream(stream)),
              "rd_chains_save")

    def load(self, path, stream=None):
        """Overwrite this state (same number of chains) from `path`
        (rd_chains_load); seed and step come from the file."""
        c = self.struct()
        check(lib().rd_chains_load(ctypes.byref(c), os.fsencode(path), _stream(stream)),
              "rd_chains_load")
        self.seed = int(c.seed)
        self.step = int(c.step)
