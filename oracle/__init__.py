"""FP64 CPU oracle for the Schnakenberg Bayesian-identification hot path.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this package; the product library never does.  It
shares no code with the HIP path (it is plain C in ``rd_oracle.c`` plus the
numpy modules beside this file).

This module compiles ``rd_oracle.c`` with gcc (OpenMP over independent
solves) and exposes it through ctypes with numpy arrays.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rd_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

NOT_CONVERGED = 1
BREAKDOWN = 2
NONFINITE = 4


def build() -> str:
    """Compile the C oracle (IEEE double, no fast-math) into liboracle.so."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
           "-fno-fast-math", "-ffp-contract=off", "-o", _LIB + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        up = ctypes.POINTER(ctypes.c_uint32)
        c_int, c_d, c_u32, c_u64 = ctypes.c_int, ctypes.c_double, ctypes.c_uint32, ctypes.c_uint64
        L.orc_laplacian.argtypes = [c_int, dp, dp]
        L.orc_apply_A.argtypes = [c_int, dp, c_d, dp, dp]
        L.orc_cg.argtypes = [c_int, dp, c_d, dp, dp, c_d, c_int, ip]
        L.orc_cg.restype = c_int
        L.orc_dense_solve.argtypes = [c_int, dp, c_d, dp, dp]
        L.orc_dense_solve.restype = c_int
        L.orc_imex_step.argtypes = [c_int, dp, c_int, c_d, c_d, c_d, c_d, c_int, dp, dp, ip]
        L.orc_imex_step.restype = c_int
        L.orc_forward_solve.argtypes = [c_int, dp, c_int, c_d, c_d, c_int, c_d, c_int, dp, dp,
                                        dp, dp, ip]
        L.orc_forward_solve.restype = c_int
        L.orc_misfit.argtypes = [c_int, dp, dp, c_d]
        L.orc_misfit.restype = c_d
        L.orc_loglik_batch.argtypes = [c_int, dp, c_int, c_int, c_d, c_d, c_int, c_d, c_int, dp,
                                       dp, dp, c_d, dp, ip, ip]
        L.orc_philox4x32_10.argtypes = [up, up, up]
        L.orc_uniform_from_words.argtypes = [c_u32, c_u32]
        L.orc_uniform_from_words.restype = c_d
        L.orc_normals4.argtypes = [c_u32, c_u32, c_u64, c_u32, dp]
        L.orc_uniform1.argtypes = [c_u32, c_u32, c_u64, c_u32]
        L.orc_uniform1.restype = c_d
        L.orc_uniforms4.argtypes = [c_u32, c_u32, c_u64, c_u32, dp]
        L.orc_normals4_at.argtypes = [c_u32, c_u32, c_u64, c_u32, c_u32, dp]
        L.orc_uniform_at.argtypes = [c_u32, c_u32, c_u64, c_u32, c_u32]
        L.orc_uniform_at.restype = c_d
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# Grid operator, CG, direct solve (Sec. 3.1.1)

def laplacian(w: np.ndarray) -> np.ndarray:
    """5-point Laplacian with mirror (zero-flux) ghosts on an n x n cell grid."""
    w = _f64(w)
    n = w.shape[-1]
    out = np.empty_like(w)
    lib().orc_laplacian(n, _d(w), _d(out))
    return out


def apply_A(sigma, c, p) -> np.ndarray:
    """(sigma I - c Lap_h) p."""
    sigma, p = _f64(sigma), _f64(p)
    out = np.empty_like(p)
    lib().orc_apply_A(p.shape[-1], _d(sigma), float(c), _d(p), _d(out))
    return out


def cg(sigma, c, b, x0, rtol=1e-12, maxit=None):
    """Unpreconditioned CG from x0; returns (x, iterations, status)."""
    sigma, b = _f64(sigma), _f64(b)
    x = _f64(x0).copy()
    n = b.shape[-1]
    it = ctypes.c_int(0)
    maxit = 10 * n * n if maxit is None else maxit
    st = lib().orc_cg(n, _d(sigma), float(c), _d(b), _d(x), float(rtol), int(maxit),
                      ctypes.byref(it))
    return x, it.value, st


def dense_solve(sigma, c, b):
    sigma, b = _f64(sigma), _f64(b)
    n = b.shape[-1]
    x = np.zeros_like(b)
    st = lib().orc_dense_solve(n, _d(sigma), float(c), _d(b), _d(x))
    return x, st


# --------------------------------------------------------------------------
# IMEX time stepping and the forward map (Sec. 3.1, Sec. 3.1.1)

def imex_step(theta, u, v, tau, t_n=0.0, growth=0, rate=0.0, rtol=1e-12, maxit=None):
    """One IMEX step; returns (u_next, v_next, iters[2], status)."""
    th = _f64(theta)
    u, v = _f64(u).copy(), _f64(v).copy()
    n = u.shape[-1]
    it = np.zeros(2, dtype=np.int32)
    maxit = 10 * n * n if maxit is None else maxit
    st = lib().orc_imex_step(n, _d(th), int(growth), float(rate), float(t_n), float(tau),
                             float(rtol), int(maxit), _d(u), _d(v), _i(it))
    return u, v, it, st


def forward_solve(theta, u0, v0, tau, n_steps, growth=0, rate=0.0, rtol=1e-12, maxit=None):
    """G(theta): fields at T = n_steps*tau; returns (u, v, iters[2], status)."""
    th = _f64(theta)
    u0, v0 = _f64(u0), _f64(v0)
    n = u0.shape[-1]
    u = np.empty_like(u0)
    v = np.empty_like(v0)
    it = np.zeros(2, dtype=np.int32)
    maxit = 10 * n * n if maxit is None else maxit
    st = lib().orc_forward_solve(n, _d(th), int(growth), float(rate), float(tau), int(n_steps),
                                 float(rtol), int(maxit), _d(u0), _d(v0), _d(u), _d(v), _i(it))
    return u, v, it, st


ST_NOT_STEADY = 32


def time_derivative_norm(u, v, u_next, v_next, tau) -> float:
    """L2 norm over the unit square of the discrete time derivative of (u, v)
    (cell-centred quadrature, h = 1/n): sqrt(h^2 sum (du^2 + dv^2)) / tau."""
    n = np.asarray(u).shape[-1]
    du = _f64(u_next) - _f64(u)
    dv = _f64(v_next) - _f64(v)
    return math.sqrt(float((du * du).sum() + (dv * dv).sum())) / (n * tau)


def forward_solve_steady(theta, u0, v0, tau, max_steps, tol, growth=0, rate=0.0, rtol=1e-12,
                         maxit=None):
    """Sec. 3.1.2: step until the L2 norm of the discrete time derivative
    of (u, v) falls below tol (the fields after that step are the result),
    at most max_steps steps (then status ST_NOT_STEADY).

    Returns (u, v, steps, iters[2], status)."""
    u, v = _f64(u0).copy(), _f64(v0).copy()
    its = np.zeros(2, dtype=np.int64)
    for s in range(max_steps):
        un, vn, it, st = imex_step(theta, u, v, tau, t_n=s * tau, growth=growth, rate=rate,
                                   rtol=rtol, maxit=maxit)
        its += it
        if st:
            return un, vn, s + 1, its, st
        dnorm = time_derivative_norm(u, v, un, vn, tau)
        u, v = un, vn
        if dnorm < tol:
            return u, v, s + 1, its, 0
    return u, v, max_steps, its, ST_NOT_STEADY


def misfit(y, u, sigma) -> float:
    """Phi = |y - u|^2 / (2 sigma^2), eq. (logl) for Gaussian noise."""
    y, u = _f64(y).ravel(), _f64(u).ravel()
    return lib().orc_misfit(y.size, _d(y), _d(u), float(sigma))


def loglik_batch(thetas, u0, v0, y, sigma, tau, n_steps, growth=0, rate=0.0, rtol=1e-12,
                 maxit=None):
    """Phi for each row of thetas [m][4] (natural parameters); +inf on failure.

    Returns (phi[m], status[m], iters[m][2])."""
    th = _f64(np.atleast_2d(thetas))
    m = th.shape[0]
    u0, v0, y = _f64(u0), _f64(v0), _f64(y)
    n = u0.shape[-1]
    phi = np.empty(m)
    st = np.zeros(m, dtype=np.int32)
    it = np.zeros((m, 2), dtype=np.int32)
    maxit = 10 * n * n if maxit is None else maxit
    lib().orc_loglik_batch(m, _d(th), n, int(growth), float(rate), float(tau), int(n_steps),
                           float(rtol), int(maxit), _d(u0), _d(v0), _d(y), float(sigma),
                           _d(phi), _i(st), _i(it))
    return phi, st, it


# --------------------------------------------------------------------------
# Counter-based random numbers (Philox4x32-10)

def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    P = ctypes.POINTER(ctypes.c_uint32)
    lib().orc_philox4x32_10(c.ctypes.data_as(P), k.ctypes.data_as(P), out.ctypes.data_as(P))
    return out


def uniform_from_words(hi, lo) -> float:
    return lib().orc_uniform_from_words(int(hi), int(lo))


def normals4(seed, chain, step, purpose):
    z = np.zeros(4)
    lib().orc_normals4(int(seed) & 0xFFFFFFFF, int(chain), int(step), int(purpose), _d(z))
    return z


def uniform1(seed, chain, step, purpose) -> float:
    return lib().orc_uniform1(int(seed) & 0xFFFFFFFF, int(chain), int(step), int(purpose))


def normals4_at(seed, chain, step, purpose, block0):
    """Four normals from blocks block0, block0 + 1 (normals4 is block0 = 0)."""
    z = np.zeros(4)
    lib().orc_normals4_at(int(seed) & 0xFFFFFFFF, int(chain), int(step), int(purpose),
                          int(block0), _d(z))
    return z


def uniform_at(seed, chain, step, purpose, block) -> float:
    return lib().orc_uniform_at(int(seed) & 0xFFFFFFFF, int(chain), int(step), int(purpose),
                                int(block))


def uniforms4(seed, chain, step, purpose):
    u = np.zeros(4)
    lib().orc_uniforms4(int(seed) & 0xFFFFFFFF, int(chain), int(step), int(purpose), _d(u))
    return u
