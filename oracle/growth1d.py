"""Oracle for Example 1 of Sec. 3.1.2: the activator-depleted system on a
one-dimensional uniformly growing domain (m = 1), whose growth function
rho(t) is the unknown (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Discretisation (Sec. 3.1.1 with m = 1): cell-centred grid of n cells on the
unit interval, h = 1/n, mirror ghost cells (zero flux); one IMEX step
  [1/tau + rho'/rho + g (1 - u v)] u' - rho^-2 Lap_h u' = u/tau + g a
  [1/tau + rho'/rho + g u^2]       v' - d rho^-2 Lap_h v' = v/tau + g b
with rho, rho' at t_n and the fields of level n in the bracketed
coefficients (the 3-point Laplacian acts on v' in the second equation).
Each step is two tridiagonal systems, solved here by a banded direct solve.

Growth: rho(t) = 1 + sum_{k=1..4} beta_k s^k with s = t / T, a degree-4
polynomial with rho(0) = 1; beta_4 = rho_T - 1 - beta_1 - beta_2 - beta_3
fixes rho(T) = rho_T, leaving three free coefficients (Example 1).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.linalg import solve_banded


def rho_poly(beta, rho_T, T, t):
    """(rho(t), rho'(t)) of the degree-4 growth polynomial."""
    b1, b2, b3 = (float(x) for x in beta)
    b4 = rho_T - 1.0 - b1 - b2 - b3
    s = t / T
    rho = 1.0 + s * (b1 + s * (b2 + s * (b3 + s * b4)))
    drho = (b1 + s * (2.0 * b2 + s * (3.0 * b3 + s * 4.0 * b4))) / T
    return rho, drho


def rho_exp(t):
    """Exponential growth of the data, eq. (grates)."""
    return math.exp(0.001 * t)


def rho_log(t):
    """Logistic growth of the data, eq. (grates), with the carrying factor
    exp(0.6) (the printed exp(0.006) gives rho(600) = 1.006, against the
    stated equal final sizes of both growth laws)."""
    e = math.exp(0.01 * t)
    return e / (1.0 + (e - 1.0) / math.exp(0.6))


def rho_exp_pair(t):
    """(rho_exp, rho_exp') for the data."""
    r = rho_exp(t)
    return r, 0.001 * r


def rho_log_pair(t):
    """(rho_log, rho_log') for the data: f = e / D with e = exp(0.01 t),
    D = 1 + (e - 1)/K, so f' = 0.01 e (1 - 1/K) / D^2."""
    K = math.exp(0.6)
    e = math.exp(0.01 * t)
    D = 1.0 + (e - 1.0) / K
    return e / D, 0.01 * e * (1.0 - 1.0 / K) / (D * D)


def initial_fields(n):
    """eq. (ic_gturing) on the cell centres x_i = (i + 1/2) / n."""
    x = (np.arange(n) + 0.5) / n
    s = sum(np.sin(k * math.pi * x) for k in range(1, 10))
    return 1.0 + 0.005 * s, 0.9 + 0.005 * s


def _tridiag(diag, c, n):
    """Banded form of diag - c Lap_h (mirror ghosts: the boundary rows have one
    neighbour); Lap_h x_i = (x_{i-1} - 2 x_i + x_{i+1}) n^2."""
    k = c * n * n
    ab = np.zeros((3, n))
    ab[0, 1:] = -k          # super-diagonal
    ab[2, :-1] = -k         # sub-diagonal
    nb = np.full(n, 2.0)
    nb[0] = nb[-1] = 1.0
    ab[1] = diag + k * nb
    return ab


def imex_step(theta, u, v, tau, rho, drho):
    """One step; theta = (a, b, gamma, d); rho, drho at t_n."""
    a, b, g, d = theta
    n = len(u)
    dil = drho / rho
    c = 1.0 / (rho * rho)
    du = 1.0 / tau + dil + g * (1.0 - u * v)
    dv = 1.0 / tau + dil + g * u * u
    un = solve_banded((1, 1), _tridiag(du, c, n), u / tau + g * a)
    vn = solve_banded((1, 1), _tridiag(dv, d * c, n), v / tau + g * b)
    return un, vn


def forward(theta, u0, v0, tau, n_steps, rho_fn):
    """Fields at T = n_steps tau; rho_fn(t) -> (rho, rho')."""
    u, v = np.array(u0, dtype=np.float64), np.array(v0, dtype=np.float64)
    for s in range(n_steps):
        rho, drho = rho_fn(s * tau)
        u, v = imex_step(theta, u, v, tau, rho, drho)
    return u, v


def forward_beta(theta, beta, rho_T, u0, v0, tau, n_steps):
    T = n_steps * tau
    return forward(theta, u0, v0, tau, n_steps, lambda t: rho_poly(beta, rho_T, T, t))


def misfit(y, u, sigma):
    """Phi = 1/2 sigma^-2 sum (y - u)^2 (Gaussian noise on u)."""
    r = np.asarray(y, dtype=np.float64) - np.asarray(u, dtype=np.float64)
    return 0.5 * float((r * r).sum()) / (sigma * sigma)


def growth_positive(beta, rho_T, tau, n_steps):
    """rho(t_k) > 0 at every step time t_k = k tau, k < n_steps (the growth
    function must stay positive; the step uses rho at t_k only)."""
    T = n_steps * tau
    return all(rho_poly(beta, rho_T, T, k * tau)[0] > 0.0 for k in range(n_steps))


def loglik_beta(theta, beta, rho_T, u0, v0, tau, n_steps, y, sigma, obs=1):
    """Phi(beta) with Gaussian noise on the observed rows of y = [y_u, y_v]
    (obs bit 0: u, bit 1: v); +inf where rho is not positive."""
    if not growth_positive(beta, rho_T, tau, n_steps):
        return math.inf
    u, v = forward_beta(theta, beta, rho_T, u0, v0, tau, n_steps)
    y = np.asarray(y, dtype=np.float64).reshape(2, -1)
    parts_y, parts_g = [], []
    if obs & 1:
        parts_y.append(y[0])
        parts_g.append(u)
    if obs & 2:
        parts_y.append(y[1])
        parts_g.append(v)
    return misfit(np.concatenate(parts_y), np.concatenate(parts_g), sigma)
