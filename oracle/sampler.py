"""Oracle Metropolis-Hastings and delayed-acceptance steps (FP64, CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 2, Algorithm 1: draw a proposal from a symmetric kernel k(x_k, .),
accept it with probability min(1, exp(Phi(x_k) - Phi(x_bar))), otherwise
stay.  Proposals are Gaussian random-walk steps in the sampling coordinates
phi = (a, b, ln gamma, ln d); the default prior is uniform on a box in phi,
so inside the box the prior ratio is 1 (the acceptance formula of Algorithm
1 is exact) and a proposal outside the box has zero posterior density and is
rejected without evaluating Phi.  The priors of Sec. 3.1.2 (Turing-space
support, Case 2; log-normal gamma and d, Case 3) add the prior ratio
pi(x_bar) / pi(x_k) to the acceptance probability (the general
Metropolis-Hastings ratio for a symmetric kernel).

Random numbers follow the sampler's counter-based contract (Philox4x32-10,
key = (chain, seed), counter = (step, purpose, block)):
purpose 0 = proposal normals, 1 = final accept uniform, 2 = first-stage
(surrogate) uniform.  Accept iff log U < log alpha.

The delayed-acceptance step (Christen and Fox, J. Comput. Graph. Stat. 14(4),
2005) screens a proposal with a cheap approximation Phi~ first:
  stage 1: accept iff log U1 < Phi~(x) - Phi~(y);
  stage 2 (only if stage 1 accepts): accept iff
           log U2 < [Phi(x) - Phi(y)] - [Phi~(x) - Phi~(y)],
which leaves the exact posterior invariant for a symmetric proposal.
"""
from __future__ import annotations

import math

import numpy as np

from . import normals4, normals4_at, uniform1, uniform_at

PURPOSE_PROPOSAL = 0
PURPOSE_ACCEPT = 1
PURPOSE_STAGE1 = 2
PURPOSE_PMH_AUX = 6       # parallel MH: the auxiliary point
PURPOSE_PMH_PROP = 7      # parallel MH: proposal j from blocks 2j, 2j + 1
PURPOSE_PMH_RESAMPLE = 8  # parallel MH: uniform of draw n from block n
PURPOSE_SUB_PROPOSAL = 9  # surrogate chain: normals of substep j >= 1 (blocks 2j, 2j + 1)
PURPOSE_SUB_ACCEPT = 10   # surrogate chain: uniform of substep j >= 1 (block j)


def propose(phi, seed, chain, step, step_sd, free_mask, chol=None):
    """phi' = phi + s .* z on the free coordinates (Algorithm 1, first step);
    with a lower-triangular factor L (4 x 4), phi' = phi + L z instead, row i
    summed over j = 0..i in that order."""
    z = normals4(seed, chain, step, PURPOSE_PROPOSAL)
    prop = np.array(phi, dtype=np.float64).copy()
    for i in range(4):
        if (free_mask >> i) & 1:
            if chol is not None:
                dz = 0.0
                for j in range(i + 1):
                    dz = dz + float(chol[i][j]) * float(z[j])
            else:
                dz = step_sd[i] * z[i]
            prop[i] = prop[i] + dz
    return prop


def in_box(phi, lo, hi) -> bool:
    return all(lo[i] <= phi[i] <= hi[i] for i in range(4))


# --------------------------------------------------------------------------
# Priors beyond the uniform box (Sec. 3.1.2, Cases 2-4)

class Prior:
    """Prior on the sampling coordinates phi = (a, b, ln gamma, ln d).

    kinds[i] = 0: uniform on [lo[i], hi[i]] (Case 1);
    kinds[i] = 1: normal N(mean[i], sd[i]^2) in phi_i, i.e. log-normal in
    gamma or d (Case 3), with no bound;
    turing: the support is also restricted to the Turing space of
    eq. (turing) at the homogeneous steady state, with d = exp(phi_3) (Case
    2: uniform on the Turing space)."""

    def __init__(self, kinds=(0, 0, 0, 0), mean=(0.0,) * 4, sd=(1.0,) * 4, turing=False):
        self.kinds = tuple(int(k) for k in kinds)
        self.mean = tuple(float(m) for m in mean)
        self.sd = tuple(float(x) for x in sd)
        self.turing = bool(turing)


def turing_space(a, b, d) -> bool:
    """The four inequalities of eq. (turing) for the activator-depleted
    kinetics at (u*, v*) = (a + b, b / (a + b)^2)."""
    s = a + b
    tr = (b - a) / s - s * s
    det = s * s
    dfg = d * ((b - a) / s) - s * s
    disc = dfg * dfg - 4.0 * d * det
    return tr < 0.0 and det > 0.0 and dfg > 0.0 and disc > 0.0


def prior_quad(phi, prior) -> float:
    """Sum over normal coordinates of (phi_i - mean_i)^2 / (2 sd_i^2), in
    index order: minus the log prior density up to a constant."""
    acc = 0.0
    for i in range(4):
        if prior.kinds[i] == 1:
            q = (float(phi[i]) - prior.mean[i]) / prior.sd[i]
            acc = acc + 0.5 * (q * q)
    return acc


def in_support(phi, lo, hi, prior=None) -> bool:
    """Zero prior density outside: the box on uniform coordinates, and the
    Turing space when the prior asks for it."""
    for i in range(4):
        if (prior is None or prior.kinds[i] == 0) and not (lo[i] <= phi[i] <= hi[i]):
            return False
    if prior is not None and prior.turing:
        return turing_space(float(phi[0]), float(phi[1]), math.exp(float(phi[3])))
    return True


def log_prior_ratio(phi, prop, prior=None) -> float:
    """log pi(prop) - log pi(phi) on the support (0 for the uniform prior)."""
    if prior is None or not any(k == 1 for k in prior.kinds):
        return 0.0
    return prior_quad(phi, prior) - prior_quad(prop, prior)


def rwm_step(phi, loglik, seed, chain, step, lo, hi, step_sd, free_mask, loglik_fn,
             prior=None, chol=None):
    """One step of Algorithm 1 for one chain; with a non-uniform prior the
    log acceptance ratio gains log pi(prop) - log pi(phi).

    Returns (phi_next, loglik_next, accepted, solved)."""
    prop = propose(phi, seed, chain, step, step_sd, free_mask, chol)
    if not in_support(prop, lo, hi, prior):
        return np.array(phi, dtype=np.float64), loglik, False, False
    ll_prop = float(loglik_fn(prop))
    u = uniform1(seed, chain, step, PURPOSE_ACCEPT)
    log_alpha = (loglik - ll_prop) + log_prior_ratio(phi, prop, prior)
    if math.log(u) < log_alpha:
        return prop, ll_prop, True, True
    return np.array(phi, dtype=np.float64), loglik, False, True


def rwm_batch_step(phis, logliks, seed, step, lo, hi, step_sd, free_mask, loglik_batch_fn,
                   prior=None, chol=None):
    """Algorithm 1 applied to every chain; loglik_batch_fn maps [m,4] -> [m].

    Returns (phis, logliks, accepted[bool], solved[bool])."""
    phis = np.array(phis, dtype=np.float64)
    logliks = np.array(logliks, dtype=np.float64)
    C = phis.shape[0]
    props = np.stack([propose(phis[c], seed, c, step, step_sd, free_mask, chol)
                      for c in range(C)])
    inside = np.array([in_support(props[c], lo, hi, prior) for c in range(C)])
    ll_prop = np.full(C, np.inf)
    if inside.any():
        ll_prop[inside] = loglik_batch_fn(props[inside])
    accepted = np.zeros(C, dtype=bool)
    for c in range(C):
        if not inside[c]:
            continue
        u = uniform1(seed, c, step, PURPOSE_ACCEPT)
        if math.log(u) < (logliks[c] - ll_prop[c]) + log_prior_ratio(phis[c], props[c], prior):
            accepted[c] = True
    phis[accepted] = props[accepted]
    logliks[accepted] = ll_prop[accepted]
    return phis, logliks, accepted, inside


def da_step(phi, loglik, loglik_sur, seed, chain, step, lo, hi, step_sd, free_mask,
            loglik_fn, surrogate_fn, prior=None):
    """One delayed-acceptance step for one chain.  The prior ratio enters
    the first stage (it cancels from the second).

    Returns (phi, loglik, loglik_sur, accepted1, accepted, solved)."""
    prop = propose(phi, seed, chain, step, step_sd, free_mask)
    keep = (np.array(phi, dtype=np.float64), loglik, loglik_sur)
    if not in_support(prop, lo, hi, prior):
        return (*keep, False, False, False)
    sur_prop = float(surrogate_fn(prop))
    u1 = uniform1(seed, chain, step, PURPOSE_STAGE1)
    if not math.log(u1) < (loglik_sur - sur_prop) + log_prior_ratio(phi, prop, prior):
        return (*keep, False, False, False)
    ll_prop = float(loglik_fn(prop))
    u2 = uniform1(seed, chain, step, PURPOSE_ACCEPT)
    log_alpha2 = (loglik - ll_prop) - (loglik_sur - sur_prop)
    if math.log(u2) < log_alpha2:
        return prop, ll_prop, sur_prop, True, True, True
    return (*keep, True, False, True)


def rw_move(x, z, step_sd, free_mask, chol=None):
    """x + s .* z, or x + L z, on the free coordinates (row i of L z summed
    over j = 0..i in that order)."""
    y = np.array(x, dtype=np.float64).copy()
    for i in range(4):
        if (free_mask >> i) & 1:
            if chol is not None:
                dz = 0.0
                for j in range(i + 1):
                    dz = dz + float(chol[i][j]) * float(z[j])
            else:
                dz = step_sd[i] * z[i]
            y[i] = y[i] + dz
    return y


def da_chain_step(phi, loglik, loglik_sur, seed, chain, step, m, lo, hi, step_sd, free_mask,
                  loglik_fn, surrogate_fn, prior=None, chol=None):
    """Delayed acceptance whose first stage is m Metropolis steps on the
    surrogate posterior (prior x exp(-Phi~)) from the present state x
    (Christen and Fox 2005 with the surrogate's own Markov kernel as the
    proposal, the surrogate transition of Liu, Monte Carlo Strategies in
    Scientific Computing, 2001).  Substep j proposes z' = z + s .* dz (or
    z + L dz) from the substep's state z and accepts it iff
    log U_j < [Phi~(z) - Phi~(z')] + [log pi(z') - log pi(z)]; the end point
    y of the m substeps is the proposal of the second stage, which accepts
    iff log U < [Phi(x) - Phi(y)] - [Phi~(x) - Phi~(y)] (the prior ratio
    cancels).  The surrogate kernel is reversible for the surrogate
    posterior, which makes the two-stage step reversible for the posterior.
    When no substep moves, y = x and nothing is solved.

    Random numbers: substep 0 uses the proposal normals (purpose 0) and the
    first-stage uniform (purpose 2) of the step, so that m = 1 is da_step;
    substep j >= 1 uses purpose 9 (blocks 2j, 2j + 1) and purpose 10
    (block j); the second stage purpose 1.

    Returns (phi, loglik, loglik_sur, moved1, accepted, solved): moved1 =
    the surrogate chain left x (the proposal reaches the second stage)."""
    z = np.array(phi, dtype=np.float64)
    lz = loglik_sur
    moves = 0
    for j in range(m):
        if j == 0:
            dz = normals4(seed, chain, step, PURPOSE_PROPOSAL)
            u = uniform1(seed, chain, step, PURPOSE_STAGE1)
        else:
            dz = normals4_at(seed, chain, step, PURPOSE_SUB_PROPOSAL, 2 * j)
            u = uniform_at(seed, chain, step, PURPOSE_SUB_ACCEPT, j)
        prop = rw_move(z, dz, step_sd, free_mask, chol)
        if not in_support(prop, lo, hi, prior):
            continue
        lp = float(surrogate_fn(prop))
        if math.log(u) < (lz - lp) + log_prior_ratio(z, prop, prior):
            z, lz = prop, lp
            moves += 1
    keep = (np.array(phi, dtype=np.float64), loglik, loglik_sur)
    if moves == 0:
        return (*keep, False, False, False)
    ll_prop = float(loglik_fn(z))
    u2 = uniform1(seed, chain, step, PURPOSE_ACCEPT)
    if math.log(u2) < (loglik - ll_prop) - (loglik_sur - lz):
        return z, ll_prop, lz, True, True, True
    return (*keep, True, False, True)


# --------------------------------------------------------------------------
# Parallel Metropolis-Hastings (Sec. 2, Algorithm 2)
#
# N proposals are evaluated at once, the acceptance probabilities of the
# N + 1 points (the N proposals and the present state x_k) are the
# stationary distribution of the transition matrix
#   A(i, j) = min(1, r(x_i, x_j)) / N  (j != i),  A(i, i) = 1 - sum_{j != i} A(i, j),
#   r(x, y) = exp(Phi(x) - Phi(y))  (times pi0(y) / pi0(x) for a non-uniform prior),
# and N draws from that distribution are the next N states.  As printed the
# proposals are drawn around x_k; here they are drawn around an auxiliary
# point z ~ k(x_k, .) (Calderhead, PNAS 111(49), 2014, the construction the
# algorithm cites), for which A with this r leaves the posterior invariant
# when k is symmetric.  The last draw is the present state of the next step.


def pmh_points(phi, seed, chain, step, n_prop, step_sd, free_mask, chol=None):
    """[n_prop + 1, 4]: row 0 the present state, rows 1..N the proposals
    (z = x_k + dz with normals of purpose 6; x_j = z + dz_j with normals of
    purpose 7, blocks 2(j-1), 2(j-1) + 1)."""

    def move(x, z):
        y = np.array(x, dtype=np.float64).copy()
        for i in range(4):
            if (free_mask >> i) & 1:
                if chol is not None:
                    dz = 0.0
                    for j in range(i + 1):
                        dz = dz + float(chol[i][j]) * float(z[j])
                else:
                    dz = step_sd[i] * z[i]
                y[i] = y[i] + dz
        return y

    aux = move(phi, normals4_at(seed, chain, step, PURPOSE_PMH_AUX, 0))
    pts = [np.array(phi, dtype=np.float64)]
    for j in range(n_prop):
        pts.append(move(aux, normals4_at(seed, chain, step, PURPOSE_PMH_PROP, 2 * j)))
    return np.stack(pts)


def pmh_matrix(logw):
    """A of Algorithm 2 from the log target densities of the N + 1 points
    (-inf outside the support): A(i, j) = min(1, w_j / w_i) / N."""
    logw = np.asarray(logw, dtype=np.float64)
    m = len(logw) - 1
    A = np.zeros((m + 1, m + 1))
    for i in range(m + 1):
        for j in range(m + 1):
            if j == i:
                continue
            if logw[i] == -np.inf:
                ratio = 1.0 if logw[j] > -np.inf else 0.0
            else:
                ratio = min(1.0, math.exp(min(0.0, logw[j] - logw[i])))
            A[i, j] = ratio / m
        A[i, i] = 1.0 - A[i].sum()
    return A


def stationary(A):
    """p with p A = p and sum p = 1 (one equation of (A^T - I) p = 0
    replaced by the normalisation, dense solve)."""
    n = A.shape[0]
    M = A.T - np.eye(n)
    M[-1, :] = 1.0
    rhs = np.zeros(n)
    rhs[-1] = 1.0
    return np.linalg.solve(M, rhs)


def pmh_draw(p, u) -> int:
    """Smallest index whose running sum of p (in index order) exceeds u."""
    acc = 0.0
    for i, pi in enumerate(p):
        acc = acc + pi
        if u < acc:
            return i
    return len(p) - 1 - int(np.argmax(np.asarray(p)[::-1] > 0))


def pmh_step(phi, loglik, seed, chain, step, n_prop, lo, hi, step_sd, free_mask, loglik_fn,
             prior=None, chol=None):
    """One step of Algorithm 2 for one chain.

    Returns (draws [N, 4], draw logliks [N], draw indices [N], points
    [N+1, 4], point logliks [N+1], stationary p [N+1]); the last draw is the
    next present state."""
    pts = pmh_points(phi, seed, chain, step, n_prop, step_sd, free_mask, chol)
    ll = np.full(n_prop + 1, np.inf)
    ll[0] = loglik
    for j in range(1, n_prop + 1):
        if in_support(pts[j], lo, hi, prior):
            ll[j] = float(loglik_fn(pts[j]))
    logw = -ll
    if prior is not None and any(k == 1 for k in prior.kinds):
        logw = np.array([logw[j] - prior_quad(pts[j], prior) for j in range(n_prop + 1)])
    if not np.any(np.isfinite(logw)):
        p = np.zeros(n_prop + 1)  # no point has positive density: stay
        idx = np.zeros(n_prop, dtype=np.int64)
    else:
        p = stationary(pmh_matrix(logw))
        idx = np.array([pmh_draw(p, uniform_at(seed, chain, step, PURPOSE_PMH_RESAMPLE, n))
                        for n in range(n_prop)])
    return pts[idx], ll[idx], idx, pts, ll, p
