/*
 * rdbayes growth1d — identification of the growth function rho(t) of a
 * one-dimensional uniformly growing domain (Sec. 3.1.2, Example 1).
 *
 * Model: eq. (schnakenberg) with m = 1 and the kinetics of eq. (reactions),
 * a, b, gamma, d fixed, on the unit interval mapped from the growing domain
 * x(t) = rho(t) x(0).  Discretisation (Sec. 3.1.1 with m = 1): n cells,
 * h = 1/n, cell centres, mirror (zero-flux) ghosts, 3-point Laplacian, and
 * the IMEX backward-Euler step with one Picard linearisation and rho, rho'
 * taken at t_k = k tau:
 *   [1/tau + rho'/rho + g (1 - u v)] u' - rho^-2 Lap_h u' = u/tau + g a
 *   [1/tau + rho'/rho + g u^2]       v' - d rho^-2 Lap_h v' = v/tau + g b
 * (g = gamma; the printed scheme has Lap_h u' in the second equation, read
 * here as Lap_h v' as in the continuous system).  Each step is two
 * tridiagonal systems, solved on the GPU by parallel cyclic reduction in
 * float64; the fields are float64 throughout.
 *
 * Growth laws: G1D_LAW_POLY, the degree-4 polynomial in s = t / T with
 * rho(0) = 1 and rho(T) = rho_T fixed, so that three coefficients
 * beta = (beta_1, beta_2, beta_3) are free (the finite-dimensional
 * approximation of Example 1):
 *   rho = 1 + beta_1 s + beta_2 s^2 + beta_3 s^3 + beta_4 s^4,
 *   beta_4 = rho_T - 1 - beta_1 - beta_2 - beta_3,   T = n_steps tau;
 * G1D_LAW_EXP and G1D_LAW_LOGISTIC, the two laws that generate the data in
 * eq. (grates): exp(0.001 t) and e / (1 + (e - 1) / exp(0.6)), e = exp(0.01 t)
 * (the carrying factor is read as exp(0.6), for which both laws reach the
 * same size at T = 600 as the text states; the printed exp(0.006) would stop
 * the logistic law at 1.006).
 * A polynomial that is not positive at some t_k (the growth function must
 * stay positive) gives status RD_ST_OUT_OF_PRIOR and Phi = +inf.
 *
 * Likelihood: Gaussian noise of standard deviation sigma on the observed
 * components at T: Phi = 1/2 sigma^-2 sum over observed rows of (y - G)^2.
 *
 * Conventions (errors, device/host arrays, streams) are those of
 * rdbayes.h.  Limits: 2 <= n <= 128.
 */
#ifndef RDBAYES_GROWTH1D_H
#define RDBAYES_GROWTH1D_H

#include <stdint.h>

#include "rdbayes.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { G1D_LAW_POLY = 0, G1D_LAW_EXP = 1, G1D_LAW_LOGISTIC = 2 };
enum { G1D_MAX_N = 128 };

typedef struct g1d_problem g1d_problem; /* opaque; owned by the library */

typedef struct {
    int32_t n;            /* cells on the unit interval, 2 <= n <= 128 */
    int32_t n_steps;      /* IMEX steps; T = n_steps * tau */
    double tau;           /* time step */
    double theta[4];      /* a, b, gamma, d */
    int32_t law;          /* G1D_LAW_* */
    double rho_T;         /* rho(T) of the polynomial law (> 0) */
    const double *u0;     /* host [n] initial u on the cell centres */
    const double *v0;     /* host [n] initial v */
    const double *y;      /* host [2][n] data at T (row 0: u, row 1: v), or NULL */
    int32_t obs;          /* observed rows: bit 0 = u, bit 1 = v (nonzero with y) */
    double sigma;         /* noise standard deviation (> 0 with y) */
    int32_t max_batch;    /* largest item count of one call, >= 1 */
    /* Metropolis sampler over beta (Sec. 2, Algorithm 1): the chain state
     * is the float64 4-vector (beta_1, beta_2, beta_3, unused); proposals
     * beta' = beta + step .* z on the three coefficients; prior per
     * coefficient uniform on [lo, hi] or normal (RD_PRIOR_*), and always
     * restricted to positive rho. */
    double lo[3], hi[3], step[3];
    int32_t prior_kind[3];
    double prior_mean[3], prior_sd[3];
} g1d_desc;

/* Creates a problem: copies u0, v0 and y to the device and allocates the
 * sampler workspace for max_batch items.  Errors: RD_EINVAL (a field out of
 * range or a required pointer NULL), RD_ENOMEM, RD_EHIP. */
int32_t g1d_init(const g1d_desc *desc, g1d_problem **out);
int32_t g1d_destroy(g1d_problem *p);

/* Fields at T of n items.  beta dev float64 [n][3] (G1D_LAW_POLY; ignored,
 * may be NULL, for the data laws); u, v dev float64 [n][n_cells]; status dev
 * int32 [n] (RD_ST_* flags) or NULL.  Errors: RD_EINVAL. */
int32_t g1d_forward_batch(g1d_problem *p, int32_t n, const double *beta, double *u, double *v,
                          int32_t *status, void *stream);

/* Fused solve + misfit: phi dev float64 [n] (Phi, +inf for a failed or
 * non-positive-growth item), status dev int32 [n] or NULL.  Needs y.
 * Errors: RD_EINVAL. */
int32_t g1d_log_likelihood_batch(g1d_problem *p, int32_t n, const double *beta, double *phi,
                                 int32_t *status, void *stream);

/* n_steps Metropolis steps of chains over beta with the fused 1-D solve:
 * proposal, accept test and random numbers as in mcmc_step_batch (purposes
 * 0 and 1), the prior box or normal prior of the description; chains->phi
 * holds the 4-vectors above, grid_id, loglik_sur, n_accept1 and cg_iters
 * are not used.  Needs y and G1D_LAW_POLY.  Errors: RD_EINVAL. */
int32_t g1d_mcmc_step_batch(g1d_problem *p, rd_chains *chains, int32_t n_steps, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RDBAYES_GROWTH1D_H */
