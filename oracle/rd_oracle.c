/*
 * FP64 CPU oracle for the Schnakenberg Bayesian-identification hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header or constant table with
 * the HIP path.
 *
 * It is deliberately plain: every loop follows the definition in the paper
 * (Campillo-Funollet, Venkataraman, Madzvamuse, "A Bayesian approach to
 * parameter identification with an application to Turing systems") in the
 * order the paper states it, in double precision, with no blocking or fusion.
 *
 *   Sec. 3.1, eq. (schnakenberg), eq. (reactions): the reaction-diffusion
 *       system on a uniformly growing domain mapped to the unit square.
 *   Sec. 3.1.1, the IMEX "modified backward Euler" scheme with one Picard
 *       linearisation, 5-point Laplacian with Neumann conditions, linear
 *       systems solved with (unpreconditioned) conjugate gradients.
 *   Sec. 2, eq. (meas_model), eq. (logl): additive Gaussian noise model and
 *       the log-likelihood Phi = -log rho(y - G(p)).
 *   Sec. 2, Algorithm 1: one Metropolis-Hastings step.
 *
 * Readings taken where the paper is silent or garbled (each is listed in the
 * design notes): the v-equation's Laplacian acts on v (not u); the dilution
 * term keeps its factor m (= 2 on a 2-D domain); rho^{2n} means (rho^n)^2 and
 * rho, rho' are evaluated at t_n; the grid is cell-centred with mirror
 * ghosts; CG stops on the recursive residual ||r|| <= rtol ||b||.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NOT_CONVERGED 1
#define ORC_BREAKDOWN 2
#define ORC_NONFINITE 4

/* ------------------------------------------------------------------------ */
/* Grid and operator (Sec. 3.1.1: "standard 5-point stencil ... with Neumann
 * boundary conditions").  n x n cells on [0,1]^2, h = 1/n, cell (i,j) at
 * index j*n + i (i along x).  A zero-flux boundary is imposed with a mirror
 * ghost cell: w(-1,j) = w(0,j), w(n,j) = w(n-1,j), likewise in j.          */

void orc_laplacian(int n, const double *w, double *out)
{
    const double inv_h2 = (double)n * (double)n;
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            double c = w[j * n + i];
            double west = (i > 0) ? w[j * n + i - 1] : c;
            double east = (i < n - 1) ? w[j * n + i + 1] : c;
            double south = (j > 0) ? w[(j - 1) * n + i] : c;
            double north = (j < n - 1) ? w[(j + 1) * n + i] : c;
            out[j * n + i] = (west + east + south + north - 4.0 * c) * inv_h2;
        }
    }
}

/* out = sigma .* p - c * Lap_h p : the matrix of one implicit half-step. */
void orc_apply_A(int n, const double *sigma, double c, const double *p, double *out)
{
    int nn = n * n;
    double *lap = (double *)malloc(sizeof(double) * (size_t)nn);
    orc_laplacian(n, p, lap);
    for (int k = 0; k < nn; ++k)
        out[k] = sigma[k] * p[k] - c * lap[k];
    free(lap);
}

static double dot(int nn, const double *a, const double *b)
{
    double s = 0.0;
    for (int k = 0; k < nn; ++k)
        s += a[k] * b[k];
    return s;
}

/* Conjugate gradients (Hestenes-Stiefel, no preconditioner) for
 * (sigma I - c Lap_h) x = b, starting from the x passed in.
 * Stops when ||r||_2 <= rtol ||b||_2 with r the recursively updated residual,
 * or after maxit iterations (flag NOT_CONVERGED).  A non-positive curvature
 * p.Ap flags BREAKDOWN (the operator is not positive definite), a non-finite
 * value flags NONFINITE.  Returns the status bits; *iters gets the count.  */
int orc_cg(int n, const double *sigma, double c, const double *b, double *x,
           double rtol, int maxit, int *iters)
{
    int nn = n * n;
    int status = 0, it = 0;
    double *r = (double *)malloc(sizeof(double) * (size_t)nn);
    double *p = (double *)malloc(sizeof(double) * (size_t)nn);
    double *q = (double *)malloc(sizeof(double) * (size_t)nn);

    orc_apply_A(n, sigma, c, x, q);
    for (int k = 0; k < nn; ++k) {
        r[k] = b[k] - q[k];
        p[k] = r[k];
    }
    double bb = dot(nn, b, b);
    double rr = dot(nn, r, r);
    double tol2 = rtol * rtol * bb;
    if (!isfinite(bb) || !isfinite(rr))
        status |= ORC_NONFINITE;

    while (!status && rr > tol2) {
        if (it >= maxit) {
            status |= ORC_NOT_CONVERGED;
            break;
        }
        orc_apply_A(n, sigma, c, p, q);
        double pq = dot(nn, p, q);
        if (!isfinite(pq)) {
            status |= ORC_NONFINITE;
            break;
        }
        if (!(pq > 0.0)) {
            status |= ORC_BREAKDOWN;
            break;
        }
        double alpha = rr / pq;
        for (int k = 0; k < nn; ++k) {
            x[k] += alpha * p[k];
            r[k] -= alpha * q[k];
        }
        double rr_new = dot(nn, r, r);
        ++it;
        if (!isfinite(rr_new)) {
            status |= ORC_NONFINITE;
            break;
        }
        double beta = rr_new / rr;
        rr = rr_new;
        for (int k = 0; k < nn; ++k)
            p[k] = r[k] + beta * p[k];
    }
    free(r);
    free(p);
    free(q);
    if (iters)
        *iters = it;
    return status;
}

/* Direct solve of the same system for tiny grids (n <= 8): the n^2 x n^2
 * matrix is written out entry by entry from the stencil and factorised by
 * Gaussian elimination with partial pivoting.  Used to pin orc_cg.
 * Returns 0 on success, ORC_BREAKDOWN if a pivot vanishes.                */
int orc_dense_solve(int n, const double *sigma, double c, const double *b, double *x)
{
    int nn = n * n;
    double inv_h2 = (double)n * (double)n;
    double *M = (double *)calloc((size_t)nn * (size_t)nn, sizeof(double));
    double *rhs = (double *)malloc(sizeof(double) * (size_t)nn);
    for (int j = 0; j < n; ++j) {
        for (int i = 0; i < n; ++i) {
            int row = j * n + i;
            /* -c Lap_h: each existing neighbour contributes -c/h^2 off the
             * diagonal and +c/h^2 on it; a mirrored (missing) neighbour
             * contributes nothing (its ghost equals the centre value).   */
            M[(size_t)row * nn + row] += sigma[row];
            int nb[4][2] = {{i - 1, j}, {i + 1, j}, {i, j - 1}, {i, j + 1}};
            for (int s = 0; s < 4; ++s) {
                int ii = nb[s][0], jj = nb[s][1];
                if (ii < 0 || ii >= n || jj < 0 || jj >= n)
                    continue;
                M[(size_t)row * nn + row] += c * inv_h2;
                M[(size_t)row * nn + (jj * n + ii)] -= c * inv_h2;
            }
            rhs[row] = b[row];
        }
    }
    int status = 0;
    for (int col = 0; col < nn && !status; ++col) {
        int piv = col;
        for (int r = col + 1; r < nn; ++r)
            if (fabs(M[(size_t)r * nn + col]) > fabs(M[(size_t)piv * nn + col]))
                piv = r;
        if (M[(size_t)piv * nn + col] == 0.0) {
            status = ORC_BREAKDOWN;
            break;
        }
        if (piv != col) {
            for (int k = 0; k < nn; ++k) {
                double t = M[(size_t)col * nn + k];
                M[(size_t)col * nn + k] = M[(size_t)piv * nn + k];
                M[(size_t)piv * nn + k] = t;
            }
            double t = rhs[col];
            rhs[col] = rhs[piv];
            rhs[piv] = t;
        }
        for (int r = col + 1; r < nn; ++r) {
            double f = M[(size_t)r * nn + col] / M[(size_t)col * nn + col];
            for (int k = col; k < nn; ++k)
                M[(size_t)r * nn + k] -= f * M[(size_t)col * nn + k];
            rhs[r] -= f * rhs[col];
        }
    }
    if (!status) {
        for (int r = nn - 1; r >= 0; --r) {
            double s = rhs[r];
            for (int k = r + 1; k < nn; ++k)
                s -= M[(size_t)r * nn + k] * x[k];
            x[r] = s / M[(size_t)r * nn + r];
        }
    }
    free(M);
    free(rhs);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Growth of the domain (Sec. 3.1): x(t) = rho(t) x(0).  growth == 0 is the
 * stationary square (rho = 1); growth == 1 is rho(t) = exp(r t), for which
 * rho'/rho = r.  The dilution term of eq. (schnakenberg) is m rho'/rho with
 * m the space dimension, m = 2 here.                                       */
static void growth_at(int growth, double rate, double t, double *rho, double *rho_dot_over_rho)
{
    if (growth == 1) {
        *rho = exp(rate * t);
        *rho_dot_over_rho = rate;
    } else {
        *rho = 1.0;
        *rho_dot_over_rho = 0.0;
    }
}

/* One IMEX step (Sec. 3.1.1) from time level n to n+1, with the reaction
 * terms of eq. (reactions) linearised by one Picard iterate:
 *   [1/tau + m r_n + gamma (1 - u^n v^n)] u - rho_n^-2 Lap_h u = u^n/tau + gamma a
 *   [1/tau + m r_n + gamma (u^n)^2]       v - d rho_n^-2 Lap_h v = v^n/tau + gamma b
 * The two systems depend only on level n and are solved one after the other.
 * u, v hold level n on entry and n+1 on exit; iters[0..1] accumulate the CG
 * iteration counts.                                                         */
int orc_imex_step(int n, const double theta[4], int growth, double rate, double t_n,
                  double tau, double rtol, int maxit, double *u, double *v, int iters[2])
{
    const double a = theta[0], b = theta[1], gamma = theta[2], d = theta[3];
    const double m = 2.0;
    int nn = n * n;
    double rho, rdr;
    growth_at(growth, rate, t_n, &rho, &rdr);
    double inv_rho2 = 1.0 / (rho * rho);

    double *sig_u = (double *)malloc(sizeof(double) * (size_t)nn);
    double *sig_v = (double *)malloc(sizeof(double) * (size_t)nn);
    double *rhs_u = (double *)malloc(sizeof(double) * (size_t)nn);
    double *rhs_v = (double *)malloc(sizeof(double) * (size_t)nn);
    for (int k = 0; k < nn; ++k) {
        sig_u[k] = 1.0 / tau + m * rdr + gamma * (1.0 - u[k] * v[k]);
        sig_v[k] = 1.0 / tau + m * rdr + gamma * u[k] * u[k];
        rhs_u[k] = u[k] / tau + gamma * a;
        rhs_v[k] = v[k] / tau + gamma * b;
    }
    int it_u = 0, it_v = 0;
    int status = orc_cg(n, sig_u, inv_rho2, rhs_u, u, rtol, maxit, &it_u);
    if (!status)
        status |= orc_cg(n, sig_v, d * inv_rho2, rhs_v, v, rtol, maxit, &it_v);
    if (iters) {
        iters[0] += it_u;
        iters[1] += it_v;
    }
    free(sig_u);
    free(sig_v);
    free(rhs_u);
    free(rhs_v);
    return status;
}

/* Forward map G(theta) (Sec. 2, the observation operator): integrate from
 * the fixed initial fields (u0, v0) over n_steps steps of size tau.  On exit
 * u_out, v_out hold the fields at T = n_steps * tau (or at the step where a
 * solve failed).  Returns status bits; iters[0..1] get total CG iterations. */
int orc_forward_solve(int n, const double theta[4], int growth, double rate, double tau,
                      int n_steps, double rtol, int maxit, const double *u0, const double *v0,
                      double *u_out, double *v_out, int iters[2])
{
    int nn = n * n;
    memcpy(u_out, u0, sizeof(double) * (size_t)nn);
    memcpy(v_out, v0, sizeof(double) * (size_t)nn);
    if (iters) {
        iters[0] = 0;
        iters[1] = 0;
    }
    int status = 0;
    for (int s = 0; s < n_steps && !status; ++s)
        status = orc_imex_step(n, theta, growth, rate, s * tau, tau, rtol, maxit, u_out, v_out, iters);
    if (!status) {
        for (int k = 0; k < nn; ++k)
            if (!isfinite(u_out[k]) || !isfinite(v_out[k])) {
                status |= ORC_NONFINITE;
                break;
            }
    }
    return status;
}

/* Gaussian misfit, eq. (logl) with rho the density of N(0, sigma^2 I):
 * Phi = 1/(2 sigma^2) sum_k (y_k - u_k)^2 (constant term dropped: only
 * differences of Phi enter the sampler, Sec. 2).                           */
double orc_misfit(int n_obs, const double *y, const double *u, double sigma)
{
    double s = 0.0;
    for (int k = 0; k < n_obs; ++k) {
        double e = y[k] - u[k];
        s += e * e;
    }
    return 0.5 * s / (sigma * sigma);
}

/* Phi for a batch of parameter vectors (independent solves, one per thread
 * when built with OpenMP).  theta is [n_theta][4] natural parameters
 * (a, b, gamma, d).  A failed solve gives Phi = +inf (its status is kept).  */
void orc_loglik_batch(int n_theta, const double *theta, int n, int growth, double rate,
                      double tau, int n_steps, double rtol, int maxit, const double *u0,
                      const double *v0, const double *y, double sigma, double *phi,
                      int *status, int *iters)
{
    int nn = n * n;
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < n_theta; ++c) {
        double *u = (double *)malloc(sizeof(double) * (size_t)nn);
        double *v = (double *)malloc(sizeof(double) * (size_t)nn);
        int it[2] = {0, 0};
        int st = orc_forward_solve(n, theta + 4 * c, growth, rate, tau, n_steps, rtol, maxit, u0,
                                   v0, u, v, it);
        phi[c] = st ? INFINITY : orc_misfit(nn, y, u, sigma);
        if (status)
            status[c] = st;
        if (iters) {
            iters[2 * c] = it[0];
            iters[2 * c + 1] = it[1];
        }
        free(u);
        free(v);
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): ten rounds of the 4x32 Philox S-box with
 * multipliers 0xD2511F53, 0xCD9E8D57 and key schedule increments
 * 0x9E3779B9, 0xBB67AE85.                                                   */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0;
        c1 = n1;
        c2 = n2;
        c3 = n3;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* A double in (0,1) from two 32-bit words: the top 52 bits k of (hi:lo)
 * give U = (k + 1/2) 2^-52, which is exact in binary64.                   */
double orc_uniform_from_words(uint32_t hi, uint32_t lo)
{
    uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)k + 0.5) * 0x1p-52;
}

/* The sampler's random-number contract: key = (chain, seed), counter =
 * (step low word, step high word, purpose, block).                         */
static void stream_words(uint32_t seed, uint32_t chain, uint64_t step, uint32_t purpose,
                         uint32_t block, uint32_t w[4])
{
    uint32_t ctr[4] = {(uint32_t)step, (uint32_t)(step >> 32), purpose, block};
    uint32_t key[2] = {chain, seed};
    orc_philox4x32_10(ctr, key, w);
}

/* Four standard normals by the Box-Muller transform on two Philox blocks. */
void orc_normals4(uint32_t seed, uint32_t chain, uint64_t step, uint32_t purpose, double z[4])
{
    for (uint32_t blk = 0; blk < 2; ++blk) {
        uint32_t w[4];
        stream_words(seed, chain, step, purpose, blk, w);
        double u1 = orc_uniform_from_words(w[0], w[1]);
        double u2 = orc_uniform_from_words(w[2], w[3]);
        double rad = sqrt(-2.0 * log(u1));
        double ang = 6.283185307179586476925286766559 * u2; /* 2 pi */
        z[2 * blk] = rad * cos(ang);
        z[2 * blk + 1] = rad * sin(ang);
    }
}

/* One uniform in (0,1) from block 0 of the stream. */
double orc_uniform1(uint32_t seed, uint32_t chain, uint64_t step, uint32_t purpose)
{
    uint32_t w[4];
    stream_words(seed, chain, step, purpose, 0, w);
    return orc_uniform_from_words(w[0], w[1]);
}

/* Four uniforms in (0,1) (two per block). */
void orc_uniforms4(uint32_t seed, uint32_t chain, uint64_t step, uint32_t purpose, double uo[4])
{
    for (uint32_t blk = 0; blk < 2; ++blk) {
        uint32_t w[4];
        stream_words(seed, chain, step, purpose, blk, w);
        uo[2 * blk] = orc_uniform_from_words(w[0], w[1]);
        uo[2 * blk + 1] = orc_uniform_from_words(w[2], w[3]);
    }
}

/* Four standard normals from blocks blk0 and blk0 + 1 of a stream (the
 * draws of orc_normals4 when blk0 = 0). */
void orc_normals4_at(uint32_t seed, uint32_t chain, uint64_t step, uint32_t purpose, uint32_t blk0,
                     double z[4])
{
    for (uint32_t b = 0; b < 2; ++b) {
        uint32_t w[4];
        stream_words(seed, chain, step, purpose, blk0 + b, w);
        double u1 = orc_uniform_from_words(w[0], w[1]);
        double u2 = orc_uniform_from_words(w[2], w[3]);
        double rad = sqrt(-2.0 * log(u1));
        double ang = 6.283185307179586476925286766559 * u2; /* 2 pi */
        z[2 * b] = rad * cos(ang);
        z[2 * b + 1] = rad * sin(ang);
    }
}

/* One uniform in (0,1) from block blk of a stream. */
double orc_uniform_at(uint32_t seed, uint32_t chain, uint64_t step, uint32_t purpose, uint32_t blk)
{
    uint32_t w[4];
    stream_words(seed, chain, step, purpose, blk, w);
    return orc_uniform_from_words(w[0], w[1]);
}
