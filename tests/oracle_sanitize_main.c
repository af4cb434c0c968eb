/* Drives the C oracle through every exported routine on small inputs so that
 * a build with AddressSanitizer and UndefinedBehaviorSanitizer can check its
 * memory accesses and arithmetic (tests/test_oracle_sanitized.py).  Prints
 * the status of each call; exits non-zero if a call returns an unexpected
 * status.  Test infrastructure: links only oracle/rd_oracle.c. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_laplacian(int n, const double *w, double *out);
void orc_apply_A(int n, const double *sigma, double c, const double *p, double *out);
int orc_cg(int n, const double *sigma, double c, const double *b, double *x, double rtol,
           int maxit, int *iters);
int orc_dense_solve(int n, const double *sigma, double c, const double *b, double *x);
int orc_forward_solve(int n, const double theta[4], int growth, double rate, double tau,
                      int n_steps, double rtol, int maxit, const double *u0, const double *v0,
                      double *u_out, double *v_out, int iters[2]);
double orc_misfit(int n_obs, const double *y, const double *u, double sigma);
void orc_loglik_batch(int n_theta, const double *theta, int n, int growth, double rate,
                      double tau, int n_steps, double rtol, int maxit, const double *u0,
                      const double *v0, const double *y, double sigma, double *phi, int *status,
                      int *iters);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void orc_normals4(uint32_t seed, uint32_t chain, uint64_t step, uint32_t purpose, double z[4]);
double orc_uniform1(uint32_t seed, uint32_t chain, uint64_t step, uint32_t purpose);

int main(void)
{
    enum { N = 12, NN = N * N, STEPS = 5, M = 3 };
    double *u0 = malloc(sizeof(double) * NN), *v0 = malloc(sizeof(double) * NN);
    double *u = malloc(sizeof(double) * NN), *v = malloc(sizeof(double) * NN);
    double *w = malloc(sizeof(double) * NN), *x = malloc(sizeof(double) * NN);
    double *x2 = malloc(sizeof(double) * NN), *sig = malloc(sizeof(double) * NN);
    int bad = 0;
    for (int k = 0; k < NN; ++k) {
        u0[k] = 1.0 + 0.01 * sin(0.7 * k);
        v0[k] = 0.9 + 0.01 * cos(1.3 * k);
        sig[k] = 4000.0 + (k % 5);
    }
    orc_laplacian(N, u0, w);
    orc_apply_A(N, sig, 100.0, u0, w);
    int it = 0;
    bad |= orc_cg(N, sig, 100.0, w, x, 1e-12, 10 * NN, &it) != 0;
    bad |= orc_dense_solve(N, sig, 100.0, w, x2) != 0;
    double e = 0.0;
    for (int k = 0; k < NN; ++k)
        e = fmax(e, fabs(x[k] - u0[k]) + fabs(x2[k] - u0[k]));
    bad |= !(e < 1e-8);
    const double theta[4 * M] = {0.1, 0.9, 200.0, 10.0, 0.2, 0.8, 100.0, 20.0,
                                 0.05, 1.0, 400.0, 8.0};
    int iters[2];
    for (int g = 0; g < 2; ++g)
        bad |= orc_forward_solve(N, theta, g, 0.01, 2.5e-4, STEPS, 1e-10, 10 * NN, u0, v0, u, v,
                                 iters) != 0;
    double phi[M];
    int st[M], its[2 * M];
    orc_loglik_batch(M, theta, N, 0, 0.0, 2.5e-4, STEPS, 1e-10, 10 * NN, u0, v0, u, 0.01, phi,
                     st, its);
    for (int c = 0; c < M; ++c)
        bad |= st[c] != 0 || !isfinite(phi[c]);
    bad |= !(orc_misfit(NN, u, u, 0.1) == 0.0);
    uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6}, out[4];
    orc_philox4x32_10(ctr, key, out);
    double z[4];
    orc_normals4(7, 3, 123456789012ull, 0, z);
    const double uu = orc_uniform1(7, 3, 123456789012ull, 1);
    bad |= !(uu > 0.0 && uu < 1.0) || !isfinite(z[0] + z[1] + z[2] + z[3]);
    printf("cg %d iterations, dense/CG error %.3g, phi %.6g %.6g %.6g, bad %d\n", it, e, phi[0],
           phi[1], phi[2], bad);
    free(u0), free(v0), free(u), free(v), free(w), free(x), free(x2), free(sig);
    return bad;
}
