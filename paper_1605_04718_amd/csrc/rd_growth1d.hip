// One-dimensional growing domain (Sec. 3.1.2, Example 1): batched float64
// IMEX solves with a growth function rho(t), the misfit at T, and the C ABI
// of include/rdbayes_growth1d.h.
//
// One wavefront per item.  Lane L owns rows L and L + 64 of both tridiagonal
// systems (u and v), so n <= 128 cells fit one wave; rows past n are
// identity rows (a = c = 0, b = 1, d = 0) that no real row couples to.
// Parallel cyclic reduction: at stride s every row eliminates its couplings
// to rows i - s and i + s with those rows' equations, which leaves
// couplings at stride 2s.  For n <= 64 the levels run until each row stands
// alone (x_i = d_i / b_i); for n > 64 they stop after stride 32, where row i
// couples only to i +- 64, so rows L and L + 64 form a 2 x 2 system inside
// lane L and the last level needs no exchange.  Every row publishes
// (a/b, c/b, d/b) once per level (one reciprocal per row and level) in LDS,
// laid out [system][component][row] so that a wave's accesses are
// consecutive.  The fields stay in registers
// for the whole horizon; only the data and the results touch HBM.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime.h>

#include "../../include/rdbayes_growth1d.h"
#include "rd_sampler.hpp"

namespace rd {
namespace g1d {

constexpr int kRows = 128;  // rows per system, two per lane

struct Args {
    int n, n_steps, law, obs;
    double inv_tau, tau, T, rho_T;
    double a, b, g, d;
    double inv_2s2;           // 1 / (2 sigma^2)
    const double *u0, *v0;    // [n]
    const double *y;          // [2][n] or null
    const double *beta;       // [m][beta_stride] (polynomial law)
    int beta_stride;
    const int *need;          // [m] or null: 0 = do not solve
    int m;
    double *u_out, *v_out;    // [m][n] or null
    double *phi;              // [m] or null
    int *status;              // [m] or null
};

// rho(t) and rho'(t).  Polynomial: Horner in s = t / T with beta_4 fixed by
// rho(T) = rho_T; the data laws of eq. (grates).
__device__ inline void growth(const Args &a, double b1, double b2, double b3, double b4, double t,
                              double &rho, double &drho)
{
    if (a.law == G1D_LAW_POLY) {
        const double s = t / a.T;
        rho = 1.0 + s * (b1 + s * (b2 + s * (b3 + s * b4)));
        drho = (b1 + s * (2.0 * b2 + s * (3.0 * b3 + s * 4.0 * b4))) / a.T;
    } else if (a.law == G1D_LAW_EXP) {
        rho = exp(0.001 * t);
        drho = 0.001 * rho;
    } else {
        const double K = exp(0.6);
        const double e = exp(0.01 * t);
        const double D = 1.0 + (e - 1.0) / K;
        rho = e / D;
        drho = 0.01 * e * (1.0 - 1.0 / K) / (D * D);
    }
}

struct Row {
    double A, B, C, D;
};

// 1/x from the hardware estimate refined by two Newton steps (e = 1 - x r,
// r <- r + r e); each step squares the relative error, so the result is
// within an ulp or two for the positive, well-scaled pivots of these
// diagonally dominant systems.
__device__ inline double recip(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
}

// One reduction level at stride s for the four rows a lane owns.
// P[sys][comp][row] holds (A/B, C/B, D/B) of every row of the level.
__device__ inline void pcr_level(Row (&r)[2][2], double (*P)[3][kRows], int lane, int s)
{
#pragma unroll
    for (int sys = 0; sys < 2; ++sys)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = lane + 64 * j;
            const double rb = recip(r[sys][j].B);
            P[sys][0][i] = r[sys][j].A * rb;
            P[sys][1][i] = r[sys][j].C * rb;
            P[sys][2][i] = r[sys][j].D * rb;
        }
    __syncthreads();
    Row nr[2][2];
#pragma unroll
    for (int sys = 0; sys < 2; ++sys)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = lane + 64 * j;
            double am = 0.0, cm = 0.0, dm = 0.0, ap = 0.0, cp = 0.0, dp = 0.0;
            if (i - s >= 0) {
                am = P[sys][0][i - s];
                cm = P[sys][1][i - s];
                dm = P[sys][2][i - s];
            }
            if (i + s < kRows) {
                ap = P[sys][0][i + s];
                cp = P[sys][1][i + s];
                dp = P[sys][2][i + s];
            }
            const Row &q = r[sys][j];
            nr[sys][j].A = -q.A * am;
            nr[sys][j].C = -q.C * cp;
            nr[sys][j].B = q.B - q.A * cm - q.C * ap;
            nr[sys][j].D = q.D - q.A * dm - q.C * dp;
        }
    __syncthreads();  // every read of this level precedes the next level's writes
#pragma unroll
    for (int sys = 0; sys < 2; ++sys)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            r[sys][j] = nr[sys][j];
}

__device__ inline double wave_sum(double x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1)
        x += __shfl_xor(x, o, 64);
    return x;
}

__global__ __launch_bounds__(64) void k_g1d_solve(Args a)
{
    __shared__ double P[2][3][kRows];
    const int lane = threadIdx.x;
    const int item = blockIdx.x;
    if (item >= a.m)
        return;
    const int n = a.n;
    int st = 0;
    double u[2], v[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = lane + 64 * j;
        u[j] = i < n ? a.u0[i] : 0.0;
        v[j] = i < n ? a.v0[i] : 0.0;
    }
    double b1 = 0.0, b2 = 0.0, b3 = 0.0, b4 = 0.0;
    if (a.law == G1D_LAW_POLY) {
        const double *bp = a.beta + (size_t)item * a.beta_stride;
        b1 = bp[0];
        b2 = bp[1];
        b3 = bp[2];
        b4 = a.rho_T - 1.0 - b1 - b2 - b3;
    }
    if (a.need && !a.need[item])
        st = RD_ST_OUT_OF_PRIOR;
    const double nn = (double)n * (double)n;
    for (int k = 0; k < a.n_steps && st == 0; ++k) {
        double rho, drho;
        growth(a, b1, b2, b3, b4, (double)k * a.tau, rho, drho);
        if (!(rho > 0.0)) {
            st = RD_ST_OUT_OF_PRIOR;  // uniform over the wave: rho depends on t only
            break;
        }
        const double dil = drho / rho;
        const double ku = nn / (rho * rho);
        const double kv = a.d * ku;
        Row r[2][2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int i = lane + 64 * j;
            if (i < n) {
                const double nb = (i == 0 || i == n - 1) ? 1.0 : 2.0;
                r[0][j].A = i > 0 ? -ku : 0.0;
                r[0][j].C = i < n - 1 ? -ku : 0.0;
                r[0][j].B = a.inv_tau + dil + a.g * (1.0 - u[j] * v[j]) + ku * nb;
                r[0][j].D = u[j] * a.inv_tau + a.g * a.a;
                r[1][j].A = i > 0 ? -kv : 0.0;
                r[1][j].C = i < n - 1 ? -kv : 0.0;
                r[1][j].B = a.inv_tau + dil + a.g * u[j] * u[j] + kv * nb;
                r[1][j].D = v[j] * a.inv_tau + a.g * a.b;
            } else {
                r[0][j] = Row{0.0, 1.0, 0.0, 0.0};
                r[1][j] = Row{0.0, 1.0, 0.0, 0.0};
            }
        }
        const int s_end = n > 64 ? 64 : n;
        for (int s = 1; s < s_end; s <<= 1)
            pcr_level(r, P, lane, s);
        if (n > 64) {
            // rows p = lane and q = lane + 64: B_p x_p + C_p x_q = D_p,
            // A_q x_p + B_q x_q = D_q (the outward couplings are zero)
            double x[2][2];
#pragma unroll
            for (int sys = 0; sys < 2; ++sys) {
                const Row &p = r[sys][0], &q = r[sys][1];
                const double inv = recip(p.B * q.B - p.C * q.A);
                x[sys][0] = (p.D * q.B - p.C * q.D) * inv;
                x[sys][1] = (p.B * q.D - q.A * p.D) * inv;
            }
            u[0] = x[0][0];
            u[1] = x[0][1];
            v[0] = x[1][0];
            v[1] = x[1][1];
        } else {
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                u[j] = r[0][j].D * recip(r[0][j].B);
                v[j] = r[1][j].D * recip(r[1][j].B);
            }
        }
    }
    double acc = 0.0;
    bool finite = true;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
        const int i = lane + 64 * j;
        if (i < n) {
            finite = finite && isfinite(u[j]) && isfinite(v[j]);
            if (a.u_out) {
                a.u_out[(size_t)item * n + i] = u[j];
                a.v_out[(size_t)item * n + i] = v[j];
            }
            if (a.y) {
                if (a.obs & 1) {
                    const double e = a.y[i] - u[j];
                    acc += e * e;
                }
                if (a.obs & 2) {
                    const double e = a.y[n + i] - v[j];
                    acc += e * e;
                }
            }
        }
    }
    if (st == 0 && __any(!finite))
        st = RD_ST_NONFINITE;
    acc = wave_sum(acc);
    if (lane == 0) {
        if (a.status)
            a.status[item] = st;
        if (a.phi)
            a.phi[item] = st == 0 ? acc * a.inv_2s2 : INFINITY;
    }
}

hipError_t launch_solve(const Args &a, hipStream_t s)
{
    if (a.m <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_g1d_solve, dim3(a.m), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace g1d
}  // namespace rd

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

using namespace rd;

extern "C" int32_t rd_set_error(int32_t code, const char *msg);

namespace {

int32_t fail(int32_t code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return rd_set_error(code, buf);
}

#define G1D_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(RD_EHIP, "%s: %s", #expr, hipGetErrorString(e_));              \
    } while (0)

}  // namespace

struct g1d_problem {
    g1d_desc desc{};
    int device = 0;
    double *u0 = nullptr, *v0 = nullptr, *y = nullptr;
    uint64_t *ctr = nullptr;      // [2] sampler step counter, step of trace row 0
    double *phi_prop = nullptr;   // [max][4]
    int *inside = nullptr;        // [max]
    double *ll_prop = nullptr;    // [max]
    int *status = nullptr;        // [max]
};

namespace {

g1d::Args base_args(const g1d_problem *p)
{
    const g1d_desc &d = p->desc;
    g1d::Args a{};
    a.n = d.n;
    a.n_steps = d.n_steps;
    a.law = d.law;
    a.obs = d.obs;
    a.tau = d.tau;
    a.inv_tau = 1.0 / d.tau;
    a.T = (double)d.n_steps * d.tau;
    a.rho_T = d.rho_T;
    a.a = d.theta[0];
    a.b = d.theta[1];
    a.g = d.theta[2];
    a.d = d.theta[3];
    a.inv_2s2 = p->y ? 1.0 / (2.0 * d.sigma * d.sigma) : 0.0;
    a.u0 = p->u0;
    a.v0 = p->v0;
    a.y = p->y;
    a.beta_stride = 3;
    return a;
}

void release(g1d_problem *p)
{
    hipFree(p->u0);
    hipFree(p->v0);
    hipFree(p->y);
    hipFree(p->ctr);
    hipFree(p->phi_prop);
    hipFree(p->inside);
    hipFree(p->ll_prop);
    hipFree(p->status);
}

int32_t check_batch(const g1d_problem *p, int32_t n, const double *beta)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (n < 0 || n > p->desc.max_batch)
        return fail(RD_EINVAL, "n = %d outside [0, max_batch = %d]", n, p->desc.max_batch);
    if (n > 0 && p->desc.law == G1D_LAW_POLY && !beta)
        return fail(RD_EINVAL, "beta is required with the polynomial growth law");
    return RD_OK;
}

}  // namespace

extern "C" int32_t g1d_init(const g1d_desc *d, g1d_problem **out)
{
    if (!d || !out)
        return fail(RD_EINVAL, "desc and out are required");
    *out = nullptr;
    if (d->n < 2 || d->n > G1D_MAX_N)
        return fail(RD_EINVAL, "n = %d outside [2, %d]", d->n, G1D_MAX_N);
    if (d->n_steps < 0 || !(d->tau > 0.0) || !isfinite(d->tau))
        return fail(RD_EINVAL, "n_steps must be >= 0 and tau > 0");
    if (d->law < G1D_LAW_POLY || d->law > G1D_LAW_LOGISTIC)
        return fail(RD_EINVAL, "law %d unknown", d->law);
    if (d->law == G1D_LAW_POLY && !(d->rho_T > 0.0))
        return fail(RD_EINVAL, "rho_T must be > 0");
    for (int i = 0; i < 4; ++i)
        if (!isfinite(d->theta[i]))
            return fail(RD_EINVAL, "theta must be finite");
    if (!d->u0 || !d->v0)
        return fail(RD_EINVAL, "u0 and v0 are required");
    if (d->y && ((d->obs & 3) == 0 || (d->obs & ~3) != 0 || !(d->sigma > 0.0)))
        return fail(RD_EINVAL, "with data, obs must be 1, 2 or 3 and sigma > 0");
    if (d->max_batch < 1)
        return fail(RD_EINVAL, "max_batch must be >= 1");
    for (int i = 0; i < 3; ++i) {
        if (d->prior_kind[i] != RD_PRIOR_UNIFORM && d->prior_kind[i] != RD_PRIOR_NORMAL)
            return fail(RD_EINVAL, "prior_kind[%d] unknown", i);
        if (d->prior_kind[i] == RD_PRIOR_NORMAL && !(d->prior_sd[i] > 0.0))
            return fail(RD_EINVAL, "prior_sd[%d] must be > 0", i);
        if (d->prior_kind[i] == RD_PRIOR_UNIFORM && !(d->lo[i] <= d->hi[i]))
            return fail(RD_EINVAL, "lo[%d] > hi[%d]", i, i);
        if (!(d->step[i] >= 0.0))
            return fail(RD_EINVAL, "step[%d] must be >= 0", i);
    }
    int device = 0;
    G1D_TRY(hipGetDevice(&device));
    g1d_problem *p = new g1d_problem;
    p->desc = *d;
    p->desc.u0 = p->desc.v0 = p->desc.y = nullptr;  // host arrays are read during the call only
    p->device = device;
    const size_t n = (size_t)d->n, mb = (size_t)d->max_batch;
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = hipMalloc(&p->u0, n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->v0, n * sizeof(double));
    if (e == hipSuccess && d->y) e = hipMalloc(&p->y, 2 * n * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->ctr, 2 * sizeof(uint64_t));
    if (e == hipSuccess) e = hipMalloc(&p->phi_prop, 4 * mb * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->inside, mb * sizeof(int));
    if (e == hipSuccess) e = hipMalloc(&p->ll_prop, mb * sizeof(double));
    if (e == hipSuccess) e = hipMalloc(&p->status, mb * sizeof(int));
    if (e != hipSuccess) {
        release(p);
        delete p;
        return fail(RD_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    }
    e = hipMemcpy(p->u0, d->u0, n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(p->v0, d->v0, n * sizeof(double), hipMemcpyHostToDevice);
    if (e == hipSuccess && d->y)
        e = hipMemcpy(p->y, d->y, 2 * n * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        release(p);
        delete p;
        return fail(RD_EHIP, "copy to device failed: %s", hipGetErrorString(e));
    }
    *out = p;
    return RD_OK;
}

extern "C" int32_t g1d_destroy(g1d_problem *p)
{
    if (!p)
        return RD_OK;
    hipDeviceSynchronize();
    release(p);
    delete p;
    return RD_OK;
}

extern "C" int32_t g1d_forward_batch(g1d_problem *p, int32_t n, const double *beta, double *u,
                                     double *v, int32_t *status, void *stream)
{
    int32_t r = check_batch(p, n, beta);
    if (r != RD_OK)
        return r;
    if (n > 0 && (!u || !v))
        return fail(RD_EINVAL, "u and v are required");
    g1d::Args a = base_args(p);
    a.beta = beta;
    a.m = n;
    a.u_out = u;
    a.v_out = v;
    a.status = status;
    a.y = nullptr;
    G1D_TRY(g1d::launch_solve(a, (hipStream_t)stream));
    return RD_OK;
}

extern "C" int32_t g1d_log_likelihood_batch(g1d_problem *p, int32_t n, const double *beta,
                                            double *phi, int32_t *status, void *stream)
{
    int32_t r = check_batch(p, n, beta);
    if (r != RD_OK)
        return r;
    if (!p->y)
        return fail(RD_EINVAL, "the problem has no data y");
    if (n > 0 && !phi)
        return fail(RD_EINVAL, "phi is required");
    g1d::Args a = base_args(p);
    a.beta = beta;
    a.m = n;
    a.phi = phi;
    a.status = status;
    G1D_TRY(g1d::launch_solve(a, (hipStream_t)stream));
    return RD_OK;
}

extern "C" int32_t g1d_mcmc_step_batch(g1d_problem *p, rd_chains *c, int32_t n_steps,
                                       void *stream)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (!c)
        return fail(RD_EINVAL, "chains is NULL");
    if (c->n_chains < 0 || c->n_chains > p->desc.max_batch)
        return fail(RD_EINVAL, "n_chains %d outside [0, max_batch = %d]", c->n_chains,
                    p->desc.max_batch);
    if (!c->phi || !c->loglik)
        return fail(RD_EINVAL, "chains->phi and chains->loglik are required");
    if (c->trace && c->trace_rows < 0)
        return fail(RD_EINVAL, "chains->trace_rows < 0");
    if (!p->y || p->desc.law != G1D_LAW_POLY)
        return fail(RD_EINVAL, "sampling needs data y and the polynomial growth law");
    if (n_steps < 0)
        return fail(RD_EINVAL, "n_steps < 0");
    if (n_steps == 0 || c->n_chains == 0) {
        c->step += (uint64_t)n_steps;
        return RD_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    const g1d_desc &d = p->desc;
    SamplerArgs sa{};
    sa.n = c->n_chains;
    sa.seed = c->seed;
    sa.ctr = p->ctr;
    sa.cfg.free_mask = 0x7u;
    sa.cfg.use_chol = 0;
    sa.cfg.any_normal = 0;
    for (int i = 0; i < 3; ++i) {
        sa.cfg.lo[i] = d.lo[i];
        sa.cfg.hi[i] = d.hi[i];
        sa.cfg.step[i] = d.step[i];
        sa.cfg.prior_kind[i] = d.prior_kind[i];
        sa.cfg.prior_mean[i] = d.prior_mean[i];
        sa.cfg.prior_sd[i] = d.prior_sd[i];
        if (d.prior_kind[i] == RD_PRIOR_NORMAL)
            sa.cfg.any_normal = 1;
    }
    // The fourth coordinate is carried unchanged and only has to lie in a
    // box that holds every value.
    sa.cfg.lo[3] = -INFINITY;
    sa.cfg.hi[3] = INFINITY;
    sa.cfg.step[3] = 0.0;
    sa.cfg.prior_kind[3] = RD_PRIOR_UNIFORM;
    sa.cfg.prior_sd[3] = 1.0;
    sa.cfg.turing = 0;
    sa.phi = c->phi;
    sa.loglik = c->loglik;
    sa.phi_prop = p->phi_prop;
    sa.theta_prop = nullptr;
    sa.inside = p->inside;
    sa.loglik_prop = p->ll_prop;
    sa.n_accept = c->n_accept;
    sa.n_solves = c->n_solves;
    sa.trace = c->trace;
    sa.trace_rows = c->trace_rows;
    g1d::Args a = base_args(p);
    a.beta = p->phi_prop;
    a.beta_stride = 4;
    a.need = p->inside;
    a.m = c->n_chains;
    a.phi = p->ll_prop;
    a.status = p->status;
    G1D_TRY(launch_set_ctr(p->ctr, c->step, c->trace_step0, s));
    for (int k = 0; k < n_steps; ++k) {
        G1D_TRY(launch_propose(sa, s));
        G1D_TRY(g1d::launch_solve(a, s));
        G1D_TRY(launch_accept(sa, s));
        G1D_TRY(launch_advance_ctr(p->ctr, s));
    }
    c->step += (uint64_t)n_steps;
    return RD_OK;
}
