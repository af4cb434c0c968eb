// Per-chain random-walk Metropolis kernels (Sec. 2, Algorithm 1) and the
// stand-alone misfit kernel.  One thread per chain; every floating-point
// decision is taken in FP64.
#include "rd_device.hpp"
#include "rd_internal.hpp"
#include "rd_sampler.hpp"

// Proposal arithmetic is kept free of fused multiply-adds so that phi' is
// the correctly rounded phi + (s * z) of its definition.
#pragma clang fp contract(off)

namespace rd {

enum : uint32_t {
    kPurposeProposal = 0,
    kPurposeAccept = 1,
    kPurposeStage1 = 2,
    kPurposePmhAux = 6,       // parallel MH: the auxiliary point
    kPurposePmhProp = 7,      // parallel MH: proposal j from blocks 2j, 2j + 1
    kPurposePmhResample = 8,  // parallel MH: uniform of draw n from block n
    kPurposeSubProp = 9,      // surrogate chain: normals of substep j >= 1 (blocks 2j, 2j + 1)
    kPurposeSubAccept = 10,   // surrogate chain: uniform of substep j >= 1 (block j)
};

// The four inequalities of eq. (turing) for the activator-depleted kinetics
// at the homogeneous steady state (a + b, b / (a + b)^2).
__device__ bool turing_space(double a, double b, double d)
{
    const double s = a + b;
    const double tr = (b - a) / s - s * s;
    const double det = s * s;
    const double dfg = d * ((b - a) / s) - s * s;
    const double disc = dfg * dfg - 4.0 * d * det;
    return tr < 0.0 && det > 0.0 && dfg > 0.0 && disc > 0.0;
}

// Sum over normal-prior coordinates of (phi_i - mean_i)^2 / (2 sd_i^2), in
// index order: minus the log prior density up to a constant.
__device__ double prior_quad(const SamplerCfg &cfg, const double *phi)
{
    double acc = 0.0;
    for (int i = 0; i < 4; ++i) {
        if (cfg.prior_kind[i] == 1) {
            const double q = (phi[i] - cfg.prior_mean[i]) / cfg.prior_sd[i];
            acc = acc + 0.5 * (q * q);
        }
    }
    return acc;
}

// log pi(proposal) - log pi(state) of chain c on the support (0 for the
// uniform prior).
__device__ double log_prior_ratio(const SamplerArgs &a, int c)
{
    if (!a.cfg.any_normal)
        return 0.0;
    return prior_quad(a.cfg, a.phi + 4 * c) - prior_quad(a.cfg, a.phi_prop + 4 * c);
}

// phi' = phi + s .* z, or phi + L z with the proposal factor (free
// coordinates), z ~ N(0, I); inside = in the prior's support (uniform
// coordinates within [lo, hi]; with the Turing support, (a, b, d) in the
// Turing space); theta' = (a, b, exp(ln gamma), exp(ln d)).
__global__ void k_propose(SamplerArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n)
        return;
    const uint64_t step = a.ctr[0];
    double z[4];
    gauss_pair(stream_block(a.seed, (uint32_t)c, step, kPurposeProposal, 0), z[0], z[1]);
    gauss_pair(stream_block(a.seed, (uint32_t)c, step, kPurposeProposal, 1), z[2], z[3]);
    double p[4];
    bool in = true;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        p[i] = a.phi[4 * c + i];
        if ((a.cfg.free_mask >> i) & 1u) {
            double dz = 0.0;
            if (a.cfg.use_chol) {
                // row i of L z, summed in column order
                for (int j = 0; j <= i; ++j)
                    dz = dz + a.cfg.chol[4 * i + j] * z[j];
            } else {
                dz = a.cfg.step[i] * z[i];
            }
            p[i] = p[i] + dz;
        }
        if (a.cfg.prior_kind[i] == 0)
            in = in && (a.cfg.lo[i] <= p[i]) && (p[i] <= a.cfg.hi[i]);
        a.phi_prop[4 * c + i] = p[i];
    }
    const double d = exp(p[3]);
    if (a.cfg.turing)
        in = in && turing_space(p[0], p[1], d);
    if (a.theta_prop) {
        a.theta_prop[4 * c + 0] = p[0];
        a.theta_prop[4 * c + 1] = p[1];
        a.theta_prop[4 * c + 2] = exp(p[2]);
        a.theta_prop[4 * c + 3] = d;
    }
    a.inside[c] = in ? 1 : 0;
}

// Random-walk move of the free coordinates: y = x + s .* z, or x + L z.
__device__ __forceinline__ void rw_move(const SamplerCfg &cfg, const double *x, const double *z,
                                        double *y)
{
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        y[i] = x[i];
        if ((cfg.free_mask >> i) & 1u) {
            double dz = 0.0;
            if (cfg.use_chol) {
                for (int j = 0; j <= i; ++j)
                    dz = dz + cfg.chol[4 * i + j] * z[j];
            } else {
                dz = cfg.step[i] * z[i];
            }
            y[i] = y[i] + dz;
        }
    }
}

__device__ __forceinline__ bool in_support(const SamplerCfg &cfg, const double *p, double d)
{
    bool in = true;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        if (cfg.prior_kind[i] == 0)
            in = in && (cfg.lo[i] <= p[i]) && (p[i] <= cfg.hi[i]);
    if (cfg.turing)
        in = in && turing_space(p[0], p[1], d);
    return in;
}

// Parallel Metropolis-Hastings (Sec. 2, Algorithm 2), step 1: item c N + j
// is proposal j of chain c, drawn around the auxiliary point z = x_c + dz
// (purpose 6) as z + dz_j (purpose 7, blocks 2j, 2j + 1); Calderhead's
// construction, for which the matrix A of the algorithm leaves the
// posterior invariant with a symmetric kernel.
__global__ void k_pmh_propose(SamplerArgs a, int n_prop)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.n * n_prop)
        return;
    const int c = t / n_prop, j = t % n_prop;
    const uint64_t step = a.ctr[0];
    double z[4], aux[4], p[4];
    gauss_pair(stream_block(a.seed, (uint32_t)c, step, kPurposePmhAux, 0), z[0], z[1]);
    gauss_pair(stream_block(a.seed, (uint32_t)c, step, kPurposePmhAux, 1), z[2], z[3]);
    rw_move(a.cfg, a.phi + 4 * c, z, aux);
    gauss_pair(stream_block(a.seed, (uint32_t)c, step, kPurposePmhProp, 2 * j), z[0], z[1]);
    gauss_pair(stream_block(a.seed, (uint32_t)c, step, kPurposePmhProp, 2 * j + 1), z[2], z[3]);
    rw_move(a.cfg, aux, z, p);
    const double d = exp(p[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        a.phi_prop[4 * t + i] = p[i];
    if (a.theta_prop) {
        a.theta_prop[4 * t + 0] = p[0];
        a.theta_prop[4 * t + 1] = p[1];
        a.theta_prop[4 * t + 2] = exp(p[2]);
        a.theta_prop[4 * t + 3] = d;
    }
    a.inside[t] = in_support(a.cfg, p, d) ? 1 : 0;
}

// Counters of one solved proposal (item t of this step's solve) of chain c:
// CG iterations, IMEX steps completed (a solve that failed at step s
// completed s), and one count per status bit.
__device__ __forceinline__ void note_solve(const SamplerArgs &a, int c, int t)
{
    if (a.n_solves)
        a.n_solves[c] += 1;
    if (a.cg_iters && a.iters) {
        a.cg_iters[2 * c] += (uint64_t)a.iters[2 * t];
        a.cg_iters[2 * c + 1] += (uint64_t)a.iters[2 * t + 1];
    }
    if (a.imex_steps && a.steps)
        a.imex_steps[c] += (uint64_t)a.steps[t];
    if (a.fail_bits && a.status) {
        const int st = a.status[t];
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if ((st >> k) & 1)
                a.fail_bits[8 * c + k] += 1;
    }
}

// Steps 3 and 4: the stationary distribution of A over the N + 1 points
// (x_c and its N proposals).  A is a Metropolis chain with a uniform choice
// among the other points, so by detailed balance that distribution is the
// normalised target, p_j = w_j / sum w with log w_j = -Phi_j + log pi0_j
// (w_j = 0 outside the support).  N draws from it by the running sum in
// index order, one uniform each (purpose 8, block n), are the chain's next
// N states (trace rows step .. step + N - 1); the last one is the present
// state of the next step.  n_accept counts draws other than x_c.
__global__ void k_pmh_resample(SamplerArgs a, int n_prop)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n)
        return;
    const uint64_t step = a.ctr[0];
    const double *x0 = a.phi + 4 * c;
    auto logw = [&](int k) -> double {
        if (k == 0)
            return -a.loglik[c] - (a.cfg.any_normal ? prior_quad(a.cfg, x0) : 0.0);
        const int t = c * n_prop + k - 1;
        if (!a.inside[t])
            return -__builtin_inf();
        return -a.loglik_prop[t] -
               (a.cfg.any_normal ? prior_quad(a.cfg, a.phi_prop + 4 * t) : 0.0);
    };
    double mx = -__builtin_inf();
    for (int k = 0; k <= n_prop; ++k) {
        const double l = logw(k);
        if (l > mx)
            mx = l;
    }
    const bool any = mx > -__builtin_inf() && mx == mx;
    double sum = 0.0;
    if (any)
        for (int k = 0; k <= n_prop; ++k) {
            const double l = logw(k);
            sum = sum + (l > -__builtin_inf() ? exp(l - mx) : 0.0);
        }
    int moved = 0, last = 0;
    for (int k = 0; k < n_prop; ++k)
        if (a.inside[c * n_prop + k])
            note_solve(a, c, c * n_prop + k);
    for (int n = 0; n < n_prop; ++n) {
        int idx = 0;
        if (any) {
            const U32x4 w = stream_block(a.seed, (uint32_t)c, step, kPurposePmhResample, n);
            const double u = unit_open(w.x, w.y);
            double acc = 0.0;
            idx = -1;
            int last_pos = 0;
            for (int k = 0; k <= n_prop; ++k) {
                const double l = logw(k);
                const double pk = l > -__builtin_inf() ? exp(l - mx) / sum : 0.0;
                if (pk > 0.0)
                    last_pos = k;
                acc = acc + pk;
                if (idx < 0 && u < acc)
                    idx = k;
            }
            if (idx < 0)
                idx = last_pos;
        }
        last = idx;
        moved += idx != 0;
        const double *src = idx == 0 ? x0 : a.phi_prop + 4 * (c * n_prop + idx - 1);
        const uint64_t s = step + (uint64_t)n;
        if (a.trace && s >= a.ctr[1] && s - a.ctr[1] < (uint64_t)a.trace_rows) {
            const uint64_t row = s - a.ctr[1];
#pragma unroll
            for (int i = 0; i < 4; ++i)
                a.trace[(row * (uint64_t)a.n + c) * 4 + i] = src[i];
        }
    }
    if (a.n_accept)
        a.n_accept[c] += (uint64_t)moved;
    if (last != 0) {
        const int t = c * n_prop + last - 1;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a.phi[4 * c + i] = a.phi_prop[4 * t + i];
        a.loglik[c] = a.loglik_prop[t];
    }
}

// Item grid class of a parallel-MH batch: item c N + j has chain c's class.
__global__ void k_pmh_expand_gid(const int *gid, int n, int n_prop, int *out)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n * n_prop)
        out[t] = gid[t / n_prop];
}

// Accept iff log U < [Phi(phi) - Phi(phi')] + [log pi(phi') - log pi(phi)],
// U from purpose 1; then record.
__global__ void k_accept(SamplerArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n)
        return;
    const uint64_t step = a.ctr[0];
    bool acc = false;
    if (a.inside[c]) {
        const U32x4 w = stream_block(a.seed, (uint32_t)c, step, kPurposeAccept, 0);
        const double u = unit_open(w.x, w.y);
        acc = log(u) < (a.loglik[c] - a.loglik_prop[c]) + log_prior_ratio(a, c);
        note_solve(a, c, c);
    }
    if (acc) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a.phi[4 * c + i] = a.phi_prop[4 * c + i];
        a.loglik[c] = a.loglik_prop[c];
        if (a.n_accept)
            a.n_accept[c] += 1;
    }
    if (a.trace && step >= a.ctr[1] && step - a.ctr[1] < (uint64_t)a.trace_rows) {
        const uint64_t row = step - a.ctr[1];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a.trace[(row * (uint64_t)a.n + c) * 4 + i] = a.phi[4 * c + i];
    }
}

// Delayed acceptance, first stage: log U1 < [Phi~(phi) - Phi~(phi')] +
// [log pi(phi') - log pi(phi)], U1 from purpose 2.  Writes need[c] (solve
// the proposal) and counts stage-1 accepts.
__global__ void k_da_stage1(SamplerArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n)
        return;
    const uint64_t step = a.ctr[0];
    bool acc1 = false;
    if (a.inside[c]) {
        const U32x4 w = stream_block(a.seed, (uint32_t)c, step, kPurposeStage1, 0);
        const double u = unit_open(w.x, w.y);
        acc1 = log(u) < (a.loglik_sur[c] - a.loglik_sur_prop[c]) + log_prior_ratio(a, c);
    }
    a.need[c] = acc1 ? 1 : 0;
    if (acc1 && a.n_accept1)
        a.n_accept1[c] += 1;
}

// Delayed acceptance whose first stage is m Metropolis steps on the
// surrogate posterior prior x exp(-Phi~), started at the present state x
// (the surrogate transition: the surrogate's own reversible kernel as the
// proposal of Christen and Fox's second stage).  Substep j proposes
// z' = z + s .* dz (or z + L dz) from the substep state z, with the normals
// of purpose 0 (j = 0) or purpose 9 (blocks 2j, 2j + 1): the same proposal
// as k_propose at j = 0, when z = x.
__global__ void k_sub_propose(SamplerArgs a, int j)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n)
        return;
    const uint64_t step = a.ctr[0];
    double *z = a.sub_phi + 4 * c;
    if (j == 0) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            z[i] = a.phi[4 * c + i];
        a.sub_ll[c] = a.loglik_sur[c];
        a.sub_moves[c] = 0;
    }
    const uint32_t purpose = j == 0 ? kPurposeProposal : kPurposeSubProp;
    const uint32_t block = j == 0 ? 0u : 2u * (uint32_t)j;
    double dz[4], p[4];
    gauss_pair(stream_block(a.seed, (uint32_t)c, step, purpose, block), dz[0], dz[1]);
    gauss_pair(stream_block(a.seed, (uint32_t)c, step, purpose, block + 1), dz[2], dz[3]);
    rw_move(a.cfg, z, dz, p);
    const double d = exp(p[3]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
        a.phi_prop[4 * c + i] = p[i];
    if (a.theta_prop) {
        a.theta_prop[4 * c + 0] = p[0];
        a.theta_prop[4 * c + 1] = p[1];
        a.theta_prop[4 * c + 2] = exp(p[2]);
        a.theta_prop[4 * c + 3] = d;
    }
    a.inside[c] = in_support(a.cfg, p, d) ? 1 : 0;
}

// Substep j's test: log U < [Phi~(z) - Phi~(z')] + [log pi(z') - log pi(z)]
// with U from purpose 2 (j = 0, the first-stage uniform of k_da_stage1) or
// purpose 10 (block j).
__global__ void k_sub_accept(SamplerArgs a, int j)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n || !a.inside[c])
        return;
    const uint64_t step = a.ctr[0];
    const U32x4 w = j == 0 ? stream_block(a.seed, (uint32_t)c, step, kPurposeStage1, 0)
                           : stream_block(a.seed, (uint32_t)c, step, kPurposeSubAccept, (uint32_t)j);
    const double u = unit_open(w.x, w.y);
    double *z = a.sub_phi + 4 * c;
    const double *prop = a.phi_prop + 4 * c;
    const double lpr = a.cfg.any_normal ? prior_quad(a.cfg, z) - prior_quad(a.cfg, prop) : 0.0;
    if (log(u) < (a.sub_ll[c] - a.loglik_sur_prop[c]) + lpr) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            z[i] = prop[i];
        a.sub_ll[c] = a.loglik_sur_prop[c];
        a.sub_moves[c] += 1;
    }
}

// The end point y of the surrogate chain becomes the proposal of the second
// stage (solved) when some substep moved; otherwise y = x and nothing is
// solved.  n_accept1 counts the proposals that reach the second stage.
__global__ void k_sub_finish(SamplerArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n)
        return;
    const bool moved = a.sub_moves[c] > 0;
    a.need[c] = moved ? 1 : 0;
    if (!moved)
        return;
    const double *z = a.sub_phi + 4 * c;
#pragma unroll
    for (int i = 0; i < 4; ++i)
        a.phi_prop[4 * c + i] = z[i];
    if (a.theta_prop) {
        a.theta_prop[4 * c + 0] = z[0];
        a.theta_prop[4 * c + 1] = z[1];
        a.theta_prop[4 * c + 2] = exp(z[2]);
        a.theta_prop[4 * c + 3] = exp(z[3]);
    }
    a.loglik_sur_prop[c] = a.sub_ll[c];
    if (a.n_accept1)
        a.n_accept1[c] += 1;
}

// Second stage: log U2 < [Phi(phi) - Phi(phi')] - [Phi~(phi) - Phi~(phi')].
__global__ void k_da_stage2(SamplerArgs a)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n)
        return;
    const uint64_t step = a.ctr[0];
    bool acc = false;
    if (a.need[c]) {
        const U32x4 w = stream_block(a.seed, (uint32_t)c, step, kPurposeAccept, 0);
        const double u = unit_open(w.x, w.y);
        const double la = (a.loglik[c] - a.loglik_prop[c]) - (a.loglik_sur[c] - a.loglik_sur_prop[c]);
        acc = log(u) < la;
        note_solve(a, c, c);
    }
    if (acc) {
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a.phi[4 * c + i] = a.phi_prop[4 * c + i];
        a.loglik[c] = a.loglik_prop[c];
        a.loglik_sur[c] = a.loglik_sur_prop[c];
        if (a.n_accept)
            a.n_accept[c] += 1;
    }
    if (a.trace && step >= a.ctr[1] && step - a.ctr[1] < (uint64_t)a.trace_rows) {
        const uint64_t row = step - a.ctr[1];
#pragma unroll
        for (int i = 0; i < 4; ++i)
            a.trace[(row * (uint64_t)a.n + c) * 4 + i] = a.phi[4 * c + i];
    }
}

__global__ void k_set_ctr(uint64_t *ctr, uint64_t step, uint64_t step0)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ctr[0] = step;
        ctr[1] = step0;
    }
}

__global__ void k_advance_ctr(uint64_t *ctr)
{
    if (threadIdx.x == 0 && blockIdx.x == 0)
        ctr[0] = ctr[0] + 1;
}

// inside -> need copy (plain sampler: solve every in-box proposal).
__global__ void k_copy_i32(const int *src, int *dst, int n)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < n)
        dst[c] = src[c];
}

template <typename Real>
__global__ void k_field_misfit(const GridDev *grids, const int *grid_id, int npts, const Real *u,
                               double *phi)
{
    __shared__ double red[4];
    const int c = blockIdx.x;
    const GridDev &gd = grids[grid_id ? grid_id[c] : 0];
    double s = 0.0;
    for (int k = threadIdx.x; k < npts; k += blockDim.x) {
        const double e = gd.y[k] - (double)u[(size_t)c * npts + k];
        s += e * e;
    }
    s = block_sum<4>(s, red);
    if (threadIdx.x == 0)
        phi[c] = finite(s) ? s * gd.inv_2s2 : __builtin_inf();
}

static inline dim3 chain_blocks(int n)
{
    return dim3((n + 255) / 256);
}

hipError_t launch_propose(const SamplerArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_propose, chain_blocks(a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_pmh_propose(const SamplerArgs &a, int n_prop, hipStream_t s)
{
    hipLaunchKernelGGL(k_pmh_propose, chain_blocks(a.n * n_prop), dim3(256), 0, s, a, n_prop);
    return hipGetLastError();
}

hipError_t launch_pmh_resample(const SamplerArgs &a, int n_prop, hipStream_t s)
{
    hipLaunchKernelGGL(k_pmh_resample, chain_blocks(a.n), dim3(256), 0, s, a, n_prop);
    return hipGetLastError();
}

hipError_t launch_pmh_expand_gid(const int *gid, int n, int n_prop, int *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_pmh_expand_gid, chain_blocks(n * n_prop), dim3(256), 0, s, gid, n,
                       n_prop, out);
    return hipGetLastError();
}

hipError_t launch_accept(const SamplerArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_accept, chain_blocks(a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_da_stage1(const SamplerArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_da_stage1, chain_blocks(a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_sub_propose(const SamplerArgs &a, int j, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub_propose, chain_blocks(a.n), dim3(256), 0, s, a, j);
    return hipGetLastError();
}

hipError_t launch_sub_accept(const SamplerArgs &a, int j, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub_accept, chain_blocks(a.n), dim3(256), 0, s, a, j);
    return hipGetLastError();
}

hipError_t launch_sub_finish(const SamplerArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_sub_finish, chain_blocks(a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_da_stage2(const SamplerArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_da_stage2, chain_blocks(a.n), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_set_ctr(uint64_t *ctr, uint64_t step, uint64_t step0, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_ctr, dim3(1), dim3(64), 0, s, ctr, step, step0);
    return hipGetLastError();
}

hipError_t launch_advance_ctr(uint64_t *ctr, hipStream_t s)
{
    hipLaunchKernelGGL(k_advance_ctr, dim3(1), dim3(64), 0, s, ctr);
    return hipGetLastError();
}

hipError_t launch_copy_i32(const int *src, int *dst, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_copy_i32, chain_blocks(n), dim3(256), 0, s, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_field_misfit(int precision, const GridDev *grids, const int *grid_id, int n,
                               int npts, const void *u, double *phi, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    if (precision == 0)
        hipLaunchKernelGGL(k_field_misfit<float>, dim3(n), dim3(256), 0, s, grids, grid_id, npts,
                           (const float *)u, phi);
    else
        hipLaunchKernelGGL(k_field_misfit<double>, dim3(n), dim3(256), 0, s, grids, grid_id, npts,
                           (const double *)u, phi);
    return hipGetLastError();
}

}  // namespace rd
