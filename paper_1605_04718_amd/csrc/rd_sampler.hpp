// Sampler kernel arguments (shared by rd_sampler.hip and the C ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rd {

struct SamplerCfg {
    uint32_t free_mask;
    int use_chol;          // proposal step L z instead of step .* z
    double lo[4], hi[4], step[4];
    double chol[16];       // lower-triangular L, row-major
    int prior_kind[4];     // 0 uniform on [lo, hi], 1 normal in the sampling coordinate
    double prior_mean[4], prior_sd[4];
    int any_normal;        // some coordinate has a normal prior
    int turing;            // support restricted to the Turing space
};

struct SamplerArgs {
    int n;                        // chains
    uint32_t seed;
    const uint64_t *ctr;          // [0] = current step, [1] = step of trace row 0
    SamplerCfg cfg;
    double *phi;                  // [n][4] state (sampling coordinates)
    double *loglik;               // [n] Phi(state)
    double *loglik_sur;           // [n] Phi~(state) (DA)
    double *phi_prop;             // [n][4] proposal
    double *theta_prop;           // [n][4] proposal in natural parameters (or null)
    int *inside;                  // [n] proposal in the prior box
    int *need;                    // [n] proposal goes to the full solve
    const double *loglik_prop;    // [n] Phi(proposal)
    double *loglik_sur_prop;      // [n] Phi~(proposal)
    uint64_t *n_accept;
    uint64_t *n_accept1;
    uint64_t *n_solves;
    uint64_t *cg_iters;           // [n][2] accumulated CG iterations or null
    const int *iters;             // [n][2] CG iterations of this step's solves
    uint64_t *imex_steps;         // [n] IMEX steps completed, summed over solves, or null
    uint64_t *fail_bits;          // [n][8] solves with status bit k set, or null
    const int *steps;             // [n] IMEX steps completed by this step's solves (or null)
    const int *status;            // [n] status of this step's solves (or null)
    double *sub_phi;              // [n][4] surrogate-chain state (delayed acceptance, m > 1)
    double *sub_ll;               // [n] Phi~ at the surrogate-chain state
    int *sub_moves;               // [n] accepted substeps of this step
    double *trace;                // [rows][n][4] or null; row = step - ctr[1]
    int trace_rows;
};

hipError_t launch_propose(const SamplerArgs &a, hipStream_t s);
hipError_t launch_accept(const SamplerArgs &a, hipStream_t s);
// Parallel Metropolis-Hastings: a.n chains, n_prop proposals each (items
// c * n_prop + j of phi_prop, theta_prop, inside and loglik_prop).
constexpr int kMaxPmhProposals = 256;
hipError_t launch_pmh_propose(const SamplerArgs &a, int n_prop, hipStream_t s);
hipError_t launch_pmh_resample(const SamplerArgs &a, int n_prop, hipStream_t s);
hipError_t launch_pmh_expand_gid(const int *gid, int n, int n_prop, int *out, hipStream_t s);
hipError_t launch_da_stage1(const SamplerArgs &a, hipStream_t s);
hipError_t launch_da_stage2(const SamplerArgs &a, hipStream_t s);
// Delayed acceptance with a surrogate chain as the first stage: substep j
// (j = 0 starts the chain at the present state) proposes into phi_prop /
// theta_prop / inside, the caller evaluates Phi~ into loglik_sur_prop, and
// the accept kernel moves the chain; finish hands the end point (or
// nothing, when no substep moved) to the solve and the second stage.
hipError_t launch_sub_propose(const SamplerArgs &a, int j, hipStream_t s);
hipError_t launch_sub_accept(const SamplerArgs &a, int j, hipStream_t s);
hipError_t launch_sub_finish(const SamplerArgs &a, hipStream_t s);
hipError_t launch_set_ctr(uint64_t *ctr, uint64_t step, uint64_t step0, hipStream_t s);
hipError_t launch_advance_ctr(uint64_t *ctr, hipStream_t s);
hipError_t launch_copy_i32(const int *src, int *dst, int n, hipStream_t s);

}  // namespace rd
