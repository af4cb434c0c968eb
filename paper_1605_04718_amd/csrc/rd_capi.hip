// C ABI of the library: problem handle, workspace, launch sequencing.
// Every entry point validates its arguments on the host, enqueues kernels
// on the caller's stream and returns; nothing here computes a step of the
// method on the host.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/rdbayes.h"
#include "rd_internal.hpp"
#include "rd_mlp.hpp"
#include "rd_sampler.hpp"

using namespace rd;

namespace {

thread_local char g_err[512] = "";

int32_t fail(int32_t code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace

// Error text for the entry points of the other translation units (not part
// of the exported interface).
extern "C" __attribute__((visibility("hidden"))) int32_t rd_set_error(int32_t code, const char *msg)
{
    snprintf(g_err, sizeof g_err, "%s", msg);
    return code;
}

namespace {

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(RD_EHIP, "%s: %s", #expr, hipGetErrorString(e_));              \
    } while (0)

// Autotuned tile per (device, n, precision), shared by every problem of the
// process.
std::mutex g_tune_mu;
std::map<long, int> g_tuned;

long tune_key(int dev, int n, int prec)
{
    return ((long)dev << 32) | ((long)n << 2) | prec;
}

}  // namespace

// Scratch of log_likelihood_batch_noalloc: the queue head (the first 256
// bytes), then one solve slot per workgroup (predictor history and the low
// parts of the compensated fields; streamed tiles also their strip arrays).
// Every device the library runs on holds one copy until the process ends.
// In host code `scratch` names a host-side stand-in: its device address is
// taken once per device with hipGetSymbolAddress and used from then on.
constexpr size_t kNoAllocHeader = 256;
constexpr size_t kNoAllocSlots = (size_t)96 << 20;  // 96 MiB of solve slots
static __device__ __align__(256) unsigned char scratch[kNoAllocHeader + kNoAllocSlots];

namespace {

std::mutex g_scratch_mu;
std::map<int, void *> g_scratch_ptr;

// This device's address of `scratch` (the device must be current).
int32_t scratch_address(int dev, void **out)
{
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_ptr.find(dev);
    if (it != g_scratch_ptr.end()) {
        *out = it->second;
        return RD_OK;
    }
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
        return fail(RD_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev,
                    hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
    *out = ptr;
    return RD_OK;
}

}  // namespace

struct GraphEntry {
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    // identity of what was captured
    rd_chains key{};
    int mode = 0;
    hipStream_t stream = nullptr;
};

struct rd_problem {
    int device = 0;
    int n_cu = 0;
    rd_problem_desc desc{};
    std::vector<rd_grid_desc> grid_desc;
    std::vector<GridDev> grids_host;
    GridDev *grids_dev = nullptr;
    std::vector<void *> allocs;
    TileChoice tile[RD_MAX_GRIDS]{};
    int wgs_per_cu[RD_MAX_GRIDS]{};  // resident workgroups per CU of tile[g]
    // batches that mix grid classes: one persistent launch of this many
    // threads per workgroup, queue ordered by class cost
    int mixed_threads = 1024;
    int mixed_wpc = 1;
    RankTable rank{};
    int *order_ws = nullptr;
    int maxit = 0;
    int max_n = 0;  // largest class: field outputs have max_n^2 values per item
    // workspace [max_batch]
    unsigned *queue = nullptr;
    double *theta_prop = nullptr;
    double *phi_prop = nullptr;
    int *inside = nullptr;
    int *need = nullptr;
    double *ll_prop = nullptr;
    double *ll_sur_prop = nullptr;
    int *status_ws = nullptr;
    int *pmh_gid = nullptr;   // [max_batch] item classes of a parallel-MH batch
    int *iters_ws = nullptr;
    int *cost_ws = nullptr;      // [max_batch] per-chain solve cost estimate (-1: none yet)
    int *steps_ws = nullptr;     // [max_batch] IMEX steps each item of a sampler solve completed
    // delayed acceptance: first-stage substeps on the surrogate (1: one
    // screened proposal) and the surrogate chain's state
    int da_substeps = 1;
    double *sub_phi = nullptr;   // [max_batch][4]
    double *sub_ll = nullptr;    // [max_batch]
    int *sub_moves = nullptr;    // [max_batch]
    void *scratch = nullptr;     // this device's address of the no-allocation scratch array
    uint64_t *ctr = nullptr;
    void *gws = nullptr;     // per-workgroup solve slots
    size_t gws_stride = 0;
    int gws_slots = 0;
    void *coop = nullptr;    // cooperative-solve workspace (256^2 FP32)
    int coop_groups = 0;
    int coop_wpc = 0;        // resident cooperative workgroups per CU
    int mixed_coop_wpc = 0;  // resident workgroups per CU of the fused mixed launch
    // cooperative waits: bound (100 MHz ticks), test-hook stall, and the
    // device count of members whose wait gave up since the last check
    unsigned long long coop_wait_ticks = 1000000000ull;
    unsigned long long coop_stall_ticks = 0;
    unsigned *coop_timeouts = nullptr;
    // timing of the fused solve kernel
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> pending;
    std::vector<hipEvent_t> free_events;
    double ms_total = 0.0;
    int64_t launches = 0;
    // captured MCMC steps
    std::vector<GraphEntry> graphs;
    // layouts (chains, mode, stream) whose step has run once directly since
    // the graphs were last dropped: the next step of such a layout is captured
    std::vector<GraphEntry> warm;
    bool use_graphs = true;
    // surrogate
    Surrogate *sur = nullptr;
};

namespace {

void *dmalloc(rd_problem *p, size_t bytes, int32_t *err)
{
    void *ptr = nullptr;
    if (bytes == 0)
        bytes = 16;
    if (hipMalloc(&ptr, bytes) != hipSuccess) {
        *err = fail(RD_ENOMEM, "hipMalloc(%zu) failed", bytes);
        return nullptr;
    }
    p->allocs.push_back(ptr);
    return ptr;
}

int32_t upload_field(rd_problem *p, const double *host, int nn, void **out)
{
    int32_t err = RD_OK;
    if (p->desc.precision == RD_PRECISION_FP32) {
        // [hi | lo]: the FP32 solver carries fields as unevaluated sums
        std::vector<float> f(2 * nn);
        for (int k = 0; k < nn; ++k) {
            f[k] = (float)host[k];
            f[nn + k] = (float)(host[k] - (double)f[k]);
        }
        *out = dmalloc(p, sizeof(float) * 2 * nn, &err);
        if (!*out)
            return err;
        HIP_TRY(hipMemcpy(*out, f.data(), sizeof(float) * 2 * nn, hipMemcpyHostToDevice));
    } else {
        *out = dmalloc(p, sizeof(double) * nn, &err);
        if (!*out)
            return err;
        HIP_TRY(hipMemcpy(*out, host, sizeof(double) * nn, hipMemcpyHostToDevice));
    }
    return RD_OK;
}

hipError_t record_solve_start(rd_problem *p, hipStream_t s, hipEvent_t *ev)
{
    *ev = nullptr;
    if (!p->timing)
        return hipSuccess;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    hipStreamIsCapturing(s, &cs);
    if (cs != hipStreamCaptureStatusNone)
        return hipSuccess;
    hipEvent_t e;
    if (!p->free_events.empty()) {
        e = p->free_events.back();
        p->free_events.pop_back();
    } else {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess)
            return r;
    }
    *ev = e;
    return hipEventRecord(e, s);
}

hipError_t record_solve_end(rd_problem *p, hipStream_t s, hipEvent_t start)
{
    if (!start)
        return hipSuccess;
    hipEvent_t e;
    if (!p->free_events.empty()) {
        e = p->free_events.back();
        p->free_events.pop_back();
    } else {
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess)
            return r;
    }
    p->pending.push_back({start, e});
    return hipEventRecord(e, s);
}

// Enqueue: reset the queue head, then the persistent fused solve.
// Without grid ids every item is of class `cls` (0 for the public calls;
// the autotuner times each class on its own).
// cost (optional, [n]): per-item cost estimates (negative: unknown); a
// single-class launch then takes its items largest first.
// Workspace of one solve launch other than the problem's own: the queue
// head and the per-workgroup slots (single-class launches of a resident or
// streamed tile only).
struct SolveWs {
    unsigned *queue;
    void *gws;
    size_t stride;
    int slots;
};

int32_t enqueue_solve(rd_problem *p, int n, const double *theta, const int *grid_id,
                      const int *need, double *phi, int *status, int *iters, void *u_out,
                      void *v_out, hipStream_t s, int cls = 0, int *steps_out = nullptr,
                      const int *cost = nullptr, const SolveWs *ws = nullptr)
{
    if (n == 0)
        return RD_OK;
    const bool mixed = p->desc.n_grids > 1 && grid_id;
    const int g = mixed ? 0 : cls;
    const int nn = p->grids_host[g].n;
    SolveArgs a{};
    // single-class launches see class g as their only class
    a.grids = mixed ? p->grids_dev : p->grids_dev + g;
    a.n_grids = mixed ? p->desc.n_grids : 1;
    a.n_items = n;
    a.order = nullptr;
    a.grid_id = grid_id;
    a.theta = theta;
    a.need = need;
    a.dt = p->desc.dt;
    a.n_steps = p->desc.n_steps;
    a.rtol2 = p->desc.cg_rtol * p->desc.cg_rtol;
    a.maxit = p->maxit;
    a.phi = phi;
    a.status = status;
    a.iters = iters;
    a.u_out = u_out;
    a.v_out = v_out;
    a.out_stride = (size_t)p->max_n * p->max_n;
    a.queue = p->queue;
    a.gws = p->gws;
    a.gws_stride = p->gws_stride;
    a.gws_slots = p->gws_slots;
    a.coop = p->coop;
    a.coop_groups = p->coop_groups;
    a.steady_tt = p->desc.steady_tol > 0.0 ? p->desc.steady_tol * p->desc.dt : 0.0;
    a.steps_out = steps_out;
    a.coop_wait_ticks = p->coop_wait_ticks;
    a.coop_stall_ticks = p->coop_stall_ticks;
    a.coop_timeouts = p->coop_timeouts;
    if (ws) {
        a.queue = ws->queue;
        a.gws = ws->gws;
        a.gws_stride = ws->stride;
        a.gws_slots = ws->slots;
        a.coop = nullptr;
        a.coop_groups = 0;
    }
    const TileChoice t = p->tile[g];
    // wgs_per_cu was queried when the tile was chosen: no runtime query may
    // run here, since this is also called while a stream is being captured.
    int wgs = p->n_cu * (mixed ? p->mixed_wpc : p->wgs_per_cu[g]);
    if (ws) {
        if (mixed || cost || tile_coop(nn, p->desc.precision, t.cpt))
            return fail(RD_EUNSUPPORTED, "external workspace: single-class, uncooperative tiles only");
        wgs = std::min(wgs, ws->slots);
    }
    // (a cooperative tile sizes its grid from the item count itself)
    if (wgs > n && (mixed || !tile_coop(nn, p->desc.precision, t.cpt)))
        wgs = n;
    // batches mixing classes with 256^2 FP32 items: groups of four resident
    // workgroups serve them (the prefix of the class-ordered queue).  With
    // 1024-thread workgroups one launch does both (the cooperative
    // workgroups join the other classes' queue when the prefix is done);
    // with 512 a cooperative launch runs first and the mixed launch skips
    // the 256^2 items.
    a.coop_wgs = 0;
    int coop_grid = 0;
    const bool fused = p->mixed_threads == kCoopThreads;
    if (mixed && p->coop && p->desc.precision == 0) {
        // every workgroup of the fused launch is resident at once, and the
        // cooperative role takes whole blocks of 32 (small batches too)
        if (fused)
            wgs = std::min(std::max(wgs, 32), p->n_cu * p->mixed_coop_wpc);
        coop_grid = std::min((fused ? wgs : p->n_cu * p->coop_wpc) / 32 * 32,
                             p->coop_groups * kCoopG);
        a.coop_wgs = coop_grid >= 32 ? coop_grid : 0;
    }
    HIP_TRY(launch_fill_u32(a.queue, 0u, 1, s));
    if (mixed) {
        HIP_TRY(launch_class_order(grid_id, n, p->desc.n_grids, p->rank, p->order_ws, s));
        a.order = p->order_ws;
    } else if (cost && n <= kMaxCostOrder) {
        HIP_TRY(launch_cost_order(n, need, cost, p->order_ws, s));
        a.order = p->order_ws;
    }
    hipEvent_t e0 = nullptr;
    if (!ws)  // (event creation may allocate: an external workspace is never timed)
        HIP_TRY(record_solve_start(p, s, &e0));
    if (!mixed) {
        HIP_TRY(launch_solve(nn, p->desc.precision, t, a, wgs, s));
    } else if (a.coop_wgs && fused) {
        HIP_TRY(launch_solve_mixed_coop(a, wgs, s));
    } else {
        if (a.coop_wgs)
            HIP_TRY(launch_solve_coop(a, coop_grid, s));
        HIP_TRY(launch_solve_mixed(p->desc.precision, p->mixed_threads, a, wgs, s));
    }
    HIP_TRY(record_solve_end(p, s, e0));
    return RD_OK;
}

int32_t check_chains(rd_problem *p, const rd_chains *c, int mode)
{
    if (!c)
        return fail(RD_EINVAL, "chains is NULL");
    if (c->n_chains < 0 || c->n_chains > p->desc.max_batch)
        return fail(RD_EINVAL, "n_chains %d outside [0, max_batch=%d]", c->n_chains,
                    p->desc.max_batch);
    if (!c->phi || !c->loglik)
        return fail(RD_EINVAL, "chains->phi and chains->loglik are required");
    if (c->trace && c->trace_rows < 0)
        return fail(RD_EINVAL, "chains->trace_rows < 0");
    if (mode == RD_MODE_DA && !c->loglik_sur)
        return fail(RD_EINVAL, "delayed acceptance needs chains->loglik_sur");
    return RD_OK;
}

SamplerArgs sampler_args(rd_problem *p, const rd_chains *c)
{
    SamplerArgs a{};
    a.n = c->n_chains;
    a.seed = c->seed;
    a.ctr = p->ctr;
    a.cfg.free_mask = p->desc.free_mask;
    a.cfg.use_chol = 0;
    for (int i = 0; i < 16; ++i) {
        a.cfg.chol[i] = p->desc.prop_chol[i];
        if (p->desc.prop_chol[i] != 0.0)
            a.cfg.use_chol = 1;
    }
    a.cfg.any_normal = 0;
    for (int i = 0; i < 4; ++i) {
        a.cfg.lo[i] = p->desc.lo[i];
        a.cfg.hi[i] = p->desc.hi[i];
        a.cfg.step[i] = p->desc.step[i];
        a.cfg.prior_kind[i] = p->desc.prior_kind[i];
        a.cfg.prior_mean[i] = p->desc.prior_mean[i];
        a.cfg.prior_sd[i] = p->desc.prior_sd[i];
        if (p->desc.prior_kind[i] == RD_PRIOR_NORMAL)
            a.cfg.any_normal = 1;
    }
    a.cfg.turing = p->desc.turing_support;
    a.phi = c->phi;
    a.loglik = c->loglik;
    a.loglik_sur = c->loglik_sur;
    a.phi_prop = p->phi_prop;
    a.theta_prop = p->theta_prop;
    a.inside = p->inside;
    a.need = p->need;
    a.loglik_prop = p->ll_prop;
    a.loglik_sur_prop = p->ll_sur_prop;
    a.n_accept = c->n_accept;
    a.n_accept1 = c->n_accept1;
    a.n_solves = c->n_solves;
    a.cg_iters = c->cg_iters;
    a.iters = p->iters_ws;
    a.imex_steps = c->imex_steps;
    a.fail_bits = c->fail_bits;
    a.steps = p->steps_ws;
    a.status = p->status_ws;
    a.sub_phi = p->sub_phi;
    a.sub_ll = p->sub_ll;
    a.sub_moves = p->sub_moves;
    a.trace = c->trace;
    a.trace_rows = c->trace ? c->trace_rows : 0;
    return a;
}

// One MCMC step as a kernel sequence (the unit that is captured in a graph).
int32_t enqueue_mcmc_step(rd_problem *p, const rd_chains *c, int mode, hipStream_t s)
{
    SamplerArgs a = sampler_args(p, c);
    HIP_TRY(launch_propose(a, s));
    if (mode == RD_MODE_PLAIN) {
        HIP_TRY(launch_copy_i32(p->inside, p->need, c->n_chains, s));
    } else if (p->da_substeps <= 1) {
        int32_t r = surrogate_enqueue_loglik(p->sur, c->n_chains, p->phi_prop, p->ll_sur_prop, s);
        if (r != RD_OK)
            return fail(r, "surrogate evaluation failed: %s", hipGetErrorString(hipGetLastError()));
        HIP_TRY(launch_da_stage1(a, s));
    } else {
        // first stage: da_substeps Metropolis steps on the surrogate posterior
        // (substep 0 starts the chain at the present state and proposes what
        // launch_propose drew)
        for (int j = 0; j < p->da_substeps; ++j) {
            HIP_TRY(launch_sub_propose(a, j, s));
            int32_t r = surrogate_enqueue_loglik(p->sur, c->n_chains, p->phi_prop,
                                                 p->ll_sur_prop, s);
            if (r != RD_OK)
                return fail(r, "surrogate evaluation failed: %s",
                            hipGetErrorString(hipGetLastError()));
            HIP_TRY(launch_sub_accept(a, j, s));
        }
        HIP_TRY(launch_sub_finish(a, s));
    }
    // cost_ws keeps, per chain, a decaying maximum of the CG iterations of
    // its solved proposals (-1 before the first): the cost estimate of this
    // step's proposal, which lies close to them
    int32_t r = enqueue_solve(p, c->n_chains, p->theta_prop, c->grid_id, p->need, p->ll_prop,
                              p->status_ws, p->iters_ws, nullptr, nullptr, s, 0, p->steps_ws,
                              p->cost_ws);
    if (r != RD_OK)
        return r;
    HIP_TRY(launch_note_cost(c->n_chains, p->need, p->iters_ws, p->cost_ws, s));
    if (mode == RD_MODE_PLAIN)
        HIP_TRY(launch_accept(a, s));
    else
        HIP_TRY(launch_da_stage2(a, s));
    HIP_TRY(launch_advance_ctr(p->ctr, s));
    return RD_OK;
}

bool same_chains(const rd_chains &a, const rd_chains &b)
{
    return a.n_chains == b.n_chains && a.phi == b.phi && a.loglik == b.loglik &&
           a.loglik_sur == b.loglik_sur && a.grid_id == b.grid_id && a.n_accept == b.n_accept &&
           a.n_accept1 == b.n_accept1 && a.n_solves == b.n_solves && a.cg_iters == b.cg_iters &&
           a.trace == b.trace && a.trace_rows == b.trace_rows && a.seed == b.seed &&
           a.imex_steps == b.imex_steps && a.fail_bits == b.fail_bits;
}

void drop_graphs(rd_problem *p)
{
    for (auto &g : p->graphs) {
        if (g.exec)
            hipGraphExecDestroy(g.exec);
        if (g.graph)
            hipGraphDestroy(g.graph);
    }
    p->graphs.clear();
    p->warm.clear();
}

}  // namespace

// ---------------------------------------------------------------------------

extern "C" int32_t init_problem(const rd_problem_desc *desc, rd_problem **out)
{
    if (!desc || !out)
        return fail(RD_EINVAL, "desc and out are required");
    *out = nullptr;
    if (desc->n_grids < 1 || desc->n_grids > RD_MAX_GRIDS || !desc->grids)
        return fail(RD_EINVAL, "n_grids must be in [1, %d]", RD_MAX_GRIDS);
    if (!(desc->dt > 0.0) || desc->n_steps < 0)
        return fail(RD_EINVAL, "dt must be > 0 and n_steps >= 0");
    if (!(desc->cg_rtol > 0.0))
        return fail(RD_EINVAL, "cg_rtol must be > 0");
    if (desc->precision != RD_PRECISION_FP32 && desc->precision != RD_PRECISION_FP64)
        return fail(RD_EINVAL, "precision must be 0 (FP32) or 1 (FP64)");
    if (desc->max_batch < 1)
        return fail(RD_EINVAL, "max_batch must be >= 1");
    for (int i = 0; i < 4; ++i)
        if (!(desc->lo[i] <= desc->hi[i]) || !(desc->step[i] >= 0.0))
            return fail(RD_EINVAL, "prior box / step of coordinate %d invalid", i);
    for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j)
            if ((j > i && desc->prop_chol[4 * i + j] != 0.0) || !std::isfinite(desc->prop_chol[4 * i + j]))
                return fail(RD_EINVAL, "prop_chol must be finite and lower-triangular");
    for (int i = 0; i < 4; ++i) {
        if (desc->prior_kind[i] != RD_PRIOR_UNIFORM && desc->prior_kind[i] != RD_PRIOR_NORMAL)
            return fail(RD_EINVAL, "prior_kind[%d] = %d is not a prior kind", i, desc->prior_kind[i]);
        if (desc->prior_kind[i] == RD_PRIOR_NORMAL &&
            (!std::isfinite(desc->prior_mean[i]) || !(desc->prior_sd[i] > 0.0) ||
             !std::isfinite(desc->prior_sd[i])))
            return fail(RD_EINVAL, "normal prior %d needs a finite mean and a positive s.d.", i);
    }
    if (desc->turing_support != 0 && desc->turing_support != 1)
        return fail(RD_EINVAL, "turing_support must be 0 or 1");
    if (!(desc->steady_tol >= 0.0) || !std::isfinite(desc->steady_tol))
        return fail(RD_EINVAL, "steady_tol must be finite and >= 0");
    for (int g = 0; g < desc->n_grids; ++g) {
        const rd_grid_desc &gd = desc->grids[g];
        if (!tile_supported(gd.n, desc->precision, default_cpt(gd.n, desc->precision)))
            return fail(RD_EUNSUPPORTED, "grid %d: n = %d has no kernel at this precision", g, gd.n);
        if (desc->n_grids > 1 &&
            !(mixed_supported(gd.n, desc->precision, 512) && mixed_supported(gd.n, desc->precision, 1024)))
            return fail(RD_EUNSUPPORTED, "grid %d: n = %d cannot join a mixed batch", g, gd.n);
        if (!gd.u0 || !gd.v0)
            return fail(RD_EINVAL, "grid %d: u0 and v0 are required", g);
        if (gd.growth != 0 && gd.growth != 1)
            return fail(RD_EINVAL, "grid %d: growth must be 0 or 1", g);
        if (gd.y && !(gd.sigma > 0.0))
            return fail(RD_EINVAL, "grid %d: sigma must be > 0", g);
    }

    rd_problem *p = new rd_problem();
    p->desc = *desc;
    p->grid_desc.assign(desc->grids, desc->grids + desc->n_grids);
    p->desc.grids = p->grid_desc.data();
    int32_t err = RD_OK;
    hipDeviceProp_t prop;
    if (hipGetDevice(&p->device) != hipSuccess ||
        hipGetDeviceProperties(&prop, p->device) != hipSuccess) {
        delete p;
        return fail(RD_EHIP, "no HIP device");
    }
    p->n_cu = prop.multiProcessorCount;
    if ((err = scratch_address(p->device, &p->scratch)) != RD_OK) {
        delete p;
        return err;
    }
    int max_n = 0;
    for (int g = 0; g < desc->n_grids; ++g) {
        const rd_grid_desc &gd = desc->grids[g];
        const int nn = gd.n * gd.n;
        max_n = std::max(max_n, gd.n);
        GridDev d{};
        d.n = gd.n;
        d.growth = gd.growth;
        d.rate = gd.growth ? gd.growth_rate : 0.0;
        if ((err = upload_field(p, gd.u0, nn, (void **)&d.u0)) != RD_OK ||
            (err = upload_field(p, gd.v0, nn, (void **)&d.v0)) != RD_OK) {
            destroy_problem(p);
            return err;
        }
        if (gd.y) {
            double *y = (double *)dmalloc(p, sizeof(double) * nn, &err);
            if (!y || hipMemcpy(y, gd.y, sizeof(double) * nn, hipMemcpyHostToDevice) != hipSuccess) {
                destroy_problem(p);
                return err != RD_OK ? err : fail(RD_EHIP, "upload of y failed");
            }
            d.y = y;
            d.inv_2s2 = 0.5 / (gd.sigma * gd.sigma);
        }
        d.cost = (double)nn;
        p->grids_host.push_back(d);
        int cpt = default_cpt(gd.n, desc->precision);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(tune_key(p->device, gd.n, desc->precision));
            if (it != g_tuned.end())
                cpt = it->second;
        }
        p->tile[g] = TileChoice{cpt, nn / cpt};
        p->wgs_per_cu[g] = solve_wgs_per_cu(gd.n, desc->precision, cpt);
    }
    p->maxit = desc->cg_maxit > 0 ? desc->cg_maxit : 10 * max_n * max_n;
    p->max_n = max_n;
    const int B = desc->max_batch;
    p->grids_dev = (GridDev *)dmalloc(p, sizeof(GridDev) * desc->n_grids, &err);
    p->queue = (unsigned *)dmalloc(p, 64, &err);
    p->ctr = (uint64_t *)dmalloc(p, 64, &err);
    p->theta_prop = (double *)dmalloc(p, sizeof(double) * 4 * B, &err);
    p->phi_prop = (double *)dmalloc(p, sizeof(double) * 4 * B, &err);
    p->inside = (int *)dmalloc(p, sizeof(int) * B, &err);
    p->need = (int *)dmalloc(p, sizeof(int) * B, &err);
    p->ll_prop = (double *)dmalloc(p, sizeof(double) * B, &err);
    p->ll_sur_prop = (double *)dmalloc(p, sizeof(double) * B, &err);
    p->status_ws = (int *)dmalloc(p, sizeof(int) * B, &err);
    p->iters_ws = (int *)dmalloc(p, sizeof(int) * 2 * B, &err);
    p->pmh_gid = (int *)dmalloc(p, sizeof(int) * B, &err);
    p->order_ws = (int *)dmalloc(p, sizeof(int) * B, &err);
    p->cost_ws = (int *)dmalloc(p, sizeof(int) * B, &err);
    p->coop_timeouts = (unsigned *)dmalloc(p, 64, &err);
    p->steps_ws = (int *)dmalloc(p, sizeof(int) * B, &err);
    p->sub_phi = (double *)dmalloc(p, sizeof(double) * 4 * B, &err);
    p->sub_ll = (double *)dmalloc(p, sizeof(double) * B, &err);
    p->sub_moves = (int *)dmalloc(p, sizeof(int) * B, &err);
    if (err != RD_OK) {
        destroy_problem(p);
        return err;
    }
    // no solve yet: every cost estimate is unknown (-1), and the first queue
    // order is the identity
    if (hipMemset(p->cost_ws, 0xFF, sizeof(int) * B) != hipSuccess ||
        hipMemset(p->iters_ws, 0, sizeof(int) * 2 * B) != hipSuccess ||
        hipMemset(p->coop_timeouts, 0, 64) != hipSuccess) {
        destroy_problem(p);
        return fail(RD_EHIP, "hipMemset of the cost and iteration workspaces failed");
    }
    if (hipMemcpy(p->grids_dev, p->grids_host.data(), sizeof(GridDev) * desc->n_grids,
                  hipMemcpyHostToDevice) != hipSuccess ||
        launch_grid_coeffs(p->grids_dev, desc->n_grids, desc->dt, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        destroy_problem(p);
        return fail(RD_EHIP, "upload of grid table failed");
    }
    // Solve workspace: one slot per resident workgroup, sized for every tile
    // the autotuner may pick (low parts and predictor history, 4 n^2 values,
    // and for streamed tiles the 6 strip arrays as well).
    size_t slot = 0;
    int slots = 0;
    for (int g = 0; g < desc->n_grids; ++g) {
        const int n = p->grids_host[g].n;
        for (int cpt : {4, 8, 16, 32, 64, 128}) {
            if (tile_supported(n, desc->precision, cpt)) {
                slot = std::max(slot, solve_slot_bytes(n, desc->precision, cpt));
                slots = std::max(slots, p->n_cu * solve_wgs_per_cu(n, desc->precision, cpt));
            }
        }
        if (desc->n_grids > 1) {
            for (int threads : {512, 1024}) {
                slot = std::max(slot, mixed_slot_bytes(n, desc->precision, threads));
                slots = std::max(slots, p->n_cu * mixed_wgs_per_cu(desc->precision, threads));
            }
        }
    }
    if (desc->n_grids > 1) {
        // queue order: larger grids first (cost per solve ~ cells)
        std::vector<int> cls(desc->n_grids);
        for (int g = 0; g < desc->n_grids; ++g)
            cls[g] = g;
        std::stable_sort(cls.begin(), cls.end(), [&](int x, int y) {
            return p->grids_host[x].n > p->grids_host[y].n;
        });
        for (int k = 0; k < desc->n_grids; ++k)
            p->rank.r[cls[k]] = k;
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            auto it = g_tuned.find(tune_key(p->device, -1, desc->precision));
            if (it != g_tuned.end())
                p->mixed_threads = it->second;
        }
        p->mixed_wpc = mixed_wgs_per_cu(desc->precision, p->mixed_threads);
    }
    // cooperative tiles: group counters, partial sums and edge rows
    for (int g = 0; g < desc->n_grids; ++g) {
        const int n = p->grids_host[g].n;
        for (int cpt : {4, 8, 16, 32, 64, 128}) {
            if (tile_coop(n, desc->precision, cpt) && !p->coop) {
                p->coop_wpc = solve_wgs_per_cu(n, desc->precision, cpt);
                p->mixed_coop_wpc = mixed_coop_wgs_per_cu();
                p->coop_groups = p->n_cu * p->coop_wpc / kCoopG + 8;
                p->coop = dmalloc(p, coop_workspace_bytes(p->coop_groups), &err);
            }
        }
    }
    slot = (slot + 255) / 256 * 256;
    p->gws = dmalloc(p, slot * (size_t)slots, &err);
    p->gws_stride = slot;
    p->gws_slots = slots;
    if (err != RD_OK) {
        destroy_problem(p);
        return err;
    }
    *out = p;
    return RD_OK;
}

extern "C" int32_t destroy_problem(rd_problem *p)
{
    if (!p)
        return RD_OK;
    hipDeviceSynchronize();
    drop_graphs(p);
    if (p->sur)
        surrogate_destroy(p->sur);
    for (auto &pr : p->pending) {
        hipEventDestroy(pr.first);
        hipEventDestroy(pr.second);
    }
    for (auto e : p->free_events)
        hipEventDestroy(e);
    for (void *a : p->allocs)
        hipFree(a);
    delete p;
    return RD_OK;
}

static int32_t check_batch(rd_problem *p, int32_t n)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (n < 0 || n > p->desc.max_batch)
        return fail(RD_EINVAL, "n = %d outside [0, max_batch=%d]", n, p->desc.max_batch);
    return RD_OK;
}

extern "C" int32_t forward_solve_batch(rd_problem *p, int32_t n, const double *theta,
                                       const int32_t *grid_id, void *u_out, void *v_out,
                                       int32_t *status, int32_t *cg_iters, void *stream)
{
    int32_t r = check_batch(p, n);
    if (r != RD_OK)
        return r;
    if (n > 0 && (!status || !theta))
        return fail(RD_EINVAL, "theta and status are required");
    return enqueue_solve(p, n, theta, grid_id, nullptr, nullptr, status, cg_iters, u_out, v_out,
                         (hipStream_t)stream);
}

extern "C" int32_t forward_solve_steady_batch(rd_problem *p, int32_t n, const double *theta,
                                              const int32_t *grid_id, void *u_out, void *v_out,
                                              int32_t *status, int32_t *cg_iters,
                                              int32_t *steps_out, void *stream)
{
    int32_t r = check_batch(p, n);
    if (r != RD_OK)
        return r;
    if (n > 0 && (!status || !theta || !steps_out))
        return fail(RD_EINVAL, "theta, status and steps_out are required");
    return enqueue_solve(p, n, theta, grid_id, nullptr, nullptr, status, cg_iters, u_out, v_out,
                         (hipStream_t)stream, 0, steps_out);
}

extern "C" int32_t log_likelihood_batch(rd_problem *p, int32_t n, const double *theta,
                                        const int32_t *grid_id, double *phi, int32_t *status,
                                        int32_t *cg_iters, void *stream)
{
    int32_t r = check_batch(p, n);
    if (r != RD_OK)
        return r;
    if (n > 0 && (!status || !phi || !theta))
        return fail(RD_EINVAL, "theta, phi and status are required");
    for (auto &g : p->grids_host)
        if (!g.y)
            return fail(RD_EINVAL, "a grid class has no data y");
    return enqueue_solve(p, n, theta, grid_id, nullptr, phi, status, cg_iters, nullptr, nullptr,
                         (hipStream_t)stream);
}

extern "C" int32_t log_likelihood_batch_noalloc(rd_problem *p, int32_t n, const double *theta,
                                                double *phi, int32_t *status, int32_t *cg_iters,
                                                void *stream)
{
    int32_t r = check_batch(p, n);
    if (r != RD_OK)
        return r;
    if (n > 0 && (!status || !phi || !theta))
        return fail(RD_EINVAL, "theta, phi and status are required");
    if (p->desc.n_grids != 1)
        return fail(RD_EUNSUPPORTED, "log_likelihood_batch_noalloc takes one grid class");
    if (!p->grids_host[0].y)
        return fail(RD_EINVAL, "grid 0 has no data y");
    const int nn = p->grids_host[0].n;
    const TileChoice t = p->tile[0];
    if (tile_coop(nn, p->desc.precision, t.cpt))
        return fail(RD_EUNSUPPORTED,
                    "log_likelihood_batch_noalloc: the cooperative %dx%d tile needs the problem's "
                    "group workspace (select a streamed tile with rd_set_tile)", nn, nn);
    if (!p->scratch)
        return fail(RD_EHIP, "no scratch address for device %d", p->device);
    const size_t stride = (solve_slot_bytes(nn, p->desc.precision, t.cpt) + 255) / 256 * 256;
    const size_t slots = kNoAllocSlots / stride;
    if (slots < 1)
        return fail(RD_EUNSUPPORTED,
                    "log_likelihood_batch_noalloc: one solve slot (%zu bytes) exceeds the %zu "
                    "bytes of scratch", stride, kNoAllocSlots);
    if (n == 0)
        return RD_OK;
    SolveWs ws{(unsigned *)p->scratch, (char *)p->scratch + kNoAllocHeader, stride,
               (int)std::min<size_t>(slots, (size_t)1 << 20)};
    return enqueue_solve(p, n, theta, nullptr, nullptr, phi, status, cg_iters, nullptr, nullptr,
                         (hipStream_t)stream, 0, nullptr, nullptr, &ws);
}

extern "C" int32_t field_misfit_batch(rd_problem *p, int32_t n, const void *u,
                                      const int32_t *grid_id, double *phi, void *stream)
{
    int32_t r = check_batch(p, n);
    if (r != RD_OK)
        return r;
    if (n > 0 && (!u || !phi))
        return fail(RD_EINVAL, "u and phi are required");
    if (p->desc.n_grids != 1)
        return fail(RD_EUNSUPPORTED, "field_misfit_batch takes problems with one grid class");
    if (!p->grids_host[0].y)
        return fail(RD_EINVAL, "grid 0 has no data y");
    (void)grid_id;  // one class: every field is compared with grid 0's data
    const int npts = p->grids_host[0].n * p->grids_host[0].n;
    HIP_TRY(launch_field_misfit(p->desc.precision, p->grids_dev, nullptr, n, npts, u, phi,
                                (hipStream_t)stream));
    return RD_OK;
}

extern "C" int32_t mcmc_step_batch(rd_problem *p, rd_chains *chains, int32_t n_steps, int32_t mode,
                                   void *stream)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (mode != RD_MODE_PLAIN && mode != RD_MODE_DA)
        return fail(RD_EINVAL, "mode must be 0 (plain) or 1 (delayed acceptance)");
    int32_t r = check_chains(p, chains, mode);
    if (r != RD_OK)
        return r;
    if (n_steps < 0)
        return fail(RD_EINVAL, "n_steps < 0");
    if (mode == RD_MODE_DA && (!p->sur || !surrogate_ready(p->sur)))
        return fail(RD_EUNSUPPORTED, "delayed acceptance needs a trained surrogate with scaling");
    for (auto &g : p->grids_host)
        if (!g.y)
            return fail(RD_EINVAL, "a grid class has no data y");
    if (n_steps == 0 || chains->n_chains == 0) {
        chains->step += (uint64_t)n_steps;
        return RD_OK;
    }
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_set_ctr(p->ctr, chains->step, chains->trace_step0, s));
    // Graph capture needs a created stream (the legacy null stream cannot
    // be captured); the null stream and timing runs use direct launches.
    const bool graphs = p->use_graphs && !p->timing && s != nullptr;
    if (!graphs) {
        for (int k = 0; k < n_steps; ++k)
            if ((r = enqueue_mcmc_step(p, chains, mode, s)) != RD_OK)
                return r;
        chains->step += (uint64_t)n_steps;
        return RD_OK;
    }
    GraphEntry *ge = nullptr;
    for (auto &g : p->graphs)
        if (same_chains(g.key, *chains) && g.mode == mode && g.stream == s)
            ge = &g;
    int done = 0;
    if (!ge) {
        // The first step of a new layout runs as direct launches, so every
        // kernel of the sequence has been loaded and launched once before
        // capture begins; capture then records launches only.  The layout
        // is remembered, so that with one step per call the second call
        // captures.
        bool warm = false;
        for (auto &w : p->warm)
            if (same_chains(w.key, *chains) && w.mode == mode && w.stream == s)
                warm = true;
        if (!warm) {
            if ((r = enqueue_mcmc_step(p, chains, mode, s)) != RD_OK)
                return r;
            GraphEntry w;
            w.key = *chains;
            w.mode = mode;
            w.stream = s;
            p->warm.push_back(w);
            done = 1;
            if (done == n_steps) {
                chains->step += (uint64_t)n_steps;
                return RD_OK;
            }
        }
        GraphEntry g;
        g.key = *chains;
        g.mode = mode;
        g.stream = s;
        HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
        r = enqueue_mcmc_step(p, chains, mode, s);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(s, &graph);
        if (r != RD_OK) {
            if (graph)
                hipGraphDestroy(graph);
            return r;
        }
        if (e != hipSuccess)
            return fail(RD_EHIP, "graph capture: %s", hipGetErrorString(e));
        g.graph = graph;
        e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) {
            hipGraphDestroy(graph);
            return fail(RD_EHIP, "graph instantiate: %s", hipGetErrorString(e));
        }
        p->graphs.push_back(g);
        ge = &p->graphs.back();
    }
    for (int k = done; k < n_steps; ++k)
        HIP_TRY(hipGraphLaunch(ge->exec, s));
    chains->step += (uint64_t)n_steps;
    return RD_OK;
}

extern "C" int32_t propose_batch(rd_problem *p, rd_chains *chains, double *phi_prop,
                                 int32_t *inside, void *stream)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    int32_t r = check_chains(p, chains, RD_MODE_PLAIN);
    if (r != RD_OK)
        return r;
    if (!phi_prop || !inside)
        return fail(RD_EINVAL, "phi_prop and inside are required");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_set_ctr(p->ctr, chains->step, chains->trace_step0, s));
    SamplerArgs a = sampler_args(p, chains);
    a.phi_prop = phi_prop;
    a.inside = inside;
    a.theta_prop = nullptr;
    HIP_TRY(launch_propose(a, s));
    return RD_OK;
}

extern "C" int32_t accept_batch(rd_problem *p, rd_chains *chains, const double *phi_prop,
                                const int32_t *inside, const double *loglik_prop, void *stream)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    int32_t r = check_chains(p, chains, RD_MODE_PLAIN);
    if (r != RD_OK)
        return r;
    if (!phi_prop || !inside || !loglik_prop)
        return fail(RD_EINVAL, "phi_prop, inside and loglik_prop are required");
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_set_ctr(p->ctr, chains->step, chains->trace_step0, s));
    SamplerArgs a = sampler_args(p, chains);
    a.phi_prop = const_cast<double *>(phi_prop);
    a.inside = const_cast<int *>(inside);
    a.loglik_prop = loglik_prop;
    // the caller's Phi did not come from this library's solve
    a.iters = nullptr;
    a.steps = nullptr;
    a.status = nullptr;
    HIP_TRY(launch_accept(a, s));
    chains->step += 1;
    return RD_OK;
}

static int32_t check_pmh(rd_problem *p, rd_chains *chains, int n_prop)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    int32_t r = check_chains(p, chains, RD_MODE_PLAIN);
    if (r != RD_OK)
        return r;
    if (n_prop < 1 || n_prop > kMaxPmhProposals)
        return fail(RD_EINVAL, "n_prop = %d outside [1, %d]", n_prop, kMaxPmhProposals);
    if ((int64_t)chains->n_chains * n_prop > p->desc.max_batch)
        return fail(RD_EINVAL, "n_chains * n_prop = %lld exceeds max_batch = %d",
                    (long long)chains->n_chains * n_prop, p->desc.max_batch);
    return RD_OK;
}

extern "C" int32_t pmh_step_batch(rd_problem *p, rd_chains *chains, int32_t n_prop,
                                  int32_t n_iter, void *stream)
{
    int32_t r = check_pmh(p, chains, n_prop);
    if (r != RD_OK)
        return r;
    if (n_iter < 0)
        return fail(RD_EINVAL, "n_iter < 0");
    for (auto &g : p->grids_host)
        if (!g.y)
            return fail(RD_EINVAL, "a grid class has no data y");
    hipStream_t s = (hipStream_t)stream;
    const int n = chains->n_chains;
    const int items = n * n_prop;
    for (int k = 0; k < n_iter && n > 0; ++k) {
        HIP_TRY(launch_set_ctr(p->ctr, chains->step, chains->trace_step0, s));
        SamplerArgs a = sampler_args(p, chains);
        a.phi_prop = p->phi_prop;
        a.theta_prop = p->theta_prop;
        a.inside = p->inside;
        a.loglik_prop = p->ll_prop;
        HIP_TRY(launch_pmh_propose(a, n_prop, s));
        const int *gid = nullptr;
        if (chains->grid_id && p->desc.n_grids > 1) {
            HIP_TRY(launch_pmh_expand_gid(chains->grid_id, n, n_prop, p->pmh_gid, s));
            gid = p->pmh_gid;
        }
        r = enqueue_solve(p, items, p->theta_prop, gid, p->inside, p->ll_prop, p->status_ws,
                          p->iters_ws, nullptr, nullptr, s, 0, p->steps_ws);
        if (r != RD_OK)
            return r;
        HIP_TRY(launch_pmh_resample(a, n_prop, s));
        chains->step += (uint64_t)n_prop;
    }
    return RD_OK;
}

extern "C" int32_t pmh_propose_batch(rd_problem *p, rd_chains *chains, int32_t n_prop,
                                     double *phi_prop, int32_t *inside, void *stream)
{
    int32_t r = check_pmh(p, chains, n_prop);
    if (r != RD_OK)
        return r;
    if (!phi_prop || !inside)
        return fail(RD_EINVAL, "phi_prop and inside are required");
    if (chains->n_chains == 0)
        return RD_OK;
    hipStream_t s = (hipStream_t)stream;
    HIP_TRY(launch_set_ctr(p->ctr, chains->step, chains->trace_step0, s));
    SamplerArgs a = sampler_args(p, chains);
    a.phi_prop = phi_prop;
    a.inside = inside;
    a.theta_prop = nullptr;
    HIP_TRY(launch_pmh_propose(a, n_prop, s));
    return RD_OK;
}

extern "C" int32_t pmh_resample_batch(rd_problem *p, rd_chains *chains, int32_t n_prop,
                                      const double *phi_prop, const int32_t *inside,
                                      const double *loglik_prop, void *stream)
{
    int32_t r = check_pmh(p, chains, n_prop);
    if (r != RD_OK)
        return r;
    if (!phi_prop || !inside || !loglik_prop)
        return fail(RD_EINVAL, "phi_prop, inside and loglik_prop are required");
    hipStream_t s = (hipStream_t)stream;
    if (chains->n_chains > 0) {
        HIP_TRY(launch_set_ctr(p->ctr, chains->step, chains->trace_step0, s));
        SamplerArgs a = sampler_args(p, chains);
        a.phi_prop = const_cast<double *>(phi_prop);
        a.inside = const_cast<int *>(inside);
        a.loglik_prop = loglik_prop;
        // the caller's Phi did not come from this library's solve
        a.iters = nullptr;
        a.steps = nullptr;
        a.status = nullptr;
        HIP_TRY(launch_pmh_resample(a, n_prop, s));
    }
    chains->step += (uint64_t)n_prop;
    return RD_OK;
}

// Trial parameters of the autotuner: a fixed low-discrepancy spread over the
// prior box (the additive recurrence with the plastic-number constants), so
// that the trial sees the mix of cheap and expensive solves a sampler sees.
static void trial_theta(const rd_problem_desc &d, int k, double *th)
{
    static const double alpha[4] = {0.7548776662466927, 0.5698402909980532, 0.4301597090019468,
                                    0.2451223337533073};
    for (int i = 0; i < 4; ++i) {
        const double f = std::fmod(0.5 + alpha[i] * (k + 1), 1.0);
        const double x = d.lo[i] + f * (d.hi[i] - d.lo[i]);
        th[i] = i < 2 ? x : exp(x);
    }
}

// A candidate replaces the current tile only when it is faster by more than
// this fraction (trial timings vary by a few per cent between runs).
constexpr float kTuneMargin = 0.03f;

extern "C" int32_t rd_autotune(rd_problem *p, int32_t *cpt_out)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    // Trial: one solve per resident workgroup slot over a short horizon, on
    // a low-discrepancy spread of the prior box; grids above 128^2 run
    // fewer steps (their tiles cost up to seconds per 160 steps).
    for (int g = 0; g < p->desc.n_grids; ++g) {
        const int n = p->grids_host[g].n;
        const int trial_steps =
            std::min(p->desc.n_steps, n > 128 ? std::max(20, 160 * 128 * 128 / (n * n)) : 160);
        int best = p->tile[g].cpt;
        float best_ms = 1e30f;
        for (int cpt : {4, 8, 16, 32, 64, 128}) {
            const bool coop = tile_coop(n, p->desc.precision, cpt);
            if (!tile_supported(n, p->desc.precision, cpt) ||
                (!coop && (n * n / cpt > 1024 || n * n / cpt < 64)))
                continue;
            int items = std::min(p->desc.max_batch, p->n_cu * solve_wgs_per_cu(n, p->desc.precision, cpt));
            if (coop)  // a group of workgroups per item
                items = std::max(1, items / kCoopG);
            std::vector<double> th(4 * items);
            for (int k = 0; k < items; ++k) {
                trial_theta(p->desc, k, &th[4 * k]);
            }
            double *d_th = nullptr;
            int *d_st = nullptr;
            HIP_TRY(hipMalloc(&d_th, sizeof(double) * th.size()));
            HIP_TRY(hipMalloc(&d_st, sizeof(int) * items));
            HIP_TRY(hipMemcpy(d_th, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice));
            const TileChoice saved = p->tile[g];
            const int saved_wpc = p->wgs_per_cu[g];
            const int saved_steps = p->desc.n_steps;
            p->tile[g] = TileChoice{cpt, n * n / cpt};
            p->wgs_per_cu[g] = solve_wgs_per_cu(n, p->desc.precision, cpt);
            p->desc.n_steps = trial_steps;
            hipEvent_t e0, e1;
            hipEventCreate(&e0);
            hipEventCreate(&e1);
            const bool saved_timing = p->timing;
            p->timing = false;
            int32_t r = enqueue_solve(p, items, d_th, nullptr, nullptr, nullptr, d_st, nullptr,
                                      nullptr, nullptr, nullptr, g);
            hipEventRecord(e0, nullptr);
            if (r == RD_OK)
                r = enqueue_solve(p, items, d_th, nullptr, nullptr, nullptr, d_st, nullptr,
                                  nullptr, nullptr, nullptr, g);
            hipEventRecord(e1, nullptr);
            hipEventSynchronize(e1);
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            p->timing = saved_timing;
            p->desc.n_steps = saved_steps;
            p->tile[g] = saved;
            p->wgs_per_cu[g] = saved_wpc;
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            hipFree(d_th);
            hipFree(d_st);
            if (r != RD_OK)
                return r;
            // time per item (the slot counts differ between tiles)
            float per_item = ms / (float)items;
            if (getenv("RDBAYES_AUTOTUNE_VERBOSE"))
                fprintf(stderr, "[rd_autotune] n=%d prec=%d cpt=%d threads=%d wgs/cu=%d: %.4f ms/item\n",
                        n, p->desc.precision, cpt, n * n / cpt,
                        solve_wgs_per_cu(n, p->desc.precision, cpt), per_item);
            if (cpt == p->tile[g].cpt)
                per_item *= 1.0f - kTuneMargin;  // incumbent
            if (per_item < best_ms) {
                best_ms = per_item;
                best = cpt;
            }
        }
        p->tile[g] = TileChoice{best, n * n / best};
        p->wgs_per_cu[g] = solve_wgs_per_cu(n, p->desc.precision, best);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned[tune_key(p->device, n, p->desc.precision)] = best;
        }
        if (cpt_out)
            cpt_out[g] = best;
    }
    if (p->desc.n_grids > 1) {
        // Mixed launch: workgroup size, on a batch that cycles through the
        // classes (one item per workgroup slot).
        const int trial_steps = std::min(p->desc.n_steps, 160);
        int best = p->mixed_threads;
        float best_ms = 1e30f;
        for (int threads : {512, 1024}) {
            const int wpc = mixed_wgs_per_cu(p->desc.precision, threads);
            const int items = std::min(p->desc.max_batch, p->n_cu * wpc);
            std::vector<double> th(4 * items);
            std::vector<int> gid(items);
            for (int k = 0; k < items; ++k) {
                trial_theta(p->desc, k, &th[4 * k]);
                gid[k] = k % p->desc.n_grids;
            }
            double *d_th = nullptr;
            int *d_st = nullptr, *d_gid = nullptr;
            HIP_TRY(hipMalloc(&d_th, sizeof(double) * th.size()));
            HIP_TRY(hipMalloc(&d_st, sizeof(int) * items));
            HIP_TRY(hipMalloc(&d_gid, sizeof(int) * items));
            HIP_TRY(hipMemcpy(d_th, th.data(), sizeof(double) * th.size(), hipMemcpyHostToDevice));
            HIP_TRY(hipMemcpy(d_gid, gid.data(), sizeof(int) * items, hipMemcpyHostToDevice));
            const int saved_threads = p->mixed_threads, saved_wpc = p->mixed_wpc;
            const int saved_steps = p->desc.n_steps;
            p->mixed_threads = threads;
            p->mixed_wpc = wpc;
            p->desc.n_steps = trial_steps;
            const bool saved_timing = p->timing;
            p->timing = false;
            hipEvent_t e0, e1;
            hipEventCreate(&e0);
            hipEventCreate(&e1);
            int32_t r = enqueue_solve(p, items, d_th, d_gid, nullptr, nullptr, d_st, nullptr,
                                      nullptr, nullptr, nullptr);
            hipEventRecord(e0, nullptr);
            if (r == RD_OK)
                r = enqueue_solve(p, items, d_th, d_gid, nullptr, nullptr, d_st, nullptr, nullptr,
                                  nullptr, nullptr);
            hipEventRecord(e1, nullptr);
            hipEventSynchronize(e1);
            float ms = 0.f;
            hipEventElapsedTime(&ms, e0, e1);
            p->timing = saved_timing;
            p->desc.n_steps = saved_steps;
            p->mixed_threads = saved_threads;
            p->mixed_wpc = saved_wpc;
            hipEventDestroy(e0);
            hipEventDestroy(e1);
            hipFree(d_th);
            hipFree(d_st);
            hipFree(d_gid);
            if (r != RD_OK)
                return r;
            float per_item = ms / (float)items;
            if (getenv("RDBAYES_AUTOTUNE_VERBOSE"))
                fprintf(stderr, "[rd_autotune] mixed prec=%d threads=%d wgs/cu=%d: %.4f ms/item\n",
                        p->desc.precision, threads, wpc, per_item);
            if (threads == p->mixed_threads)
                per_item *= 1.0f - kTuneMargin;  // incumbent
            if (per_item < best_ms) {
                best_ms = per_item;
                best = threads;
            }
        }
        p->mixed_threads = best;
        p->mixed_wpc = mixed_wgs_per_cu(p->desc.precision, best);
        {
            std::lock_guard<std::mutex> lk(g_tune_mu);
            g_tuned[tune_key(p->device, -1, p->desc.precision)] = best;
        }
    }
    drop_graphs(p);
    return RD_OK;
}

extern "C" int32_t rd_set_tile(rd_problem *p, int32_t grid, int32_t cpt)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (grid < 0 || grid >= p->desc.n_grids)
        return fail(RD_EINVAL, "grid %d outside [0, %d)", grid, p->desc.n_grids);
    const int n = p->grids_host[grid].n;
    if (cpt <= 0 || !tile_supported(n, p->desc.precision, cpt))
        return fail(RD_EUNSUPPORTED, "no tile with %d cells per thread at n = %d", cpt, n);
    // the workspace was sized for every supported tile of this class
    p->tile[grid] = TileChoice{cpt, n * n / cpt};
    p->wgs_per_cu[grid] = solve_wgs_per_cu(n, p->desc.precision, cpt);
    drop_graphs(p);  // captured steps launch with the tile of their capture
    return RD_OK;
}

extern "C" int32_t rd_set_mixed_threads(rd_problem *p, int32_t threads)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (threads != 512 && threads != 1024)
        return fail(RD_EINVAL, "threads must be 512 or 1024, got %d", threads);
    p->mixed_threads = threads;
    p->mixed_wpc = mixed_wgs_per_cu(p->desc.precision, threads);
    drop_graphs(p);  // captured steps launch with the shape of their capture
    return RD_OK;
}

extern "C" int32_t rd_check_solves(rd_problem *p, int64_t *group_timeouts, int32_t reset)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    HIP_TRY(hipDeviceSynchronize());
    unsigned count = 0;
    HIP_TRY(hipMemcpy(&count, p->coop_timeouts, sizeof(unsigned), hipMemcpyDeviceToHost));
    if (group_timeouts)
        *group_timeouts = (int64_t)count;
    if (reset && count)
        HIP_TRY(hipMemset(p->coop_timeouts, 0, sizeof(unsigned)));
    if (count)
        return fail(RD_ETIMEOUT,
                    "%u cooperative workgroup(s) gave up a group wait: the items they served "
                    "carry RD_ST_GROUP_TIMEOUT (Phi = +inf)",
                    count);
    return RD_OK;
}

extern "C" int32_t rd_set_coop_wait(rd_problem *p, int64_t wait_ticks, int64_t stall_ticks)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (wait_ticks < 0 || stall_ticks < 0 || stall_ticks > 100000000)
        return fail(RD_EINVAL, "wait_ticks >= 0 and 0 <= stall_ticks <= 1e8 required");
    p->coop_wait_ticks = wait_ticks > 0 ? (unsigned long long)wait_ticks : 1000000000ull;
    p->coop_stall_ticks = (unsigned long long)stall_ticks;
    drop_graphs(p);  // captured launches carry the old values
    return RD_OK;
}

extern "C" int32_t rd_set_da_substeps(rd_problem *p, int32_t substeps)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (substeps < 1 || substeps > 256)
        return fail(RD_EINVAL, "substeps must be in [1, 256], got %d", substeps);
    p->da_substeps = substeps;
    drop_graphs(p);  // captured steps carry the substep count of their capture
    return RD_OK;
}

extern "C" int32_t rd_captured_graphs(const rd_problem *p, int32_t *count)
{
    if (!p || !count)
        return fail(RD_EINVAL, "problem and count are required");
    *count = (int32_t)p->graphs.size();
    return RD_OK;
}

extern "C" int32_t rd_mixed_threads(const rd_problem *p, int32_t *threads)
{
    if (!p || !threads)
        return fail(RD_EINVAL, "problem and threads are required");
    *threads = p->mixed_threads;
    return RD_OK;
}

extern "C" int32_t rd_solver_timing(rd_problem *p, int32_t enable, double *ms_total,
                                    int64_t *launches, int32_t reset)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    for (auto &pr : p->pending) {
        HIP_TRY(hipEventSynchronize(pr.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, pr.first, pr.second));
        p->ms_total += ms;
        p->launches += 1;
        p->free_events.push_back(pr.first);
        p->free_events.push_back(pr.second);
    }
    p->pending.clear();
    if (ms_total)
        *ms_total = p->ms_total;
    if (launches)
        *launches = p->launches;
    if (reset) {
        p->ms_total = 0.0;
        p->launches = 0;
    }
    p->timing = enable != 0;
    return RD_OK;
}

extern "C" const char *rd_status_string(int32_t s)
{
    switch (s) {
    case RD_OK: return "ok";
    case RD_EINVAL: return "invalid argument";
    case RD_EHIP: return "HIP runtime error";
    case RD_ENOMEM: return "out of device memory";
    case RD_EUNSUPPORTED: return "unsupported configuration";
    case RD_ETIMEOUT: return "a cooperative group wait gave up";
    case RD_EIO: return "file error";
    case RD_ST_NOT_CONVERGED: return "CG not converged";
    case RD_ST_BREAKDOWN: return "CG breakdown (operator not positive definite)";
    case RD_ST_NONFINITE: return "non-finite value";
    case RD_ST_OUT_OF_PRIOR: return "outside the prior box";
    case RD_ST_BAD_GRID: return "grid id outside [0, n_grids)";
    case RD_ST_NOT_STEADY: return "no steady state within n_steps";
    case RD_ST_GROUP_TIMEOUT: return "cooperative group wait gave up (solve abandoned)";
    default: return "combination of status flags";
    }
}

extern "C" const char *rd_last_error(void)
{
    return g_err;
}

// ---------------------------------------------------------------------------
// Surrogate entry points (implemented in rd_mlp.hip).

extern "C" int32_t surrogate_create(rd_problem *p, int32_t width, int32_t depth, int32_t out_side,
                                    uint32_t seed)
{
    if (!p)
        return fail(RD_EINVAL, "problem is NULL");
    if (width <= 0 || width % 64 || depth < 1 || depth > 8 || out_side <= 0 ||
        p->grids_host[0].n % out_side || (out_side * out_side) % 64)
        return fail(RD_EINVAL, "surrogate shape: width %% 64 == 0, 1 <= depth <= 8, out_side | n");
    if (p->sur)
        surrogate_destroy(p->sur);
    p->sur = nullptr;
    drop_graphs(p);
    SurrogateDesc d{};
    d.width = width;
    d.depth = depth;
    d.out_side = out_side;
    d.n = p->grids_host[0].n;
    d.precision = p->desc.precision;
    for (int i = 0; i < 4; ++i) {
        d.lo[i] = p->desc.lo[i];
        d.hi[i] = p->desc.hi[i];
    }
    d.y = p->grids_host[0].y;
    d.max_batch = std::max(p->desc.max_batch, 4096);
    int32_t r = surrogate_new(&p->sur, d, seed);
    if (r != RD_OK)
        return fail(r, "surrogate allocation failed");
    return RD_OK;
}

extern "C" int32_t downsample_batch(rd_problem *p, int32_t n, const void *u, float *out,
                                    void *stream)
{
    int32_t r = check_batch(p, n);
    if (r != RD_OK && n <= 0)
        return r;
    if (!p || !p->sur)
        return fail(RD_EINVAL, "downsample_batch needs surrogate_create first");
    if (n < 0 || (n > 0 && (!u || !out)))
        return fail(RD_EINVAL, "u and out are required");
    HIP_TRY(surrogate_downsample(p->sur, n, u, out, (hipStream_t)stream));
    return RD_OK;
}

extern "C" int32_t surrogate_set_scaling(rd_problem *p, const float *mean, const float *sd,
                                         double sigma1, void *stream)
{
    if (!p || !p->sur)
        return fail(RD_EINVAL, "surrogate_set_scaling needs surrogate_create first");
    if (!mean || !sd || !(sigma1 > 0.0))
        return fail(RD_EINVAL, "mean, sd and sigma1 > 0 are required");
    if (!p->grids_host[0].y)
        return fail(RD_EINVAL, "grid 0 has no data y");
    HIP_TRY(surrogate_scaling(p->sur, mean, sd, sigma1, (hipStream_t)stream));
    drop_graphs(p);
    return RD_OK;
}

extern "C" int32_t surrogate_set_input_box(rd_problem *p, const double *lo, const double *hi)
{
    if (!p || !p->sur)
        return fail(RD_EINVAL, "surrogate_set_input_box needs surrogate_create first");
    if (!lo || !hi)
        return fail(RD_EINVAL, "lo and hi are required");
    for (int i = 0; i < 4; ++i)
        if (!(lo[i] < hi[i]) || !std::isfinite(lo[i]) || !std::isfinite(hi[i]))
            return fail(RD_EINVAL, "input box coordinate %d: need finite lo < hi", i);
    surrogate_input_box(p->sur, lo, hi);
    drop_graphs(p);
    return RD_OK;
}

extern "C" int32_t surrogate_train_step(rd_problem *p, int32_t batch, const double *phi,
                                        const float *target, double lr, double *loss_out,
                                        void *stream)
{
    if (!p || !p->sur)
        return fail(RD_EINVAL, "surrogate_train_step needs surrogate_create first");
    if (batch < 1 || batch > surrogate_max_batch(p->sur) || !phi || !target || !(lr > 0.0))
        return fail(RD_EINVAL, "batch in [1, %d], phi, target and lr > 0 required",
                    surrogate_max_batch(p->sur));
    HIP_TRY(surrogate_train(p->sur, batch, phi, target, lr, loss_out, (hipStream_t)stream));
    return RD_OK;
}

extern "C" int32_t surrogate_forward(rd_problem *p, int32_t n, const double *phi, float *out,
                                     int32_t raw, void *stream)
{
    if (!p || !p->sur)
        return fail(RD_EINVAL, "surrogate_forward needs surrogate_create first");
    if (n < 0 || n > surrogate_max_batch(p->sur) || (n > 0 && (!phi || !out)))
        return fail(RD_EINVAL, "n in [0, %d], phi and out required", surrogate_max_batch(p->sur));
    if (!raw && !surrogate_ready(p->sur))
        return fail(RD_EINVAL, "de-standardised output needs surrogate_set_scaling");
    HIP_TRY(surrogate_predict(p->sur, n, phi, out, raw, (hipStream_t)stream));
    return RD_OK;
}

extern "C" int32_t surrogate_loglik_batch(rd_problem *p, int32_t n, const double *phi,
                                          double *phi_sur, void *stream)
{
    if (!p || !p->sur || !surrogate_ready(p->sur))
        return fail(RD_EINVAL, "surrogate_loglik_batch needs a surrogate with scaling");
    if (n < 0 || n > surrogate_max_batch(p->sur) || (n > 0 && (!phi || !phi_sur)))
        return fail(RD_EINVAL, "n in [0, %d], phi and phi_sur required", surrogate_max_batch(p->sur));
    int32_t r = surrogate_enqueue_loglik(p->sur, n, phi, phi_sur, (hipStream_t)stream);
    if (r != RD_OK)
        return fail(r, "surrogate evaluation failed");
    return RD_OK;
}

extern "C" int32_t surrogate_params(rd_problem *p, int32_t layer, float *w, float *b, int32_t dir,
                                    void *stream)
{
    if (!p || !p->sur)
        return fail(RD_EINVAL, "surrogate_params needs surrogate_create first");
    if (layer < 0 || layer > surrogate_layers(p->sur) - 1 || dir < 0 || dir > 2 || !w || !b)
        return fail(RD_EINVAL, "layer in [0, %d], dir 0/1/2, w and b required",
                    surrogate_layers(p->sur) - 1);
    HIP_TRY(surrogate_copy_params(p->sur, layer, w, b, dir, (hipStream_t)stream));
    if (dir == 1)
        drop_graphs(p);
    return RD_OK;
}

// ---- chain state to and from a file ---------------------------------------
// Layout (little-endian, as the host writes it): a 48-byte header, then the
// arrays the header's mask names, in the order of kChainArrays, each
// n_chains x width elements of elem bytes.
namespace {

constexpr char kChainMagic[8] = {'R', 'D', 'C', 'H', 'A', 'I', 'N', 'S'};
constexpr uint32_t kChainVersion = 1;

struct ChainFileHeader {
    char magic[8];
    uint32_t version;
    int32_t n_chains;
    uint32_t seed;
    uint32_t mask;  // bit k: array k of kChainArrays follows
    uint64_t step;
    uint64_t reserved[2];
};
static_assert(sizeof(ChainFileHeader) == 48, "chain file header is 48 bytes");

struct ChainArray {
    const char *name;
    size_t elem, width;
};
// the order of the arrays in the file
constexpr ChainArray kChainArrays[] = {
    {"phi", 8, 4},        {"loglik", 8, 1},   {"loglik_sur", 8, 1}, {"grid_id", 4, 1},
    {"n_accept", 8, 1},   {"n_accept1", 8, 1}, {"n_solves", 8, 1},  {"cg_iters", 8, 2},
    {"imex_steps", 8, 1}, {"fail_bits", 8, 8},
};
constexpr int kNChainArrays = (int)(sizeof(kChainArrays) / sizeof(kChainArrays[0]));

// Device address of array k of the chains (NULL where the caller has none).
const void *chain_array(const rd_chains *c, int k)
{
    switch (k) {
    case 0: return c->phi;
    case 1: return c->loglik;
    case 2: return c->loglik_sur;
    case 3: return c->grid_id;
    case 4: return c->n_accept;
    case 5: return c->n_accept1;
    case 6: return c->n_solves;
    case 7: return c->cg_iters;
    case 8: return c->imex_steps;
    case 9: return c->fail_bits;
    default: return nullptr;
    }
}

struct File {
    FILE *f = nullptr;
    ~File()
    {
        if (f)
            fclose(f);
    }
};

}  // namespace

extern "C" int32_t rd_chains_save(const rd_chains *c, const char *path, void *stream)
{
    if (!c || !path)
        return fail(RD_EINVAL, "rd_chains_save: chains and path are required");
    if (c->n_chains < 0 || !c->phi || !c->loglik)
        return fail(RD_EINVAL, "rd_chains_save: n_chains >= 0, phi and loglik are required");
    const hipStream_t s = (hipStream_t)stream;
    ChainFileHeader h{};
    memcpy(h.magic, kChainMagic, sizeof h.magic);
    h.version = kChainVersion;
    h.n_chains = c->n_chains;
    h.seed = c->seed;
    h.step = c->step;
    std::vector<std::vector<unsigned char>> host(kNChainArrays);
    for (int k = 0; k < kNChainArrays; ++k) {
        const void *d = chain_array(c, k);
        if (!d)
            continue;
        h.mask |= 1u << k;
        host[k].resize((size_t)c->n_chains * kChainArrays[k].elem * kChainArrays[k].width);
        if (!host[k].empty())
            HIP_TRY(hipMemcpyAsync(host[k].data(), d, host[k].size(), hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    File out;
    out.f = fopen(path, "wb");
    if (!out.f)
        return fail(RD_EIO, "rd_chains_save: cannot open %s for writing", path);
    bool ok = fwrite(&h, sizeof h, 1, out.f) == 1;
    for (int k = 0; k < kNChainArrays && ok; ++k)
        if (!host[k].empty())
            ok = fwrite(host[k].data(), 1, host[k].size(), out.f) == host[k].size();
    ok = (fclose(out.f) == 0) && ok;
    out.f = nullptr;
    if (!ok)
        return fail(RD_EIO, "rd_chains_save: write to %s failed", path);
    return RD_OK;
}

extern "C" int32_t rd_chains_load(rd_chains *c, const char *path, void *stream)
{
    if (!c || !path)
        return fail(RD_EINVAL, "rd_chains_load: chains and path are required");
    if (c->n_chains < 0 || !c->phi || !c->loglik)
        return fail(RD_EINVAL, "rd_chains_load: n_chains >= 0, phi and loglik are required");
    File in;
    in.f = fopen(path, "rb");
    if (!in.f)
        return fail(RD_EIO, "rd_chains_load: cannot open %s", path);
    ChainFileHeader h{};
    if (fread(&h, sizeof h, 1, in.f) != 1)
        return fail(RD_EIO, "rd_chains_load: %s is shorter than the header", path);
    if (memcmp(h.magic, kChainMagic, sizeof h.magic) != 0 || h.version != kChainVersion)
        return fail(RD_EINVAL, "rd_chains_load: %s is not a version-%u chain file", path,
                    kChainVersion);
    if (h.n_chains != c->n_chains)
        return fail(RD_EINVAL, "rd_chains_load: the file holds %d chains, the state %d",
                    h.n_chains, c->n_chains);
    if (h.mask >> kNChainArrays)
        return fail(RD_EINVAL, "rd_chains_load: unknown arrays in %s", path);
    std::vector<std::vector<unsigned char>> host(kNChainArrays);
    for (int k = 0; k < kNChainArrays; ++k) {
        if (!(h.mask >> k & 1u))
            continue;
        host[k].resize((size_t)h.n_chains * kChainArrays[k].elem * kChainArrays[k].width);
        if (fread(host[k].data(), 1, host[k].size(), in.f) != host[k].size())
            return fail(RD_EIO, "rd_chains_load: %s ends inside array %s", path,
                        kChainArrays[k].name);
    }
    if (fgetc(in.f) != EOF)
        return fail(RD_EINVAL, "rd_chains_load: %s has bytes after its last array", path);
    for (int k = 0; k < kNChainArrays; ++k)
        if (chain_array(c, k) && k != 3 && !(h.mask >> k & 1u))
            return fail(RD_EINVAL, "rd_chains_load: the state has %s, the file does not",
                        kChainArrays[k].name);
    const hipStream_t s = (hipStream_t)stream;
    if (c->grid_id && (h.mask >> 3 & 1u) && c->n_chains > 0) {
        // grid classes are an input of the caller: check, never overwrite
        std::vector<unsigned char> g(host[3].size());
        HIP_TRY(hipMemcpyAsync(g.data(), c->grid_id, g.size(), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (memcmp(g.data(), host[3].data(), g.size()) != 0)
            return fail(RD_EINVAL, "rd_chains_load: the chains' grid_id differs from the file's");
    }
    for (int k = 0; k < kNChainArrays; ++k) {
        void *d = const_cast<void *>(chain_array(c, k));
        if (k == 3 || !d || host[k].empty())
            continue;
        HIP_TRY(hipMemcpyAsync(d, host[k].data(), host[k].size(), hipMemcpyHostToDevice, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    c->seed = h.seed;
    c->step = h.step;
    return RD_OK;
}
