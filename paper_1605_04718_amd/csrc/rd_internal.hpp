// Internal declarations shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rd {

enum : int {
    kStNotConverged = 1,
    kStBreakdown = 2,
    kStNonfinite = 4,
    kStOutOfPrior = 8,
    kStBadGrid = 16,
    kStNotSteady = 32,
    kStGroupTimeout = 64
};

// One grid class as the kernels see it (device memory).
struct GridDev {
    int n;             // cells per side
    int growth;        // 0 stationary, 1 rho = exp(rate t)
    double rate;       // growth rate r
    const void *u0;    // initial u in the problem precision: FP64 [n*n]; FP32
                       // [2][n*n], rounded value then the rounding remainder
    const void *v0;    // initial v, same layout
    const double *y;   // [n*n] data (float64) or null
    double inv_2s2;    // 1 / (2 sigma^2)
    double cost;       // relative cost of one solve (for queue ordering)
    double dil;        // 2 r (set on the device by k_grid_coeffs)
    double decay;      // exp(-2 r dt) (set on the device by k_grid_coeffs)
};

// Arguments of one fused solve launch.
struct SolveArgs {
    const GridDev *grids;    // device array [n_grids]
    int n_grids;
    int n_items;             // queue length
    const int *order;        // item -> index into the batch (null: identity)
    const int *grid_id;      // batch index -> grid class (null: 0)
    const double *theta;     // [n][4] natural parameters (a, b, gamma, d)
    const int *need;         // [n] nonzero: solve this index (null: all)
    double dt;
    int n_steps;
    double rtol2;            // cg_rtol^2
    int maxit;
    double *phi;             // [n] misfit out (null: skip misfit)
    int *status;             // [n] status out (required)
    int *iters;              // [n][2] CG iteration totals (null: skip)
    void *u_out;             // [n][out_stride] final u, first N*N values of a row
                             // (null: skip)
    void *v_out;             // same layout, final v
    size_t out_stride;       // values per item in u_out / v_out
    unsigned *queue;         // work-queue head (zeroed before the launch)
    void *gws;               // per-workgroup workspace slots (predictor history,
                             // streamed strip arrays)
    size_t gws_stride;       // bytes per slot
    int gws_slots;           // number of slots
    void *coop;              // cooperative-solve workspace (per group: partial sums
                             // and edge rows), or null
    int coop_groups;         // groups the workspace holds
    double steady_tt;        // steady-state stopping: threshold x dt (0: fixed horizon)
    int *steps_out;          // [n] IMEX steps taken (null: skip)
    int coop_wgs;            // class-ordered batch: nonzero when a cooperative
                             // launch serves the 256^2 items (the mixed launch
                             // then skips them)
    unsigned long long coop_wait_ticks;   // bound of a group wait (100 MHz ticks)
    unsigned long long coop_stall_ticks;  // test hook: member 1 of every group
                                          // sleeps this long first (0: off)
    unsigned *coop_timeouts;  // count of members whose group wait gave up (or null)
};

// Cooperative solve of one large grid by a group of workgroups.
constexpr int kCoopN = 256;       // grid size served this way
constexpr int kCoopG = 4;         // workgroups per item (horizontal strips of 64 rows)
constexpr int kCoopThreads = 1024;
__host__ __device__ size_t coop_workspace_bytes(int groups);
hipError_t launch_solve_coop(const SolveArgs &a, int grid_wgs, hipStream_t s);
hipError_t launch_solve_mixed_coop(const SolveArgs &a, int grid_wgs, hipStream_t s);
int mixed_coop_wgs_per_cu();

// Class ranks of a mixed batch (queue order: rank 0 first).
constexpr int kMaxClasses = 8;
struct RankTable {
    int r[kMaxClasses];
};

// Solver tile choices: cells per thread (rows of the strip a thread owns).
struct TileChoice {
    int cpt;      // cells per thread
    int threads;  // workgroup size = n*n / cpt
};

// Host launchers (rd_solver.hip).
hipError_t launch_solve(int n, int precision, TileChoice tile, const SolveArgs &a, int grid_wgs,
                        hipStream_t s);
hipError_t launch_solve_mixed(int precision, int threads, const SolveArgs &a, int grid_wgs,
                              hipStream_t s);
hipError_t launch_class_order(const int *grid_id, int n, int n_grids, const RankTable &rank,
                              int *order, hipStream_t s);
// Largest-first queue order of a single-class launch from per-item cost
// estimates (cost [n], negative = unknown); need may be null.
// n <= kMaxCostOrder.  launch_note_cost updates the estimates of the solved
// items from a solve's CG iterations (iters [n][2]).
constexpr int kMaxCostOrder = 8192;
hipError_t launch_cost_order(int n, const int *need, const int *cost, int *order, hipStream_t s);
hipError_t launch_note_cost(int n, const int *need, const int *iters, int *cost, hipStream_t s);
bool mixed_supported(int n, int precision, int threads);
bool tile_coop(int n, int precision, int cpt);  // a group of workgroups per item
size_t mixed_slot_bytes(int n, int precision, int threads);
int mixed_wgs_per_cu(int precision, int threads);
bool tile_supported(int n, int precision, int cpt);
bool tile_streamed(int n, int precision, int cpt);
int solve_wgs_per_cu(int n, int precision, int cpt);
int default_cpt(int n, int precision);
size_t solve_slot_bytes(int n, int precision, int cpt);
hipError_t launch_fill_u32(unsigned *p, unsigned v, int count, hipStream_t s);
hipError_t launch_grid_coeffs(GridDev *grids, int n_grids, double dt, hipStream_t s);

// Misfit of given fields (rd_sampler.hip).
hipError_t launch_field_misfit(int precision, const GridDev *grids, const int *grid_id, int n,
                               int npts, const void *u, double *phi, hipStream_t s);

}  // namespace rd
