// Fused forward solve + misfit for batches of Schnakenberg parameter vectors.
//
// One workgroup integrates one parameter vector (one "item") through all
// IMEX steps of Sec. 3.1.1 and then forms the Gaussian misfit of eq. (logl);
// workgroups pull items from an atomic queue (persistent launch), so a batch
// of any length and of mixed cost runs in one launch.
//
// Thread layout: thread t owns a vertical strip of R cells of column
// i = t % N, rows j0 .. j0+R-1 with j0 = (t / N) * R.  A wave covers 64
// consecutive columns of one strip row, so every LDS/global row access is
// contiguous across lanes.
//
// Resident variant (N <= 128): the strip arrays (u, v, the two reaction
// diagonals, the CG residual and A p) live in VGPRs; only the CG search
// direction p is shared, through LDS, for the 5-point stencil, and v is
// parked in LDS while the u system is solved.  The whole
// solve touches HBM only to read the initial fields and the data once.
// Streamed variant (large N or FP64 at N = 128): the same algorithm with
// the strip arrays and p in a per-workgroup global-memory slot.
//
// Precision: Real = float keeps the fields and CG vectors in FP32 and every
// dot product, CG scalar and the misfit in FP64; Real = double is FP64
// throughout.
//
// CG (unpreconditioned, as with SciPy's default): per iteration one stencil
// pass (q = A p, partial p.q), one update pass (r -= alpha q, partial r.r)
// and one pass x += alpha p, p = r + beta p, with three workgroup barriers.
// The 5-point stencil is evaluated as sum of (p_c - p_nb) differences so
// that FP32 keeps the small reaction part of A p for smooth p (the
// diffusion diagonal 4c/h^2 dominates by ~10^2 at N = 128).
#include "rd_device.hpp"
#include "rd_internal.hpp"

namespace rd {

template <int N, int R>
struct Geo {
    int i, j0, iw, ie;
    __device__ Geo()
    {
        i = threadIdx.x % N;
        j0 = (threadIdx.x / N) * R;
        iw = i > 0 ? i - 1 : i;      // mirror ghost at x = 0
        ie = i < N - 1 ? i + 1 : i;  // mirror ghost at x = 1
    }
    __device__ int idx(int k) const { return (j0 + k) * N + i; }
};

// Memory-motion fence every kGroup cells of an unrolled strip loop: without
// it the compiler merges and hoists the LDS loads of all R cells ahead of
// their use and the live ranges overflow the VGPR file.  The empty asm with
// a memory clobber stops IR-level motion of memory operations across it and
// the scheduling barrier stops the machine scheduler from sinking the
// arithmetic below it.
constexpr int kGroup = 4;
#define RD_GROUP_FENCE(k)                                   \
    if (((k) % kGroup) == kGroup - 1) {                     \
        asm volatile("" ::: "memory");                      \
        __builtin_amdgcn_sched_barrier(0);                  \
    }

template <typename Real, int R>
struct RegArr {
    Real v[R];
    __device__ __forceinline__ Real &operator[](int k) { return v[k]; }
};

// Strip view of an N*N array in global memory (k-th own cell at base[k*N]).
template <typename Real, int N>
struct GlobArr {
    Real *base;
    __device__ __forceinline__ Real &operator[](int k) const { return base[k * N]; }
};

// For each own cell k: f(k, p_c, t) with t = sum over the four neighbours of
// (p_c - p_nb) = -h^2 Lap_h p at the cell (mirror ghosts give 0 terms).
template <int N, int R, int U, typename Real, typename F>
__device__ __forceinline__ void sweep(const Real *P, const Geo<N, R> &g, F &&f)
{
    Real cur = P[g.j0 * N + g.i];
    Real south = (g.j0 > 0) ? P[(g.j0 - 1) * N + g.i] : cur;
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        const int j = g.j0 + k;
        const Real north = (k + 1 < R || j + 1 < N) ? P[(j + 1) * N + g.i] : cur;
        const Real west = P[j * N + g.iw];
        const Real east = P[j * N + g.ie];
        const Real t = ((cur - west) + (cur - east)) + ((cur - south) + (cur - north));
        f(k, cur, t);
        south = cur;
        cur = north;
        RD_GROUP_FENCE(k)
    }
}

// LDS reduction slots: [0, 2W) setup pair, [2W, 3W) p.q, [3W, 4W) r.r,
// [4W, 5W) misfit.
template <int NW>
struct Slots {
    static constexpr int setup = 0, pq = 2 * NW, rr = 3 * NW, misfit = 4 * NW, total = 5 * NW;
};

// CG for (1/dt + e) x - c' Lap_h x = x_old/dt + src, from x = x_old.
// On entry `es` holds e (reaction + dilution part of the diagonal); on exit
// it holds sigma = 1/dt + e.  r and q are scratch.  Returns RD status bits.
template <int N, int R, int U, int NW, typename Real, class Arr>
__device__ int cg_solve(Arr &x, Arr &es, Arr &r, Arr &q, Real inv_dt, Real c, Real src,
                        double rtol2, int maxit, Real *P, double *red, const Geo<N, R> &g,
                        int &it_acc)
{
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        P[g.idx(k)] = x[k];
        RD_GROUP_FENCE(k)
    }
    __syncthreads();

    // r0 = b - A x0 = src - e x0 - c t(x0): the 1/dt terms cancel exactly,
    // so r0 (the scaled time derivative) keeps full relative precision.
    // Two interleaved FP64 partial sums per dot product halve the dependent
    // accumulation chains.
    double bb0 = 0.0, bb1 = 0.0, rr0 = 0.0, rr1 = 0.0;
    sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
        const Real b = own * inv_dt + src;
        const Real res = src - es[k] * own - c * t;
        r[k] = res;
        es[k] = es[k] + inv_dt;
        if (k & 1) {
            bb1 += (double)b * (double)b;
            rr1 += (double)res * (double)res;
        } else {
            bb0 += (double)b * (double)b;
            rr0 += (double)res * (double)res;
        }
    });
    double bb = bb0 + bb1, rr = rr0 + rr1;
    block_sum2<NW>(bb, rr, red + Slots<NW>::setup);
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        P[g.idx(k)] = r[k];
        RD_GROUP_FENCE(k)
    }

    const double tol2 = rtol2 * bb;
    int st = (finite(bb) && finite(rr)) ? 0 : kStNonfinite;
    int it = 0;
    while (st == 0 && rr > tol2) {
        if (it >= maxit) {
            st = kStNotConverged;
            break;
        }
        __syncthreads();  // p visible to the neighbours
        double pq0 = 0.0, pq1 = 0.0;
        sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
            const Real qq = c * t + es[k] * own;
            q[k] = qq;
            if (k & 1)
                pq1 += (double)own * (double)qq;
            else
                pq0 += (double)own * (double)qq;
        });
        const double pq = block_sum<NW>(pq0 + pq1, red + Slots<NW>::pq);
        if (!finite(pq)) {
            st = kStNonfinite;
            break;
        }
        if (!(pq > 0.0)) {
            st = kStBreakdown;
            break;
        }
        const Real a = uniform((Real)(rr / pq));
        double rn0 = 0.0, rn1 = 0.0;
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            const Real v = r[k] - a * q[k];
            r[k] = v;
            if (k & 1)
                rn1 += (double)v * (double)v;
            else
                rn0 += (double)v * (double)v;
            RD_GROUP_FENCE(k)
        }
        const double rn = block_sum<NW>(rn0 + rn1, red + Slots<NW>::rr);
        ++it;
        if (!finite(rn)) {
            st = kStNonfinite;
            break;
        }
        const Real bt = uniform((Real)(rn / rr));
        // x += alpha p_old and p = r + beta p_old (own cells only; the
        // stencil reads of p finished before the p.q barrier).
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            const Real p = P[g.idx(k)];
            x[k] = x[k] + a * p;
            P[g.idx(k)] = r[k] + bt * p;
            RD_GROUP_FENCE(k)
        }
        rr = rn;
    }
    it_acc += it;
    __syncthreads();
    return st;
}

// All IMEX steps of one item (Sec. 3.1.1):
//   (1/dt + 2 r_n + g (1 - u v)) u' - rho_n^-2 Lap u' = u/dt + g a
//   (1/dt + 2 r_n + g u^2)       v' - d rho_n^-2 Lap v' = v/dt + g b
// `stash` (LDS, N*N, resident variant only; null otherwise) parks v during
// the u solve, where it is not used, so that the u solve keeps only five
// strip arrays in VGPRs.
template <int N, int R, int U, int NW, typename Real, class Arr>
__device__ int integrate(Arr &xu, Arr &xv, Arr &eu, Arr &ev, Arr &r, Arr &q, const double th[4],
                         const GridDev &gd, double dt, int n_steps, double rtol2, int maxit,
                         Real *P, Real *stash, double *red, const Geo<N, R> &g, int &itu,
                         int &itv)
{
    // Per-item and per-step scalars are wave-uniform; keeping them in SGPRs
    // leaves the VGPRs to the strip arrays.
    const Real inv_dt = uniform((Real)(1.0 / dt));
    const Real gam = uniform((Real)th[2]);
    const Real src_u = uniform((Real)(th[2] * th[0]));
    const Real src_v = uniform((Real)(th[2] * th[1]));
    const double n2 = (double)N * (double)N;  // 1/h^2
    // rho_n^-2 = exp(-2 r t_n), t_n = n dt, advanced by the per-class factor
    // exp(-2 r dt) (k_grid_coeffs) each step; relative drift ~n ulp in FP64.
    const double dil = gd.dil;  // m rho'/rho with m = 2
    const double decay = gd.decay;
    double rho_m2 = 1.0;
    int st = 0;
    for (int s = 0; s < n_steps; ++s, rho_m2 = uniform(rho_m2 * decay)) {
        const Real cu = uniform((Real)(rho_m2 * n2));
        const Real cv = uniform((Real)(th[3] * rho_m2 * n2));
        const Real dl = uniform((Real)dil);
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            const Real u = xu[k], v = xv[k];
            eu[k] = dl + gam * (Real(1) - u * v);
            ev[k] = dl + gam * (u * u);
        }
        if (stash) {
#pragma unroll U
            for (int k = 0; k < R; ++k)
                stash[g.idx(k)] = xv[k];
        }
        st = cg_solve<N, R, U, NW>(xu, eu, r, q, inv_dt, cu, src_u, rtol2, maxit, P, red, g, itu);
        if (stash) {
#pragma unroll U
            for (int k = 0; k < R; ++k)
                xv[k] = stash[g.idx(k)];
        }
        if (st)
            break;
        st = cg_solve<N, R, U, NW>(xv, ev, r, q, inv_dt, cv, src_v, rtol2, maxit, P, red, g, itv);
        if (st)
            break;
    }
    return st;
}

template <int N, int R, typename Real, class Arr>
__device__ void finish_item(const SolveArgs &a, const GridDev &gd, int c, Arr &xu, Arr &xv, int st,
                            int itu, int itv, const Geo<N, R> &g, double *red)
{
    constexpr int NW = (N * N / R) / kWave;
    constexpr int U = (R <= 32) ? R : 4;
    const size_t off = (size_t)c * N * N;
    if (a.u_out) {
#pragma unroll U
        for (int k = 0; k < R; ++k)
            ((Real *)a.u_out)[off + g.idx(k)] = xu[k];
    }
    if (a.v_out) {
#pragma unroll U
        for (int k = 0; k < R; ++k)
            ((Real *)a.v_out)[off + g.idx(k)] = xv[k];
    }
    if (a.phi) {
        double s = 0.0;
        if (gd.y) {
#pragma unroll U
            for (int k = 0; k < R; ++k) {
                const double e = gd.y[g.idx(k)] - (double)xu[k];
                s += e * e;
            }
        }
        s = block_sum<NW>(s, red + Slots<NW>::misfit);
        if (threadIdx.x == 0)
            a.phi[c] = (st != 0 || !gd.y || !finite(s)) ? __builtin_inf() : s * gd.inv_2s2;
    }
    if (threadIdx.x == 0) {
        a.status[c] = st;
        if (a.iters) {
            a.iters[2 * c] = itu;
            a.iters[2 * c + 1] = itv;
        }
    }
}

// Pull the next queue item; every thread gets the same (scalar) value.
// The leading barrier keeps thread 0 from overwriting the slot before every
// wave has read the previous item.
__device__ __forceinline__ int next_item(unsigned *queue, int *s_item)
{
    __syncthreads();
    if (threadIdx.x == 0)
        *s_item = (int)atomicAdd(queue, 1u);
    __syncthreads();
    return uniform(*s_item);
}

template <int N, int R, typename Real>
__global__ __launch_bounds__(N *N / R) void k_solve_resident(SolveArgs a)
{
    constexpr int NW = (N * N / R) / kWave;
    __shared__ Real P[N * N];
    __shared__ Real stash[N * N];
    __shared__ double red[Slots<NW>::total];
    __shared__ int s_item;
    const Geo<N, R> g;
    for (int item = next_item(a.queue, &s_item); item < a.n_items;
         item = next_item(a.queue, &s_item)) {
        const int c = uniform(a.order ? a.order[item] : item);
        if (!a.need || uniform(a.need[c])) {
            const GridDev &gd = a.grids[uniform(a.grid_id ? a.grid_id[c] : 0)];
            const double th[4] = {a.theta[4 * c], a.theta[4 * c + 1], a.theta[4 * c + 2],
                                  a.theta[4 * c + 3]};
            RegArr<Real, R> xu, xv, eu, ev, r, q;
            const Real *u0 = (const Real *)gd.u0;
            const Real *v0 = (const Real *)gd.v0;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                xu[k] = u0[g.idx(k)];
                xv[k] = v0[g.idx(k)];
            }
            int itu = 0, itv = 0;
            const int st = integrate<N, R, R, NW>(xu, xv, eu, ev, r, q, th, gd, a.dt, a.n_steps,
                                                  a.rtol2, a.maxit, P, stash, red, g, itu, itv);
            finish_item<N, R, Real>(a, gd, c, xu, xv, st, itu, itv, g, red);
        }
    }
}

// Streamed variant: strip arrays and p in a global slot of 7 N*N arrays.
template <int N, int R, typename Real>
__global__ __launch_bounds__(N *N / R) void k_solve_streamed(SolveArgs a)
{
    constexpr int NW = (N * N / R) / kWave;
    constexpr int U = 4;
    __shared__ double red[Slots<NW>::total];
    __shared__ int s_item;
    const Geo<N, R> g;
    Real *slot = (Real *)a.gws + (size_t)blockIdx.x * 7 * N * N;
    Real *P = slot + 6 * (size_t)N * N;
    const int base = g.j0 * N + g.i;
    GlobArr<Real, N> xu{slot + base}, xv{slot + (size_t)N * N + base},
        eu{slot + 2 * (size_t)N * N + base}, ev{slot + 3 * (size_t)N * N + base},
        r{slot + 4 * (size_t)N * N + base}, q{slot + 5 * (size_t)N * N + base};
    for (int item = next_item(a.queue, &s_item); item < a.n_items;
         item = next_item(a.queue, &s_item)) {
        const int c = uniform(a.order ? a.order[item] : item);
        if (!a.need || uniform(a.need[c])) {
            const GridDev &gd = a.grids[uniform(a.grid_id ? a.grid_id[c] : 0)];
            const double th[4] = {a.theta[4 * c], a.theta[4 * c + 1], a.theta[4 * c + 2],
                                  a.theta[4 * c + 3]};
            const Real *u0 = (const Real *)gd.u0;
            const Real *v0 = (const Real *)gd.v0;
#pragma unroll U
            for (int k = 0; k < R; ++k) {
                xu[k] = u0[g.idx(k)];
                xv[k] = v0[g.idx(k)];
            }
            int itu = 0, itv = 0;
            const int st = integrate<N, R, U, NW>(xu, xv, eu, ev, r, q, th, gd, a.dt, a.n_steps,
                                                  a.rtol2, a.maxit, P, (Real *)nullptr, red, g,
                                                  itu, itv);
            finish_item<N, R, Real>(a, gd, c, xu, xv, st, itu, itv, g, red);
        }
    }
}

// Per-class time-stepping coefficients of the growing domain rho = exp(r t):
// dilution m rho'/rho = 2 r and the per-step factor of rho^-2, exp(-2 r dt).
__global__ void k_grid_coeffs(GridDev *grids, int n_grids, double dt)
{
    const int g = threadIdx.x;
    if (g < n_grids) {
        const double r = grids[g].growth ? grids[g].rate : 0.0;
        grids[g].dil = 2.0 * r;
        grids[g].decay = exp(-2.0 * r * dt);
    }
}

hipError_t launch_grid_coeffs(GridDev *grids, int n_grids, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_grid_coeffs, dim3(1), dim3(64), 0, s, grids, n_grids, dt);
    return hipGetLastError();
}

__global__ void k_fill_u32(unsigned *p, unsigned v, int count)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p[i] = v;
}

hipError_t launch_fill_u32(unsigned *p, unsigned v, int count, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((count + 255) / 256), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Tile table.  Resident tiles exist where the strip arrays (6 x cpt values)
// fit the VGPR budget of the workgroup size.
namespace {

enum Kind { kNone, kResident, kStreamed };

Kind tile_kind(int n, int precision, int cpt)
{
    if (precision == 0) {
        if (n == 32 && (cpt == 4 || cpt == 8 || cpt == 16))
            return kResident;
        if (n == 64 && (cpt == 4 || cpt == 8 || cpt == 16))
            return kResident;
        if (n == 128 && (cpt == 16 || cpt == 32))
            return kResident;
        if (n == 256 && (cpt == 64 || cpt == 128))
            return kStreamed;
    } else {
        if (n == 32 && (cpt == 4 || cpt == 8 || cpt == 16))
            return kResident;
        if (n == 64 && (cpt == 8 || cpt == 16))
            return kResident;
        if (n == 128 && cpt == 32)
            return kStreamed;
        if (n == 256 && cpt == 128)
            return kStreamed;
    }
    return kNone;
}

template <int N, int R, typename Real>
hipError_t go_resident(const SolveArgs &a, int wgs, hipStream_t s)
{
    hipLaunchKernelGGL((k_solve_resident<N, R, Real>), dim3(wgs), dim3(N * N / R), 0, s, a);
    return hipGetLastError();
}

template <int N, int R, typename Real>
hipError_t go_streamed(const SolveArgs &a, int wgs, hipStream_t s)
{
    if (wgs > a.gws_slots)
        wgs = a.gws_slots;
    hipLaunchKernelGGL((k_solve_streamed<N, R, Real>), dim3(wgs), dim3(N * N / R), 0, s, a);
    return hipGetLastError();
}

}  // namespace

bool tile_supported(int n, int precision, int cpt)
{
    return tile_kind(n, precision, cpt) != kNone;
}

// Defaults measured by rd_autotune on MI355X (40-step trial solves): in FP32
// 16 cells per thread wins at every resident size (64, 256 and 1024-thread
// workgroups at 32^2, 64^2 and 128^2).
int default_cpt(int n, int precision)
{
    if (precision == 0)
        return n == 32 ? 16 : n == 64 ? 16 : n == 128 ? 16 : n == 256 ? 128 : 0;
    return n == 32 ? 8 : n == 64 ? 16 : n == 128 ? 32 : n == 256 ? 128 : 0;
}

size_t streamed_slot_bytes(int n, int precision)
{
    return (size_t)7 * n * n * (precision ? sizeof(double) : sizeof(float));
}

template <typename K>
static int occupancy(K kernel, int threads)
{
    int blocks = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, kernel, threads, 0) != hipSuccess)
        return 1;
    return blocks > 0 ? blocks : 1;
}

int solve_wgs_per_cu(int n, int precision, int cpt)
{
#define RD_OCC_R(NN, RR, T)                                                     \
    if (n == NN && cpt == RR)                                                   \
        return occupancy(k_solve_resident<NN, RR, T>, NN * NN / RR);
#define RD_OCC_S(NN, RR, T)                                                     \
    if (n == NN && cpt == RR)                                                   \
        return occupancy(k_solve_streamed<NN, RR, T>, NN * NN / RR);
    if (precision == 0) {
        RD_OCC_R(32, 4, float) RD_OCC_R(32, 8, float) RD_OCC_R(32, 16, float)
        RD_OCC_R(64, 4, float) RD_OCC_R(64, 8, float) RD_OCC_R(64, 16, float)
        RD_OCC_R(128, 16, float) RD_OCC_R(128, 32, float)
        RD_OCC_S(256, 64, float) RD_OCC_S(256, 128, float)
    } else {
        RD_OCC_R(32, 4, double) RD_OCC_R(32, 8, double) RD_OCC_R(32, 16, double)
        RD_OCC_R(64, 8, double) RD_OCC_R(64, 16, double)
        RD_OCC_S(128, 32, double)
        RD_OCC_S(256, 128, double)
    }
#undef RD_OCC_R
#undef RD_OCC_S
    return 1;
}

bool tile_streamed(int n, int precision, int cpt)
{
    return tile_kind(n, precision, cpt) == kStreamed;
}

hipError_t launch_solve(int n, int precision, TileChoice tile, const SolveArgs &a, int wgs,
                        hipStream_t s)
{
    const int cpt = tile.cpt;
#define RD_RES(NN, RR, T)                                     \
    if (n == NN && cpt == RR)                                 \
        return go_resident<NN, RR, T>(a, wgs, s);
#define RD_STR(NN, RR, T)                                     \
    if (n == NN && cpt == RR)                                 \
        return go_streamed<NN, RR, T>(a, wgs, s);
    if (precision == 0) {
        RD_RES(32, 4, float) RD_RES(32, 8, float) RD_RES(32, 16, float)
        RD_RES(64, 4, float) RD_RES(64, 8, float) RD_RES(64, 16, float)
        RD_RES(128, 16, float) RD_RES(128, 32, float)
        RD_STR(256, 64, float) RD_STR(256, 128, float)
    } else {
        RD_RES(32, 4, double) RD_RES(32, 8, double) RD_RES(32, 16, double)
        RD_RES(64, 8, double) RD_RES(64, 16, double)
        RD_STR(128, 32, double)
        RD_STR(256, 128, double)
    }
#undef RD_RES
#undef RD_STR
    return hipErrorInvalidValue;
}

}  // namespace rd
