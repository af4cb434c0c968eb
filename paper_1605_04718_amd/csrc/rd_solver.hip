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
    // Own-cell offset for global-memory accesses, made opaque at each use:
    // otherwise the compiler hoists the R per-cell 64-bit addresses of every
    // global array out of the time loop and keeps them all live.
    __device__ __forceinline__ int off() const
    {
        int o = j0 * N + i;
        asm volatile("" : "+v"(o));
        return o;
    }
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

// Pins a value in a register at this point of the program: the empty
// volatile asm keeps its order with the group fences, so the arithmetic that
// produces the value cannot sink below the next fence.  Without it the
// compiler hoists the LDS reads of a whole strip above the arithmetic of the
// first cells and keeps them all live.
#define RD_PIN(x) asm volatile("" : "+v"(x))

template <typename Real, int R>
struct RegArr {
    Real v[R];
    __device__ __forceinline__ Real &operator[](int k) { return v[k]; }
    __device__ __forceinline__ Real operator[](int k) const { return v[k]; }
};

// Strip view of an N*N array in LDS (k-th own cell at base[k*N]).
template <typename Real, int N>
struct LdsArr {
    Real *base;
    __device__ __forceinline__ Real &operator[](int k) const { return base[k * N]; }
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

// P <- own cells of a global array (src = own-cell pointer, cell k at
// src[k N]).  kLds: P is in LDS (resident variant).  When the 64 lanes of a wave own 64 consecutive words of every
// strip row (N >= 64) the copy uses direct global->LDS loads, which need no
// VGPRs and keep all R loads in flight at once; otherwise it goes through
// registers.  The caller places a barrier before the stencil reads P.
template <int N, int R, int U, bool kLds, typename Real>
__device__ __forceinline__ void copy_to_lds(const Real *src, Real *P, const Geo<N, R> &g)
{
    if constexpr (kLds && N >= kWave && sizeof(Real) == 4) {
        const int row0 = uniform(g.j0 * N + (g.i & ~(kWave - 1)));
#pragma unroll
        for (int k = 0; k < R; ++k)
            __builtin_amdgcn_global_load_lds(src + k * N, P + row0 + k * N, 4, 0, 0);
        __builtin_amdgcn_s_waitcnt(0);  // the LDS writes have landed
    } else {
#pragma unroll U
        for (int k = 0; k < R; ++k)
            P[g.idx(k)] = src[k * N];
    }
}

// LDS reduction slots: [0, 4W) set-up, [4W, 5W) p.q, [5W, 6W) r.r,
// [6W, 7W) misfit.
template <int NW>
struct Slots {
    static constexpr int setup = 0, pq = 4 * NW, rr = 5 * NW, misfit = 6 * NW, total = 7 * NW;
};

// In FP32 a field is carried as an unevaluated sum hi + lo (|lo| <= ulp(hi)/2):
// the residual of an FP32-rounded field alone has a floor of about
// 2^-24 (1/dt + 8 c' n^2) |x| from the rounding noise, which for the stiff
// v system lies far above any useful CG tolerance, and CG would spend its
// iterations on that noise.  With the low part the residual is exact to
// FP32 rounding of its own terms, CG solves for the increment of the step
// (a small quantity, well represented in FP32), and the increment is folded
// back into hi + lo without loss.
template <typename Real>
struct Compensated {
    static constexpr bool on = sizeof(Real) == 4;
};

// Error-free sum (Knuth's TwoSum): s + e == a + b exactly.
__device__ __forceinline__ void two_sum(float a, float b, float &s, float &e)
{
    s = a + b;
    const float bv = s - a;
    e = (a - (s - bv)) + (b - bv);
}

// CG for the increment d of one implicit step of species kSp (0: u, 1: v),
//   (1/dt + e) x' - c' Lap_h x' = x/dt + src,  x' = x + d,
// where x = hi (+ lo in FP32, global memory, this item's slot), and e, the
// reaction + dilution part of the diagonal, is formed at each use from the
// level-n fields: e_u = 2r + g (1 - u v), e_v = 2r + g u^2, with S the other
// species' field (v^n for u, u^n for v).  Not storing the diagonal keeps
// one strip array fewer in VGPRs.  hi is not changed (the caller folds d
// in).  r and q are scratch.  Returns RD status bits.
//
// H (global, the previous step's increment, or null): with `pred`, CG starts
// from one minimal-residual step along it, d0 = w H with
// w = (r0, A H) / (A H, A H), which can only lower the residual.  When the
// trajectory is smooth in time this removes the part of r0 that the last
// step predicts.  The system and the stopping test are unchanged:
// |r| <= rtol |b| on the recursively updated residual.
template <int N, int R, int U, int NW, bool kLds, int kSp, typename Real, class Arr, class SArr>
__device__ int cg_solve(const Arr &hi, const SArr &S, Arr &r, Arr &q, Arr &d, Real inv_dt, Real c,
                        Real src, Real dl, Real gam, double rtol2, int maxit, Real *P,
                        const Real *lo, const Real *H, bool pred, double *red, const Geo<N, R> &g,
                        int &it_acc)
{
    constexpr bool comp = Compensated<Real>::on;
    // e(k) and sigma(k) = 1/dt + e(k)
    const Real e0 = uniform(kSp == 0 ? dl + gam : dl);
    const Real s0 = uniform(e0 + inv_dt);
    auto e_at = [&](int k) -> Real {
        if constexpr (kSp == 0)
            return e0 - gam * (hi[k] * S[k]);
        else
            return e0 + gam * (S[k] * S[k]);
    };
    auto sigma_at = [&](int k) -> Real {
        if constexpr (kSp == 0)
            return s0 - gam * (hi[k] * S[k]);
        else
            return s0 + gam * (S[k] * S[k]);
    };
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        P[g.idx(k)] = hi[k];
        RD_GROUP_FENCE(k)
    }
    __syncthreads();

    // r0 = b - A x = src - e x - c t(x): the 1/dt terms cancel exactly, so
    // r0 (the scaled time derivative) keeps full relative precision.
    double bb = 0.0, rr = 0.0;
    sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
        const Real b = own * inv_dt + src;
        Real res = src - e_at(k) * own - c * t;
        RD_PIN(res);
        r[k] = res;
        bb += (double)b * (double)b;
        RD_PIN(bb);
        if constexpr (!comp) {
            rr += (double)res * (double)res;
            RD_PIN(rr);
        }
    });
    if constexpr (comp) {
        // the low part's share of A x
        __syncthreads();
        copy_to_lds<N, R, U, kLds>(lo + g.off(), P, g);
        __syncthreads();
        sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
            Real res = r[k] - (e_at(k) * own + c * t);
            RD_PIN(res);
            r[k] = res;
            rr += (double)res * (double)res;
            RD_PIN(rr);
        });
    }
    bool rr_pending = false;
    if (H && pred) {
        __syncthreads();  // every stencil read of P is done
        copy_to_lds<N, R, U, kLds>(H + g.off(), P, g);
        __syncthreads();
        double rw = 0.0, ww = 0.0;
        sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
            Real w = c * t + sigma_at(k) * own;  // (A H) at the cell
            RD_PIN(w);
            q[k] = w;
            rw += (double)r[k] * (double)w;
            ww += (double)w * (double)w;
            RD_PIN(rw);
            RD_PIN(ww);
        });
        double v4[4] = {bb, rr, rw, ww};
        block_sum_n<NW>(v4, red + Slots<NW>::setup);
        bb = v4[0];
        rr = v4[1];
        rw = v4[2];
        ww = v4[3];
        const Real w = uniform((Real)((ww > 0.0 && finite(rw)) ? rw / ww : 0.0));
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            d[k] = w * P[g.idx(k)];
            r[k] = r[k] - w * q[k];
            RD_GROUP_FENCE(k)
        }
        // |r0 - w A H|^2 is not formed by expanding the square: when the
        // predictor is good the expansion cancels to rounding noise and could
        // end the solve before it converges.  It is summed from the updated r
        // in the first CG sweep instead (rr_pending).
        rr_pending = true;
    } else {
        block_sum2<NW>(bb, rr, red + Slots<NW>::setup);
#pragma unroll U
        for (int k = 0; k < R; ++k)
            d[k] = Real(0);
    }
    // The reduction barrier above also ends every stencil read of P, and each
    // thread now only rewrites its own cells.
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        P[g.idx(k)] = r[k];
        RD_GROUP_FENCE(k)
    }

    const double tol2 = rtol2 * bb;
    int st = (finite(bb) && finite(rr)) ? 0 : kStNonfinite;
    int it = 0;
    while (st == 0 && (rr_pending || rr > tol2)) {
        if (it >= maxit) {
            st = kStNotConverged;
            break;
        }
        __syncthreads();  // p visible to the neighbours
        // Two interleaved FP64 partial sums per dot product halve the
        // dependent accumulation chains.  With rr_pending, p = r here and
        // the same sweep sums r.r.
        double pq0 = 0.0, pq1 = 0.0, rp = 0.0;
        sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
            Real qq = c * t + sigma_at(k) * own;
            RD_PIN(qq);
            q[k] = qq;
            if (k & 1) {
                pq1 += (double)own * (double)qq;
                RD_PIN(pq1);
            } else {
                pq0 += (double)own * (double)qq;
                RD_PIN(pq0);
            }
            if (rr_pending) {
                rp += (double)own * (double)own;
                RD_PIN(rp);
            }
        });
        double pq;
        if (rr_pending) {
            double v2[2] = {pq0 + pq1, rp};
            block_sum_n<NW>(v2, red + Slots<NW>::setup);
            pq = v2[0];
            rr = v2[1];
            rr_pending = false;
            if (!finite(rr)) {
                st = kStNonfinite;
                break;
            }
            if (!(rr > tol2))
                break;  // the predictor alone met the tolerance
        } else {
            pq = block_sum<NW>(pq0 + pq1, red + Slots<NW>::pq);
        }
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
        // d += alpha p_old and p = r + beta p_old (own cells only; the
        // stencil reads of p finished before the p.q barrier).
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            const Real p = P[g.idx(k)];
            d[k] = d[k] + a * p;
            P[g.idx(k)] = r[k] + bt * p;
            RD_GROUP_FENCE(k)
        }
        rr = rn;
    }
    it_acc += it;
    __syncthreads();
    return st;
}

// x' = x + d: hi (+ lo) absorb the increment.  kDGlobal: d is read from the
// global array H (own-cell layout); otherwise d is in registers and is also
// recorded in H (when non-null) for the next step's predictor.  The global
// loads are all issued before the first use: on this architecture stores
// count in the same counter as loads, so a load placed after the previous
// cell's store would wait for that store as well, one round trip per cell.
template <int N, int R, int U, bool kDGlobal, typename Real, class Arr>
__device__ __forceinline__ void fold(Arr &hi, Arr &d, Real *lo, Real *H, const Geo<N, R> &g)
{
    constexpr bool comp = Compensated<Real>::on;
    const int o = g.off();
    if constexpr (R * sizeof(Real) > 32 * sizeof(float)) {
        // long strips (streamed variant): one pass, the loads overlap with
        // the other workgroups' work instead
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            const Real dk = kDGlobal ? H[o + k * N] : d[k];
            if constexpr (comp) {
                float s, e;
                two_sum(hi[k], dk, s, e);
                const float lk = lo[o + k * N] + e;
                const float nh = s + lk;
                hi[k] = nh;
                lo[o + k * N] = lk - (nh - s);
            } else {
                hi[k] = hi[k] + dk;
            }
            if (!kDGlobal && H)
                H[o + k * N] = dk;
        }
        return;
    }
    Real l[R], dd[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if constexpr (comp)
            l[k] = lo[o + k * N];
        dd[k] = kDGlobal ? H[o + k * N] : d[k];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if constexpr (comp)
            RD_PIN(l[k]);
        RD_PIN(dd[k]);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        if constexpr (comp) {
            float s, e;
            two_sum(hi[k], dd[k], s, e);
            const float lk = l[k] + e;
            const float nh = s + lk;
            hi[k] = nh;
            lo[o + k * N] = lk - (nh - s);
        } else {
            hi[k] = hi[k] + dd[k];
        }
        if (!kDGlobal && H)
            H[o + k * N] = dd[k];
    }
}

// d -> H (own cells).
template <int N, int R, int U, typename Real, class Arr>
__device__ __forceinline__ void store_increment(Arr &d, Real *H, const Geo<N, R> &g)
{
    const int o = g.off();
#pragma unroll U
    for (int k = 0; k < R; ++k)
        H[o + k * N] = d[k];
}

// Per-workgroup global slot of the solve: the low parts of u and v (FP32),
// the last increments of u and v (predictor), then (streamed variant only)
// the strip arrays and p.
template <typename Real>
struct SlotLayout {
    static constexpr int lo_u = 0, lo_v = 1, h_u = 2, h_v = 3, arrays = 4;
};

// All IMEX steps of one item (Sec. 3.1.1):
//   (1/dt + 2 r_n + g (1 - u v)) u' - rho_n^-2 Lap u' = u/dt + g a
//   (1/dt + 2 r_n + g u^2)       v' - d rho_n^-2 Lap v' = v/dt + g b
// Both systems use the fields of level n only, so they are solved one after
// the other with one set of CG work arrays (r, q, d); u is advanced only
// after the v solve, which needs u^n.  Resident variant (kLds): P and
// `stash` are in LDS and the stash parks the field not being solved for
// (v^n during the u solve, u^n during the v solve), so that a solve keeps
// four strip arrays in VGPRs.  Streamed variant: all arrays are global and
// `stash` is null.  `slot` is the item's global slot (SlotLayout).
template <int N, int R, int U, int NW, bool kLds, typename Real, class Arr>
__device__ int integrate(Arr &xu, Arr &xv, Arr &r, Arr &q, Arr &d, const double th[4],
                         const GridDev &gd, double dt, int n_steps, double rtol2, int maxit,
                         Real *P, Real *stash, Real *slot, double *red, const Geo<N, R> &g,
                         int &itu, int &itv)
{
    using L = SlotLayout<Real>;
    constexpr bool comp = Compensated<Real>::on;
    Real *const lo_u = comp ? slot + L::lo_u * N * N : nullptr;
    Real *const lo_v = comp ? slot + L::lo_v * N * N : nullptr;
    Real *const h_u = slot + L::h_u * N * N;
    Real *const h_v = slot + L::h_v * N * N;
    // Per-item and per-step scalars are wave-uniform; keeping them in SGPRs
    // leaves the VGPRs to the strip arrays.
    const Real inv_dt = uniform((Real)(1.0 / dt));
    const Real gam = uniform((Real)th[2]);
    const Real src_u = uniform((Real)(th[2] * th[0]));
    const Real src_v = uniform((Real)(th[2] * th[1]));
    const Real dl = uniform((Real)gd.dil);  // m rho'/rho with m = 2
    const double n2 = (double)N * (double)N;  // 1/h^2
    // rho_n^-2 = exp(-2 r t_n), t_n = n dt, advanced by the per-class factor
    // exp(-2 r dt) (k_grid_coeffs) each step; relative drift ~n ulp in FP64.
    const double decay = gd.decay;
    double rho_m2 = 1.0;
    int st = 0;
    // The predictor pays off only while the field moves: a species whose
    // last solve needed no CG iteration skips it (its residual was already
    // below the tolerance without it).
    int last_u = 0, last_v = 0;
    for (int s = 0; s < n_steps; ++s, rho_m2 = uniform(rho_m2 * decay)) {
        const Real cu = uniform((Real)(rho_m2 * n2));
        const Real cv = uniform((Real)(th[3] * rho_m2 * n2));
        const bool pred_u = s > 0 && last_u > 0;
        const bool pred_v = s > 0 && last_v > 0;
        const int itu0 = itu, itv0 = itv;
        if constexpr (kLds) {
            LdsArr<Real, N> sv{stash + g.idx(0)};
#pragma unroll U
            for (int k = 0; k < R; ++k)
                sv[k] = xv[k];
            st = cg_solve<N, R, U, NW, kLds, 0>(xu, sv, r, q, d, inv_dt, cu, src_u, dl, gam, rtol2,
                                                maxit, P, lo_u, h_u, pred_u, red, g, itu);
#pragma unroll U
            for (int k = 0; k < R; ++k) {
                xv[k] = sv[k];
                if (!st)
                    sv[k] = xu[k];
            }
            if (st)
                break;
            store_increment<N, R, U>(d, h_u, g);
            st = cg_solve<N, R, U, NW, kLds, 1>(xv, sv, r, q, d, inv_dt, cv, src_v, dl, gam, rtol2,
                                                maxit, P, lo_v, h_v, pred_v, red, g, itv);
#pragma unroll U
            for (int k = 0; k < R; ++k)
                xu[k] = sv[k];
        } else {
            st = cg_solve<N, R, U, NW, kLds, 0>(xu, xv, r, q, d, inv_dt, cu, src_u, dl, gam, rtol2,
                                                maxit, P, lo_u, h_u, pred_u, red, g, itu);
            if (st)
                break;
            store_increment<N, R, U>(d, h_u, g);
            st = cg_solve<N, R, U, NW, kLds, 1>(xv, xu, r, q, d, inv_dt, cv, src_v, dl, gam, rtol2,
                                                maxit, P, lo_v, h_v, pred_v, red, g, itv);
        }
        if (st)
            break;
        fold<N, R, U, false>(xv, d, lo_v, h_v, g);
        fold<N, R, U, true>(xu, d, lo_u, h_u, g);
        last_u = uniform(itu - itu0);
        last_v = uniform(itv - itv0);
    }
    return st;
}

// Item start: hi in registers (or the streamed arrays), lo in the slot.
template <int N, int R, int U, typename Real, class Arr>
__device__ __forceinline__ void load_initial(const GridDev &gd, Arr &xu, Arr &xv, Real *slot,
                                             const Geo<N, R> &g)
{
    using L = SlotLayout<Real>;
    const int o = g.off();
    const Real *u0 = (const Real *)gd.u0 + o;
    const Real *v0 = (const Real *)gd.v0 + o;
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        xu[k] = u0[k * N];
        xv[k] = v0[k * N];
        if constexpr (Compensated<Real>::on) {
            // the FP32 initial fields are stored as [hi | lo]
            slot[L::lo_u * N * N + o + k * N] = u0[N * N + k * N];
            slot[L::lo_v * N * N + o + k * N] = v0[N * N + k * N];
        }
    }
}

template <int N, int R, typename Real, class Arr>
__device__ void finish_item(const SolveArgs &a, const GridDev &gd, int c, Arr &xu, Arr &xv, int st,
                            int itu, int itv, const Real *slot, const Geo<N, R> &g, double *red)
{
    using L = SlotLayout<Real>;
    constexpr int NW = (N * N / R) / kWave;
    constexpr int U = (R <= 32) ? R : 4;
    const size_t off = (size_t)c * a.out_stride;
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
            const int o = g.off();
#pragma unroll U
            for (int k = 0; k < R; ++k) {
                double u = (double)xu[k];
                if constexpr (Compensated<Real>::on)
                    u += (double)slot[L::lo_u * N * N + o + k * N];
                const double e = gd.y[o + k * N] - u;
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

// Grid class of batch index c, or -1 (and the item is marked failed) when
// grid_id is outside [0, n_grids).
__device__ __forceinline__ int item_grid(const SolveArgs &a, int c)
{
    const int gid = uniform(a.grid_id ? a.grid_id[c] : 0);
    if ((unsigned)gid < (unsigned)a.n_grids)
        return gid;
    if (threadIdx.x == 0) {
        a.status[c] = kStBadGrid;
        if (a.phi)
            a.phi[c] = __builtin_inf();
    }
    return -1;
}

// One item, resident variant: P and stash are LDS arrays of at least N*N.
template <int N, int R, typename Real>
__device__ __forceinline__ void solve_item_resident(const SolveArgs &a, int c, const GridDev &gd,
                                                    Real *P, Real *stash, double *red, Real *slot)
{
    constexpr int NW = (N * N / R) / kWave;
    const Geo<N, R> g;
    const double th[4] = {a.theta[4 * c], a.theta[4 * c + 1], a.theta[4 * c + 2],
                          a.theta[4 * c + 3]};
    RegArr<Real, R> xu, xv, r, q, d;
    load_initial<N, R, R>(gd, xu, xv, slot, g);
    int itu = 0, itv = 0;
    const int st = integrate<N, R, R, NW, true>(xu, xv, r, q, d, th, gd, a.dt, a.n_steps, a.rtol2,
                                                a.maxit, P, stash, slot, red, g, itu, itv);
    finish_item<N, R, Real>(a, gd, c, xu, xv, st, itu, itv, slot, g, red);
}

// One item, streamed variant: the strip arrays and p follow the SlotLayout
// arrays in the workgroup's global slot.
template <int N, int R, typename Real>
__device__ __forceinline__ void solve_item_streamed(const SolveArgs &a, int c, const GridDev &gd,
                                                    double *red, Real *slot)
{
    constexpr int NW = (N * N / R) / kWave;
    constexpr int U = 4;
    constexpr size_t NN = (size_t)N * N;
    const Geo<N, R> g;
    Real *arr = slot + SlotLayout<Real>::arrays * NN;
    Real *P = arr + 5 * NN;
    const int base = g.j0 * N + g.i;
    GlobArr<Real, N> xu{arr + base}, xv{arr + NN + base}, r{arr + 2 * NN + base},
        q{arr + 3 * NN + base}, d{arr + 4 * NN + base};
    const double th[4] = {a.theta[4 * c], a.theta[4 * c + 1], a.theta[4 * c + 2],
                          a.theta[4 * c + 3]};
    load_initial<N, R, U>(gd, xu, xv, slot, g);
    int itu = 0, itv = 0;
    const int st = integrate<N, R, U, NW, false>(xu, xv, r, q, d, th, gd, a.dt, a.n_steps, a.rtol2,
                                                 a.maxit, P, (Real *)nullptr, slot, red, g, itu,
                                                 itv);
    finish_item<N, R, Real>(a, gd, c, xu, xv, st, itu, itv, slot, g, red);
}

template <int N, int R, typename Real>
__global__ __launch_bounds__(N *N / R) void k_solve_resident(SolveArgs a)
{
    constexpr int NW = (N * N / R) / kWave;
    __shared__ Real P[N * N];
    __shared__ Real stash[N * N];
    __shared__ double red[Slots<NW>::total];
    __shared__ int s_item;
    Real *slot = (Real *)((char *)a.gws + (size_t)blockIdx.x * a.gws_stride);
    for (int item = next_item(a.queue, &s_item); item < a.n_items;
         item = next_item(a.queue, &s_item)) {
        const int c = uniform(a.order ? a.order[item] : item);
        if (!a.need || uniform(a.need[c])) {
            const int gid = item_grid(a, c);
            if (gid >= 0)
                solve_item_resident<N, R, Real>(a, c, a.grids[gid], P, stash, red, slot);
        }
    }
}

template <int N, int R, typename Real>
__global__ __launch_bounds__(N *N / R) void k_solve_streamed(SolveArgs a)
{
    constexpr int NW = (N * N / R) / kWave;
    __shared__ double red[Slots<NW>::total];
    __shared__ int s_item;
    Real *slot = (Real *)((char *)a.gws + (size_t)blockIdx.x * a.gws_stride);
    for (int item = next_item(a.queue, &s_item); item < a.n_items;
         item = next_item(a.queue, &s_item)) {
        const int c = uniform(a.order ? a.order[item] : item);
        if (!a.need || uniform(a.need[c])) {
            const int gid = item_grid(a, c);
            if (gid >= 0)
                solve_item_streamed<N, R, Real>(a, c, a.grids[gid], red, slot);
        }
    }
}

// Uneven batches: one persistent launch of T-thread workgroups serves items
// of every grid class.  Each class runs the strip layout that T threads give
// it (R = n^2 / T cells per thread): resident where its arrays fit the VGPR
// and LDS budget, streamed otherwise.  The queue is ordered by decreasing
// cost (a.order), so that the large solves start first and the small ones
// fill the tail.
template <typename Real>
struct MixedTraits {
    static constexpr int kMaxResident = sizeof(Real) == 4 ? 128 : 64;
};

template <int N, int T, typename Real>
__device__ __forceinline__ void solve_item_class(const SolveArgs &a, int c, const GridDev &gd,
                                                 Real *P, Real *stash, double *red, Real *slot)
{
    if constexpr (N * N >= T) {
        constexpr int R = N * N / T;
        if constexpr (N <= MixedTraits<Real>::kMaxResident && R <= 32 / (sizeof(Real) / 4))
            solve_item_resident<N, R, Real>(a, c, gd, P, stash, red, slot);
        else
            solve_item_streamed<N, R, Real>(a, c, gd, red, slot);
    }
}

template <int T, typename Real>
__global__ __launch_bounds__(T) void k_solve_mixed(SolveArgs a)
{
    constexpr int NW = T / kWave;
    constexpr int NM = MixedTraits<Real>::kMaxResident;
    __shared__ Real P[NM * NM];
    __shared__ Real stash[NM * NM];
    __shared__ double red[Slots<NW>::total];
    __shared__ int s_item;
    Real *slot = (Real *)((char *)a.gws + (size_t)blockIdx.x * a.gws_stride);
    for (int item = next_item(a.queue, &s_item); item < a.n_items;
         item = next_item(a.queue, &s_item)) {
        const int c = uniform(a.order ? a.order[item] : item);
        const int gid = (!a.need || uniform(a.need[c])) ? item_grid(a, c) : -1;
        if (gid >= 0) {
            const GridDev &gd = a.grids[gid];
            const int n = uniform(gd.n);
            if (n == 32)
                solve_item_class<32, T, Real>(a, c, gd, P, stash, red, slot);
            else if (n == 64)
                solve_item_class<64, T, Real>(a, c, gd, P, stash, red, slot);
            else if (n == 128)
                solve_item_class<128, T, Real>(a, c, gd, P, stash, red, slot);
            else if (n == 256)
                solve_item_class<256, T, Real>(a, c, gd, P, stash, red, slot);
        }
    }
}

// Queue order of a mixed batch: the stable counting sort of the items by
// grid class in the order `rank` (rank[g] = position of class g, most costly
// first).  One workgroup; thread t sorts a contiguous chunk.
__device__ __forceinline__ int class_rank(const RankTable &rank, int gid, int n_grids)
{
    return (unsigned)gid < (unsigned)n_grids ? rank.r[gid] : kMaxClasses - 1;
}

__global__ __launch_bounds__(1024) void k_class_order(const int *grid_id, int n, int n_grids,
                                                      RankTable rank, int *order)
{
    __shared__ int counts[1024][kMaxClasses];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int lo = t * chunk, hi = min(n, lo + chunk);
    int local[kMaxClasses];
    for (int g = 0; g < kMaxClasses; ++g)
        local[g] = 0;
    for (int i = lo; i < hi; ++i)
        local[class_rank(rank, grid_id[i], n_grids)]++;
    for (int g = 0; g < kMaxClasses; ++g)
        counts[t][g] = local[g];
    __syncthreads();
    if (t == 0) {
        int run = 0;
        for (int g = 0; g < kMaxClasses; ++g) {
            for (int u = 0; u < 1024; ++u) {
                const int v = counts[u][g];
                counts[u][g] = run;
                run += v;
            }
        }
    }
    __syncthreads();
    for (int g = 0; g < kMaxClasses; ++g)
        local[g] = counts[t][g];
    for (int i = lo; i < hi; ++i)
        order[local[class_rank(rank, grid_id[i], n_grids)]++] = i;
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

size_t solve_slot_bytes(int n, int precision, int cpt)
{
    const size_t arrays = tile_kind(n, precision, cpt) == kStreamed ? 10 : 4;
    return arrays * n * n * (precision ? sizeof(double) : sizeof(float));
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

// Mixed launch: T threads per workgroup for every class.
static bool mixed_resident(int n, int precision, int threads)
{
    const int r = n * n / threads;
    return n <= (precision ? 64 : 128) && r <= (precision ? 16 : 32);
}

bool mixed_supported(int n, int precision, int threads)
{
    return (threads == 512 || threads == 1024) && (n == 32 || n == 64 || n == 128 || n == 256) &&
           n * n >= threads;
}

size_t mixed_slot_bytes(int n, int precision, int threads)
{
    const size_t arrays = mixed_resident(n, precision, threads) ? 4 : 10;
    return arrays * n * n * (precision ? sizeof(double) : sizeof(float));
}

int mixed_wgs_per_cu(int precision, int threads)
{
    if (precision == 0)
        return threads == 512 ? occupancy(k_solve_mixed<512, float>, 512)
                              : occupancy(k_solve_mixed<1024, float>, 1024);
    return threads == 512 ? occupancy(k_solve_mixed<512, double>, 512)
                          : occupancy(k_solve_mixed<1024, double>, 1024);
}

hipError_t launch_class_order(const int *grid_id, int n, int n_grids, const RankTable &rank,
                              int *order, hipStream_t s)
{
    hipLaunchKernelGGL(k_class_order, dim3(1), dim3(1024), 0, s, grid_id, n, n_grids, rank, order);
    return hipGetLastError();
}

hipError_t launch_solve_mixed(int precision, int threads, const SolveArgs &a, int wgs,
                              hipStream_t s)
{
    if (!a.gws || wgs > a.gws_slots || !a.order)
        return hipErrorInvalidValue;
    if (precision == 0) {
        if (threads == 512)
            hipLaunchKernelGGL((k_solve_mixed<512, float>), dim3(wgs), dim3(512), 0, s, a);
        else
            hipLaunchKernelGGL((k_solve_mixed<1024, float>), dim3(wgs), dim3(1024), 0, s, a);
    } else {
        if (threads == 512)
            hipLaunchKernelGGL((k_solve_mixed<512, double>), dim3(wgs), dim3(512), 0, s, a);
        else
            hipLaunchKernelGGL((k_solve_mixed<1024, double>), dim3(wgs), dim3(1024), 0, s, a);
    }
    return hipGetLastError();
}

bool tile_streamed(int n, int precision, int cpt)
{
    return tile_kind(n, precision, cpt) == kStreamed;
}

hipError_t launch_solve(int n, int precision, TileChoice tile, const SolveArgs &a, int wgs,
                        hipStream_t s)
{
    const int cpt = tile.cpt;
    // Every workgroup owns one workspace slot (predictor history; streamed
    // tiles also keep their strip arrays there).
    if (!a.gws || wgs > a.gws_slots || a.gws_stride < solve_slot_bytes(n, precision, cpt))
        return hipErrorInvalidValue;
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
