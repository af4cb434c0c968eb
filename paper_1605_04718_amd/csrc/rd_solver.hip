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
    int wid;  // this wave's index in the workgroup (scalar)
    __device__ Geo()
    {
        i = threadIdx.x % N;
        j0 = (threadIdx.x / N) * R;
        iw = i > 0 ? i - 1 : i;      // mirror ghost at x = 0
        ie = i < N - 1 ? i + 1 : i;  // mirror ghost at x = 1
        wid = wave_index();
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

// As sweep(), but f(k, p_c, s) gets the plain sum of the four neighbours
// (mirror ghosts give p_c), so that A p = (sigma + 4c) p - c s: three
// additions per cell instead of seven.  For the CG iteration on a step
// increment only: there the rounding of the sum form stays below the other
// FP32 roundings of the iteration (an FP32 emulation of the increment solves
// reaches the same true residual with the same iteration counts), while the
// residual of the field itself keeps the exact difference form.
template <int N, int R, int U, typename Real, typename F>
__device__ __forceinline__ void sweep_nsum(const Real *P, const Geo<N, R> &g, F &&f)
{
    Real cur = P[g.j0 * N + g.i];
    Real south = (g.j0 > 0) ? P[(g.j0 - 1) * N + g.i] : cur;
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        const int j = g.j0 + k;
        const Real north = (k + 1 < R || j + 1 < N) ? P[(j + 1) * N + g.i] : cur;
        const Real west = P[j * N + g.iw];
        const Real east = P[j * N + g.ie];
        const Real sn = (west + east) + (south + north);
        f(k, cur, sn);
        south = cur;
        cur = north;
        RD_GROUP_FENCE(k)
    }
}

// sweep() over two arrays with the same layout at once: f(k, p_c, t(p),
// q_c, t(q)).
template <int N, int R, int U, typename Real, typename F>
__device__ __forceinline__ void sweep_pair(const Real *P, const Real *Q, const Geo<N, R> &g, F &&f)
{
    Real cur = P[g.j0 * N + g.i], qcur = Q[g.j0 * N + g.i];
    Real south = (g.j0 > 0) ? P[(g.j0 - 1) * N + g.i] : cur;
    Real qsouth = (g.j0 > 0) ? Q[(g.j0 - 1) * N + g.i] : qcur;
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        const int j = g.j0 + k;
        const bool in = k + 1 < R || j + 1 < N;
        const Real north = in ? P[(j + 1) * N + g.i] : cur;
        const Real qnorth = in ? Q[(j + 1) * N + g.i] : qcur;
        const Real t = ((cur - P[j * N + g.iw]) + (cur - P[j * N + g.ie])) +
                       ((cur - south) + (cur - north));
        const Real qt = ((qcur - Q[j * N + g.iw]) + (qcur - Q[j * N + g.ie])) +
                        ((qcur - qsouth) + (qcur - qnorth));
        f(k, cur, t, qcur, qt);
        south = cur;
        cur = north;
        qsouth = qcur;
        qcur = qnorth;
        RD_GROUP_FENCE(k)
    }
}

// sweep_pair() with the first array's differences formed and summed in FP64:
// f(k, p_c, t64(p), q_c, t(q)).  The differences of FP32 values are exact
// in FP64, so t64 carries no rounding error to speak of; the residual of a
// compensated field needs it (the FP32 sum of the four differences, scaled
// by c, rounds at about 2^-24 of the diffusion term, which lies above
// rtol |b| for rtol 1e-9).
template <int N, int R, int U, typename F>
__device__ __forceinline__ void sweep_pair64(const float *P, const float *Q, const Geo<N, R> &g,
                                             F &&f)
{
    float cur = P[g.j0 * N + g.i], qcur = Q[g.j0 * N + g.i];
    double cur64 = cur;
    double south64 = (g.j0 > 0) ? (double)P[(g.j0 - 1) * N + g.i] : cur64;
    float qsouth = (g.j0 > 0) ? Q[(g.j0 - 1) * N + g.i] : qcur;
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        const int j = g.j0 + k;
        const bool in = k + 1 < R || j + 1 < N;
        const float north = in ? P[(j + 1) * N + g.i] : cur;
        const float qnorth = in ? Q[(j + 1) * N + g.i] : qcur;
        const double north64 = north;
        const double t64 = ((cur64 - (double)P[j * N + g.iw]) + (cur64 - (double)P[j * N + g.ie])) +
                           ((cur64 - south64) + (cur64 - north64));
        const float qt = ((qcur - Q[j * N + g.iw]) + (qcur - Q[j * N + g.ie])) +
                         ((qcur - qsouth) + (qcur - qnorth));
        f(k, cur, t64, qcur, qt);
        south64 = cur64;
        cur64 = north64;
        cur = north;
        qsouth = qcur;
        qcur = qnorth;
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
// The CG step lengths alpha = rr / pq and beta = rn / rr (FP64 sums) in
// the working precision.  FP32 tiles take them from the hardware reciprocal
// (within 1 ulp) times the numerator, about 1.5 ulp in all: the iteration
// updates r and d with the same value, so the recursion stays consistent,
// and the FP64 division (a chain of about ten dependent operations) sat on
// the path every wave of the workgroup waits on after each reduction.
template <typename Real>
__device__ __forceinline__ Real step_ratio(double num, double den)
{
    if constexpr (sizeof(Real) == 4)
        return uniform((float)num * __builtin_amdgcn_rcpf((float)den));
    else
        return uniform(num / den);
}

// Squared CG tolerance below which the resident FP32 solve evaluates its
// step residual in FP64 (rtol < 3e-8: ten times the FP32 evaluation's
// rounding floor relative to |b|).
constexpr double kRes64Rtol2 = 9e-16;

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
// H1, H2 (global): the increments of the last two steps.  npred = 1: CG
// starts from one minimal-residual step along H1, d0 = w H1 with
// w = (r0, A H1) / (A H1, A H1), which can only lower the residual.
// npred = 2: d0 = w1 H1 + w2 H2 with the Galerkin condition
// (H_i, r0 - A d0) = 0, i.e. the 2 x 2 system (H_i, A H_j) w = (H_i, r0): the
// start vector of least error in the A-norm over span{H1, H2}, which CG's own
// iterates also minimise (a minimal-residual pair cancels smoothness the
// energy norm keeps; measured on the CPU, it saves fewer iterations).  When
// the trajectory is smooth in time the pair extrapolates the increment to
// second order.  npred = 0: d0 = 0.  The system and the stopping test are
// unchanged: |r| <= rtol |b| on the recursively updated residual.  `quiet`
// returns whether r0 itself met the tolerance (the field did not move).
//
// kFuse (resident FP32): on entry the other species' field is still in
// registers (Sreg) and the LDS stash behind S is free.  The residuals of hi
// and of lo are then formed in one pass, lo staged in the stash, and Sreg
// is parked in the stash afterwards (S reads it from there on).
template <int N, int R, int U, int NW, bool kLds, int kSp, bool kFuse = false, bool kPred2 = false,
          typename Real, class Arr, class SArr>
__device__ int cg_solve(const Arr &hi, const SArr &S, Arr &r, Arr &q, Arr &d, Real inv_dt, Real c,
                        Real src, Real dl, Real gam, double rtol2, int maxit, Real *P,
                        const Real *lo, const Real *H1, const Real *H2, int npred, double *red,
                        const Geo<N, R> &g, int &it_acc, int &quiet, const Arr *Sreg = nullptr,
                        Real *stash = nullptr, const Real *Slo = nullptr)
{
    constexpr bool comp = Compensated<Real>::on;
    static_assert(!kFuse || (comp && kLds), "the fused set-up is for resident FP32 solves");
    // the two-increment start reads the histories a group of kGroup cells at
    // the group's first cell and indexes its group buffers with k % kGroup,
    // a constant only when the unroll factor is a multiple of the group (the
    // other grouped loops run only fully unrolled)
    static_assert(!kPred2 || (U % kGroup == 0 && R % kGroup == 0), "unroll by whole groups");
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
    // sigma_at() for a sweep that visits k = 0 .. R-1 in order (the set-up
    // sweeps): with the sweep fully unrolled, S (the LDS stash in FP32
    // tiles) is read a pinned group of cells at a time, at the group's
    // first cell; read at each cell, every read was waited for before the
    // next.
    Real sgrp[kGroup];
    auto sigma_seq = [&](int k) -> Real {
        if constexpr (U == R) {
            if (k % kGroup == 0) {
#pragma unroll
                for (int j = 0; j < kGroup; ++j)
                    sgrp[j] = k + j < R ? S[k + j] : Real(0);
            }
            const Real sk = sgrp[k % kGroup];
            if constexpr (kSp == 0)
                return s0 - gam * (hi[k] * sk);
            else
                return s0 + gam * (sk * sk);
        } else {
            return sigma_at(k);
        }
    };
    // sigma + 4c, the diagonal of the neighbour-sum form
    const Real s04 = uniform(s0 + Real(4) * c);
    auto sigma4_at = [&](int k) -> Real {
        if constexpr (kSp == 0)
            return s04 - gam * (hi[k] * S[k]);
        else
            return s04 + gam * (S[k] * S[k]);
    };
    double bb = 0.0, rr = 0.0;
    if constexpr (kFuse) {
        const Arr &Sr = *Sreg;
        const bool use64 = rtol2 < kRes64Rtol2;
        // the stash's last reads (own cells) are complete before lo lands there
        __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
        copy_to_lds<N, R, U, kLds>(lo + g.off(), stash, g);
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            P[g.idx(k)] = hi[k];
            RD_GROUP_FENCE(k)
        }
        // r0 = src - e x - c t(x) for x = hi + lo.  Evaluated in FP32 its
        // rounding (about 2^-24 of the reaction and diffusion terms, 2-3e-9
        // of |b|) lies above rtol |b| once rtol drops below about 3e-8, and
        // CG would spend iterations on that noise every step; there it is
        // evaluated in FP64, with e from the other field's hi + lo too.
        // At looser tolerances the FP32 form costs less.  The operator of the
        // CG itself stays FP32: its rounding enters only through the
        // increment, far below the tolerance.
        if (use64) {
            // the other field's low part (level n, in the slot; q is free
            // until the predictor).  Loaded here, not ahead of the copy of
            // lo: held across it, the 16 registers made the compiler spill
            // inside the CG loop.
            const int o = g.off();
#pragma unroll U
            for (int k = 0; k < R; ++k)
                q[k] = Slo[o + k * N];
            __syncthreads();
            const double e0d = e0, gamd = gam, srcd = src, cd = c;
            sweep_pair64<N, R, U>(P, stash, g, [&](int k, Real own, double t64, Real lown, Real lt) {
                const double x64 = (double)own + (double)lown;
                const double s64 = (double)Sr[k] + (double)q[k];
                const double e = kSp == 0 ? e0d - gamd * (x64 * s64) : e0d + gamd * (s64 * s64);
                const Real b = own * inv_dt + src;
                const double res64 = (srcd - e * x64) - cd * (t64 + (double)lt);
                Real res = (Real)res64;
                RD_PIN(res);
                r[k] = res;
                bb += (double)b * (double)b;
                rr += (double)res * (double)res;
                RD_PIN(bb);
                RD_PIN(rr);
            });
        } else {
            __syncthreads();
            auto e_reg = [&](int k) -> Real {
                if constexpr (kSp == 0)
                    return e0 - gam * (hi[k] * Sr[k]);
                else
                    return e0 + gam * (Sr[k] * Sr[k]);
            };
            sweep_pair<N, R, U>(P, stash, g, [&](int k, Real own, Real t, Real lown, Real lt) {
                const Real e = e_reg(k);
                const Real b = own * inv_dt + src;
                Real res = src - e * own - c * t;
                res = res - (e * lown + c * lt);
                RD_PIN(res);
                r[k] = res;
                bb += (double)b * (double)b;
                rr += (double)res * (double)res;
                RD_PIN(bb);
                RD_PIN(rr);
            });
        }
        __syncthreads();  // every stencil read of P and of the stash is done
#pragma unroll U
        for (int k = 0; k < R; ++k)
            stash[g.idx(k)] = Sr[k];
    } else {
#pragma unroll U
    for (int k = 0; k < R; ++k) {
        P[g.idx(k)] = hi[k];
        RD_GROUP_FENCE(k)
    }
    __syncthreads();

    // r0 = b - A x = src - e x - c t(x): the 1/dt terms cancel exactly, so
    // r0 (the scaled time derivative) keeps full relative precision.
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
    }
    bool rr_pending = false;
    if (kPred2 && npred == 2) {
        // Gram entries (H_i, A H_j) and (H_i, r0) from two stencil sweeps;
        // then d0 = w1 H1 + w2 H2 goes to P and one more sweep forms A d0.
        // No stencil result is kept across sweeps (register pressure).
        if constexpr (!kFuse)
            __syncthreads();  // every stencil read of P is done
        copy_to_lds<N, R, U, kLds>(H1 + g.off(), P, g);
        __syncthreads();
        const Real *h2 = H2 + g.off();
        // H2's own cells are loaded a group of cells at a time, at the
        // group's first cell: loaded at each cell, between the pinned sums,
        // every load was waited for before the next (one global round trip
        // per cell); a window of more cells ahead made the compiler spill
        double g11 = 0.0, g12 = 0.0, b1 = 0.0;
        Real h2g[kGroup];
        sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
            if (k % kGroup == 0) {
#pragma unroll
                for (int j = 0; j < kGroup; ++j)
                    h2g[j] = k + j < R ? h2[(k + j) * N] : Real(0);
            }
            Real w = c * t + sigma_seq(k) * own;  // (A H1) at the cell
            RD_PIN(w);
            const double wd = (double)w;
            g11 += (double)own * wd;
            g12 += (double)h2g[k % kGroup] * wd;  // (H2, A H1) = (H1, A H2)
            b1 += (double)own * (double)r[k];
            RD_PIN(g11);
            RD_PIN(g12);
            RD_PIN(b1);
        });
        __syncthreads();  // every stencil read of H1 is done
        copy_to_lds<N, R, U, kLds>(h2, P, g);
        __syncthreads();
        double g22 = 0.0, b2 = 0.0;
        sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
            Real w = c * t + sigma_seq(k) * own;  // (A H2) at the cell
            RD_PIN(w);
            g22 += (double)own * (double)w;
            b2 += (double)own * (double)r[k];
            RD_PIN(g22);
            RD_PIN(b2);
        });
        double v7[7] = {bb, rr, g11, g12, g22, b1, b2};
        block_sum_n<NW>(v7, red + Slots<NW>::setup, g.wid);
        bb = v7[0];
        rr = v7[1];
        g11 = v7[2];
        g12 = v7[3];
        g22 = v7[4];
        b1 = v7[5];
        b2 = v7[6];
        quiet = !(rr > rtol2 * bb);
        double w1 = 0.0, w2 = 0.0;
        const double det = g11 * g22 - g12 * g12;
        if (g11 > 0.0 && g22 > 0.0 && finite(det) && det > 1e-12 * g11 * g22 && finite(b1) &&
            finite(b2)) {
            w1 = (b1 * g22 - b2 * g12) / det;
            w2 = (b2 * g11 - b1 * g12) / det;
        } else if (g11 > 0.0 && finite(b1)) {
            w1 = b1 / g11;  // the pair is (nearly) dependent: H1 alone
        }
        const Real W1 = uniform((Real)w1), W2 = uniform((Real)w2);
        // d0 = w1 H1 + w2 H2 (own cells; the reduction barrier ended the
        // stencil reads of H2), then r0 - A d0 from its stencil
        const Real *h1 = H1 + g.off();
        Real hg[kGroup];  // H1's own cells, a group at a time (as H2 above)
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            if (k % kGroup == 0) {
#pragma unroll
                for (int j = 0; j < kGroup; ++j)
                    hg[j] = k + j < R ? h1[(k + j) * N] : Real(0);
            }
            Real dk = W1 * hg[k % kGroup];
            dk = dk + W2 * P[g.idx(k)];
            RD_PIN(dk);
            d[k] = dk;
            P[g.idx(k)] = dk;
            RD_GROUP_FENCE(k)
        }
        __syncthreads();
        sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
            Real w = c * t + sigma_seq(k) * own;  // (A d0) at the cell
            RD_PIN(w);
            r[k] = r[k] - w;
        });
        // every stencil read of P is done before the threads overwrite
        // their own cells with the residual below
        __syncthreads();
        // |r0 - A d0|^2 is summed from the updated r in the first CG sweep
        rr_pending = true;
    } else if (npred == 1) {
        if constexpr (!kFuse)
            __syncthreads();  // every stencil read of P is done
        copy_to_lds<N, R, U, kLds>(H1 + g.off(), P, g);
        __syncthreads();
        double rw = 0.0, ww = 0.0;
        sweep<N, R, U>(P, g, [&](int k, Real own, Real t) {
            Real w = c * t + sigma_seq(k) * own;  // (A H) at the cell
            RD_PIN(w);
            q[k] = w;
            rw += (double)r[k] * (double)w;
            ww += (double)w * (double)w;
            RD_PIN(rw);
            RD_PIN(ww);
        });
        double v4[4] = {bb, rr, rw, ww};
        block_sum_n<NW>(v4, red + Slots<NW>::setup, g.wid);
        bb = v4[0];
        rr = v4[1];
        rw = v4[2];
        ww = v4[3];
        quiet = !(rr > rtol2 * bb);
        const Real w = uniform((Real)((ww > 0.0 && finite(rw)) ? rw / ww : 0.0));
        Real pg[kGroup];  // H's own cells, a group at a time (as in the CG loop)
#pragma unroll U
        for (int k = 0; k < R; ++k) {
            if constexpr (U == R) {
                if (k % kGroup == 0) {
#pragma unroll
                    for (int j = 0; j < kGroup; ++j)
                        pg[j] = k + j < R ? P[g.idx(k + j)] : Real(0);
                }
                d[k] = w * pg[k % kGroup];
            } else {
                d[k] = w * P[g.idx(k)];
            }
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
        quiet = !(rr > rtol2 * bb);
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
        sweep_nsum<N, R, U>(P, g, [&](int k, Real own, Real sn) {
            Real qq = sigma4_at(k) * own - c * sn;
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
            block_sum_n<NW>(v2, red + Slots<NW>::setup, g.wid);
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
            pq = block_sum<NW>(pq0 + pq1, red + Slots<NW>::pq, g.wid);
        }
        if (!finite(pq)) {
            st = kStNonfinite;
            break;
        }
        if (!(pq > 0.0)) {
            st = kStBreakdown;
            break;
        }
        const Real a = step_ratio<Real>(rr, pq);
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
        const double rn = block_sum<NW>(rn0 + rn1, red + Slots<NW>::rr, g.wid);
        ++it;
        if (!finite(rn)) {
            st = kStNonfinite;
            break;
        }
        const Real bt = step_ratio<Real>(rn, rr);
        // d += alpha p_old and p = r + beta p_old (own cells only; the
        // stencil reads of p finished before the p.q barrier).  Fully
        // unrolled, the reads of a group of cells are issued together
        // before its writes: read cell by cell, each read waited for the
        // write before it (the compiler does not separate the cells'
        // addresses), one LDS round trip per cell on every wave's path.
        if constexpr (U == R) {
            Real pg[kGroup];
#pragma unroll
            for (int k = 0; k < R; ++k) {
                if (k % kGroup == 0) {
#pragma unroll
                    for (int j = 0; j < kGroup; ++j)
                        pg[j] = k + j < R ? P[g.idx(k + j)] : Real(0);
                }
                const Real p = pg[k % kGroup];
                d[k] = d[k] + a * p;
                P[g.idx(k)] = r[k] + bt * p;
                RD_GROUP_FENCE(k)
            }
        } else {
#pragma unroll U
            for (int k = 0; k < R; ++k) {
                const Real p = P[g.idx(k)];
                d[k] = d[k] + a * p;
                P[g.idx(k)] = r[k] + bt * p;
                RD_GROUP_FENCE(k)
            }
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
//
// acc (optional): adds sum over own cells of d^2 (FP64), the squared size of
// the step for the steady-state test.
template <int N, int R, int U, bool kDGlobal, typename Real, class Arr>
__device__ __forceinline__ void fold(Arr &hi, Arr &d, Real *lo, Real *H, const Geo<N, R> &g,
                                     double *acc = nullptr)
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
            if (acc)
                *acc += (double)dk * (double)dk;
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
        if (acc)
            *acc += (double)dd[k] * (double)dd[k];
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
// the increments of u and v of the last two steps (predictor history, two
// buffers per species that alternate by step parity), then (streamed
// variant only) the strip arrays and p.
template <typename Real>
struct SlotLayout {
    static constexpr int lo_u = 0, lo_v = 1, arrays = 6;
    // history buffer k (0 or 1) of species sp (0 u, 1 v)
    static constexpr int hist(int sp, int k) { return 2 + sp + 2 * k; }
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
//
// kPred2: the CG start vector uses the increments of the last two steps
// (cg_solve, npred = 2); otherwise the last one only.  Kernels that inline
// several grid classes keep the one-increment start (its fewer live values
// keep their register spills down).
template <int N, int R, int U, int NW, bool kLds, typename Real, bool kPred2, class Arr>
//
// steady_tt > 0 (Sec. 3.1.2): stop after the first step whose discrete time
// derivative has an L2 norm over the unit square below the threshold,
// sqrt(h^2 sum (du^2 + dv^2)) / dt < tol with h = 1/N, i.e. sum (du^2 + dv^2)
// < (tol dt N)^2 with steady_tt = tol dt; n_steps is then the cap, and an
// item that reaches it gets kStNotSteady.  `steps` returns the steps taken.
__device__ int integrate(Arr &xu, Arr &xv, Arr &r, Arr &q, Arr &d, const double th[4],
                         const GridDev &gd, double dt, int n_steps, double rtol2, int maxit,
                         Real *P, Real *stash, Real *slot, double *red, const Geo<N, R> &g,
                         int &itu, int &itv, double steady_tt, int &steps)
{
    using L = SlotLayout<Real>;
    constexpr bool comp = Compensated<Real>::on;
    Real *const lo_u = comp ? slot + L::lo_u * N * N : nullptr;
    Real *const lo_v = comp ? slot + L::lo_v * N * N : nullptr;
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
    // last residual met the tolerance before any correction skips it.  The
    // start vector from two increments costs two more stencil sweeps than
    // the one from the last increment, so it is taken only after a solve
    // that needed at least two CG iterations.
    int quiet_u = 0, quiet_v = 0, last_u = 0, last_v = 0;
    for (int s = 0; s < n_steps; ++s, rho_m2 = uniform(rho_m2 * decay)) {
        const Real cu = uniform((Real)(rho_m2 * n2));
        const Real cv = uniform((Real)(th[3] * rho_m2 * n2));
        // history: buffer (s & 1) holds the increment of step s - 2 and
        // receives this step's; buffer (s & 1) ^ 1 holds step s - 1's
        const int kn = s & 1;
        Real *const hu_new = slot + L::hist(0, kn) * N * N;
        Real *const hv_new = slot + L::hist(1, kn) * N * N;
        const Real *const hu_last = slot + L::hist(0, kn ^ 1) * N * N;
        const Real *const hv_last = slot + L::hist(1, kn ^ 1) * N * N;
        const int npred_u = (s == 0 || quiet_u) ? 0 : (s == 1 || !kPred2 || last_u < 2) ? 1 : 2;
        const int npred_v = (s == 0 || quiet_v) ? 0 : (s == 1 || !kPred2 || last_v < 2) ? 1 : 2;
        const int itu0 = itu, itv0 = itv;
        if constexpr (kLds && comp) {
            // FP32: each solve parks the other field itself, after its fused
            // residual pass has used the stash for the low part
            LdsArr<Real, N> sv{stash + g.idx(0)};
            st = cg_solve<N, R, U, NW, kLds, 0, true, kPred2>(xu, sv, r, q, d, inv_dt, cu, src_u, dl, gam,
                                                      rtol2, maxit, P, lo_u, hu_last, hu_new,
                                                      npred_u, red, g, itu, quiet_u, &xv, stash,
                                                      lo_v);
#pragma unroll U
            for (int k = 0; k < R; ++k)
                xv[k] = sv[k];
            if (st)
                break;
            store_increment<N, R, U>(d, hu_new, g);
            st = cg_solve<N, R, U, NW, kLds, 1, true, kPred2>(xv, sv, r, q, d, inv_dt, cv, src_v, dl, gam,
                                                      rtol2, maxit, P, lo_v, hv_last, hv_new,
                                                      npred_v, red, g, itv, quiet_v, &xu, stash,
                                                      lo_u);
#pragma unroll U
            for (int k = 0; k < R; ++k)
                xu[k] = sv[k];
        } else if constexpr (kLds) {
            LdsArr<Real, N> sv{stash + g.idx(0)};
#pragma unroll U
            for (int k = 0; k < R; ++k)
                sv[k] = xv[k];
            st = cg_solve<N, R, U, NW, kLds, 0, false, kPred2>(xu, sv, r, q, d, inv_dt, cu, src_u, dl, gam, rtol2,
                                                maxit, P, lo_u, hu_last, hu_new, npred_u, red, g,
                                                itu, quiet_u);
#pragma unroll U
            for (int k = 0; k < R; ++k) {
                xv[k] = sv[k];
                if (!st)
                    sv[k] = xu[k];
            }
            if (st)
                break;
            store_increment<N, R, U>(d, hu_new, g);
            st = cg_solve<N, R, U, NW, kLds, 1, false, kPred2>(xv, sv, r, q, d, inv_dt, cv, src_v, dl, gam, rtol2,
                                                maxit, P, lo_v, hv_last, hv_new, npred_v, red, g,
                                                itv, quiet_v);
#pragma unroll U
            for (int k = 0; k < R; ++k)
                xu[k] = sv[k];
        } else {
            st = cg_solve<N, R, U, NW, kLds, 0, false, kPred2>(xu, xv, r, q, d, inv_dt, cu, src_u, dl, gam, rtol2,
                                                maxit, P, lo_u, hu_last, hu_new, npred_u, red, g,
                                                itu, quiet_u);
            if (st)
                break;
            store_increment<N, R, U>(d, hu_new, g);
            st = cg_solve<N, R, U, NW, kLds, 1, false, kPred2>(xv, xu, r, q, d, inv_dt, cv, src_v, dl, gam, rtol2,
                                                maxit, P, lo_v, hv_last, hv_new, npred_v, red, g,
                                                itv, quiet_v);
        }
        if (st)
            break;
        steps = s + 1;
        if (steady_tt > 0.0) {
            double acc = 0.0;
            fold<N, R, U, false>(xv, d, lo_v, hv_new, g, &acc);
            fold<N, R, U, true>(xu, d, lo_u, hu_new, g, &acc);
            const double thr = steady_tt * (double)N;
            if (block_sum<NW>(acc, red + Slots<NW>::misfit) < thr * thr)
                return st;
        } else {
            fold<N, R, U, false>(xv, d, lo_v, hv_new, g);
            fold<N, R, U, true>(xu, d, lo_u, hu_new, g);
        }
        last_u = uniform(itu - itu0);
        last_v = uniform(itv - itv0);
    }
    if (!st && steady_tt > 0.0)
        st = kStNotSteady;  // the cap came first
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
                            int itu, int itv, const Real *slot, const Geo<N, R> &g, double *red,
                            int steps)
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
        if (a.steps_out)
            a.steps_out[c] = steps;
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
        if (a.iters) {
            a.iters[2 * c] = 0;
            a.iters[2 * c + 1] = 0;
        }
        if (a.steps_out)
            a.steps_out[c] = 0;
    }
    return -1;
}

// One item, resident variant: P and stash are LDS arrays of at least N*N.
template <int N, int R, typename Real, bool kPred2 = false>
__device__ __forceinline__ void solve_item_resident(const SolveArgs &a, int c, const GridDev &gd,
                                                    Real *P, Real *stash, double *red, Real *slot)
{
    constexpr int NW = (N * N / R) / kWave;
    const Geo<N, R> g;
    const double th[4] = {a.theta[4 * c], a.theta[4 * c + 1], a.theta[4 * c + 2],
                          a.theta[4 * c + 3]};
    RegArr<Real, R> xu, xv, r, q, d;
    load_initial<N, R, R>(gd, xu, xv, slot, g);
    int itu = 0, itv = 0, steps = 0;
    const int st = integrate<N, R, R, NW, true, Real, kPred2>(xu, xv, r, q, d, th, gd, a.dt,
                                                              a.n_steps, a.rtol2,
                                                a.maxit, P, stash, slot, red, g, itu, itv,
                                                a.steady_tt, steps);
    finish_item<N, R, Real>(a, gd, c, xu, xv, st, itu, itv, slot, g, red, steps);
}

// One item, streamed variant: the strip arrays and p follow the SlotLayout
// arrays in the workgroup's global slot.
template <int N, int R, typename Real, bool kPred2 = false>
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
    int itu = 0, itv = 0, steps = 0;
    const int st = integrate<N, R, U, NW, false, Real, kPred2>(xu, xv, r, q, d, th, gd, a.dt,
                                                               a.n_steps, a.rtol2,
                                                 a.maxit, P, (Real *)nullptr, slot, red, g, itu,
                                                 itv, a.steady_tt, steps);
    finish_item<N, R, Real>(a, gd, c, xu, xv, st, itu, itv, slot, g, red, steps);
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
                solve_item_resident<N, R, Real, true>(a, c, a.grids[gid], P, stash, red, slot);
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
                solve_item_streamed<N, R, Real, true>(a, c, a.grids[gid], red, slot);
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

// Queue order of a single-class launch: items by decreasing cost estimate
// (cost[i], CG iterations as kept by k_note_cost; a negative estimate means
// no solve yet, and such items go first, since any of them may be among the
// costliest), items that are not solved last, ties in index order.  Solve costs are heavy-tailed (a few
// parameters need tens of CG iterations per step where most need two or
// three), and a persistent queue that meets its costliest items last ends
// with most workgroups idle; largest first bounds that tail by the smallest
// items.  Only the order in which workgroups take items changes, not what an
// item computes.  One workgroup: bitonic sort of (inverted key, index) in LDS.
__global__ __launch_bounds__(1024) void k_cost_order(int n, const int *need, const int *cost,
                                                     int *order)
{
    __shared__ unsigned long long s[kMaxCostOrder];
    int np = 1;
    while (np < n)
        np <<= 1;
    for (int i = threadIdx.x; i < np; i += 1024) {
        unsigned long long v = ~0ull;  // padding sorts after every item
        if (i < n) {
            unsigned key = 0xFFFFFFFFu;  // not solved: last
            if (!need || need[i]) {
                const int c = cost[i];
                const unsigned cc = c < 0 ? 0x7FFFFFFFu : (unsigned)c;
                key = 0x7FFFFFFFu - cc;  // larger cost sorts first
            }
            v = ((unsigned long long)key << 32) | (unsigned)i;
        }
        s[i] = v;
    }
    __syncthreads();
    for (int k = 2; k <= np; k <<= 1) {
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < np; i += 1024) {
                const int l = i ^ j;
                if (l > i) {
                    const unsigned long long x = s[i], y = s[l];
                    if ((x > y) == ((i & k) == 0)) {
                        s[i] = y;
                        s[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < n; i += 1024)
        order[i] = (int)(unsigned)(s[i] & 0xFFFFFFFFull);
}

// The cost estimate of each solved item after a solve: its CG iterations
// (both species), or 7/8 of the previous estimate when that is larger.  A
// decaying maximum keeps a chain that was costly recently near the front of
// the queue (a chain near the stiff edge of the prior jumps between cheap and
// costly solves) and forgets it after a few cheap ones.
__global__ void k_note_cost(int n, const int *need, const int *iters, int *cost)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n || (need && !need[c]))
        return;
    const long long s = (long long)iters[2 * c] + (long long)iters[2 * c + 1];
    const int it = s < 0 ? 0 : (s > 0x7FFFFFFF ? 0x7FFFFFFF : (int)s);
    const int e = cost[c];
    cost[c] = e < 0 ? it : max(it, e - (e >> 3));
}

// ---------------------------------------------------------------------------
// Cooperative solve of a large grid (256 x 256) by a group of G workgroups.
//
// A single workgroup cannot hold a 256^2 item in VGPRs and LDS, and the
// streamed variant (arrays in HBM) takes ~30 s per solve on one CU.  Here
// member m of the group owns the horizontal strip of rows 64m .. 64m+63 and
// keeps it resident exactly as the 128^2 kernel does (16 cells per thread,
// 1024 threads); the 5-point stencil needs the neighbouring members' edge
// rows, and CG's dot products need the group's sums.  Both go through a
// per-group area of global memory with agent-coherent (sc1) loads and
// stores.  A group exchange publishes each member's partial sums tagged
// with the exchange's sequence number and polls the other members' slots
// until their tags match; it doubles as the group barrier, since a member
// publishes only after its own edge-row stores have completed.  No cache
// flush or invalidate is involved, so other workgroups' cached data is left
// alone.  The members of a group get workgroup ids that are congruent
// modulo 8, which the dispatcher places on the same XCD.
//
// Edge rows travel one iteration ahead: a member publishes its new residual
// edge rows before the r.r reduction, and after it computes the neighbours'
// new search-direction edge rows itself, p_nb = r_nb + beta p_nb, so one CG
// iteration needs two group exchanges (p.q and r.r).  A member rewrites an
// exchange buffer or an edge row only after an exchange that every member
// entered after its last read of it.

constexpr int kCoopStrip = kCoopN / kCoopG;              // 64 rows per member
constexpr int kCoopR = kCoopStrip * kCoopN / kCoopThreads;  // 16 cells per thread
// A group barrier gives up after SolveArgs::coop_wait_ticks ticks of the
// 100 MHz real-time counter (10 s by default): far beyond any legitimate
// wait, it only bounds the damage of a member that can never arrive.

struct CoopArea {
    // header: the item queue; then per group: partial sums [2][G][4]
    // doubles, then edge rows [4 fields][G][2][N]
    static constexpr size_t header_bytes = 256;
    static constexpr size_t partial_bytes = 2 * kCoopG * 4 * sizeof(double);
    static constexpr size_t group_bytes =
        partial_bytes + (size_t)4 * kCoopG * 2 * kCoopN * sizeof(float);
};

__host__ __device__ size_t coop_workspace_bytes(int groups)
{
    return CoopArea::header_bytes + (size_t)groups * CoopArea::group_bytes;
}

enum CoopField : int { kFieldHi = 0, kFieldLo = 1, kFieldH = 2, kFieldR = 3 };

struct CoopCtx {
    unsigned char *base;  // the group's area
    int m;                // member index
    unsigned seq;         // exchanges so far (this launch)
    int *fail;            // LDS flag: an exchange timed out
    double *gather;       // LDS [G * 4]
    unsigned long long wait_ticks;  // bound of one wait

    __device__ double *partial(unsigned k) const
    {
        return (double *)base + (size_t)(k & 1u) * kCoopG * 4;
    }
    __device__ float *halo_row(int field, int member, int side) const
    {
        return (float *)(base + CoopArea::partial_bytes) +
               (((size_t)field * kCoopG + member) * 2 + side) * kCoopN;
    }
};

// Per-lane offset made opaque at its use: the address is formed next to the
// access from the uniform base, instead of a 64-bit lane address hoisted out
// of the CG loop (which the register allocator then spills).
__device__ __forceinline__ int lane_off(int o)
{
    asm volatile("" : "+v"(o));
    return o;
}

__device__ __forceinline__ void coop_store(float *p, float v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float coop_load(const float *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void coop_store(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double coop_load(const double *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// A published value carries the exchange's sequence number in its 8 lowest
// mantissa bits, so the value is its own arrival flag: one coherent store
// and one poll per member, no counter.  The change is below 2^-44 relative,
// far under the rounding error of the FP64 sums themselves, and every
// member sums the same tagged values in the same order.  Exchanges are
// double buffered by sequence parity, and every exchange rewrites all four
// slots of its member (unused ones carry zero), so a slot's stale tag is
// always exactly two behind.  (Were only the M slots in use rewritten, a
// slot that a long run of one-value exchanges leaves alone would hold the
// tag of an exchange 256 k sequence numbers back, which the 8-bit tag
// cannot tell from the present one: the poll would take the old value, and
// the exchange would stop being a barrier.)
__device__ __forceinline__ double with_tag(double v, unsigned tag)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    return __longlong_as_double((long long)((b & ~0xFFull) | (tag & 0xFFu)));
}
__device__ __forceinline__ unsigned tag_of(double v)
{
    return (unsigned)((unsigned long long)__double_as_longlong(v) & 0xFFu);
}

// Group exchange of M values that every thread of the member holds: on
// return v holds the sums over the members, in member order (the same in
// every member).  Also a group barrier: every coherent store that a thread
// of any member issued before the exchange is visible after it.  Bounded:
// after x.wait_ticks the member gives up and raises *fail, and a member
// that has failed no longer waits, so every exchange ends.
template <int M>
__device__ void coop_exchange(double (&v)[M], CoopCtx &x)
{
    // this thread's coherent stores are complete before the value is published
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
    x.seq += 1;
    const unsigned tag = x.seq & 0xFFu;
    double *buf = x.partial(x.seq);
    const int t = threadIdx.x;
    // The store and the polls are separate blocks, store first: as the
    // two sides of one branch they could run in either order within the
    // wave, and a wave that polls before it stores waits for members that
    // do the same.
    if (t < 4) {  // this member's four slots, value t (zero past M)
        double mine = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q)
            if (t == q)
                mine = v[q];
        const double pub = with_tag(mine, tag);
        coop_store(buf + lane_off(x.m * 4 + t), pub);
        if (t < M)
            x.gather[x.m * M + t] = pub;
    }
    asm volatile("" ::: "memory");
    if (t < kCoopG * M && t / M != x.m) {
        const int mm = t / M, j = t % M;  // lane t: value j of member mm
        double got = 0.0;
        if (!*x.fail) {
            got = coop_load(buf + lane_off(mm * 4 + j));
            if (tag_of(got) != tag) {
                const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
                do {
                    __builtin_amdgcn_s_sleep(1);
                    got = coop_load(buf + lane_off(mm * 4 + j));
                    if (__builtin_amdgcn_s_memrealtime() - t0 > x.wait_ticks) {
                        *x.fail = 1;
                        break;
                    }
                } while (tag_of(got) != tag);
            }
        }
        x.gather[t] = got;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double sum = 0.0;
#pragma unroll
        for (int mm = 0; mm < kCoopG; ++mm)
            sum += x.gather[mm * M + j];
        v[j] = uniform(sum);
    }
}

// Group barrier (an exchange of nothing).
__device__ __forceinline__ void coop_sync(CoopCtx &x)
{
    double z[1] = {0.0};
    coop_exchange<1>(z, x);
}

// Sums of M per-thread values over the group's threads.
template <int NW, int M>
__device__ void coop_sum(double (&v)[M], double *red, CoopCtx &x)
{
    // as block_sum_n followed by coop_exchange, with one workgroup barrier
    // fewer: the lanes that publish form this member's sums themselves
#pragma unroll
    for (int m = 0; m < M; ++m)
        v[m] = wave_sum_last_lane(v[m]);
    // this thread's coherent stores are complete before the value is published
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
    const int t = threadIdx.x;
    if ((t & (kWave - 1)) == kLastLane) {
#pragma unroll
        for (int m = 0; m < M; ++m)
            red[m * NW + t / kWave] = v[m];
    }
    __syncthreads();
    double own[M];
    slots_sum<NW>(own, red);  // this member's sums (wave-uniform)
    x.seq += 1;
    const unsigned tag = x.seq & 0xFFu;
    double *buf = x.partial(x.seq);
    if (t < 4) {  // lanes 0..3 publish this member's four slots (zero past M)
        double sum = 0.0;
#pragma unroll
        for (int q = 0; q < M; ++q)
            if (t == q)
                sum = own[q];
        const double pub = with_tag(sum, tag);
        coop_store(buf + lane_off(x.m * 4 + t), pub);
        if (t < M)
            x.gather[x.m * M + t] = pub;
    }
    asm volatile("" ::: "memory");  // the store is issued before any poll
    if (t < kCoopG * M && t / M != x.m) {
        const int mm = t / M, j = t % M;  // lane t: value j of member mm
        double got = 0.0;
        if (!*x.fail) {
            got = coop_load(buf + lane_off(mm * 4 + j));
            if (tag_of(got) != tag) {
                const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
                do {
                    __builtin_amdgcn_s_sleep(1);
                    got = coop_load(buf + lane_off(mm * 4 + j));
                    if (__builtin_amdgcn_s_memrealtime() - t0 > x.wait_ticks) {
                        *x.fail = 1;
                        break;
                    }
                } while (tag_of(got) != tag);
            }
        }
        x.gather[t] = got;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < M; ++j) {
        double sum = 0.0;
#pragma unroll
        for (int mm = 0; mm < kCoopG; ++mm)
            sum += x.gather[mm * M + j];
        v[j] = uniform(sum);
    }
}

// Thread layout of a member: thread t owns column i = t % N, local rows
// jl0 .. jl0 + R - 1 of the strip.  LDS P has one halo row on each side:
// local row jl is at P[(jl + 1) N + i].
struct CoopGeo {
    int i, jl0, iw, ie;
    __device__ CoopGeo()
    {
        i = threadIdx.x % kCoopN;
        jl0 = (threadIdx.x / kCoopN) * kCoopR;
        iw = i > 0 ? i - 1 : i;
        ie = i < kCoopN - 1 ? i + 1 : i;
    }
    __device__ int idx(int k) const { return (jl0 + k + 1) * kCoopN + i; }  // into P (halo rows)
    __device__ int sidx(int k) const { return (jl0 + k) * kCoopN + i; }     // strip arrays
    __device__ __forceinline__ int off() const
    {
        int o = jl0 * kCoopN + i;
        asm volatile("" : "+v"(o));
        return o;
    }
    __device__ bool top() const { return jl0 == 0; }                           // owns row 0
    __device__ bool bottom() const { return jl0 + kCoopR == kCoopStrip; }      // owns last row
};

// 5-point sweep over own cells with the halo rows in place.
template <typename F>
__device__ __forceinline__ void sweep_coop(const float *P, const CoopGeo &g, F &&f)
{
    constexpr int N = kCoopN, R = kCoopR;
    float cur = P[g.idx(0)];
    float south = P[g.idx(0) - N];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const float north = P[g.idx(k) + N];
        const float west = P[g.idx(k) - g.i + g.iw];
        const float east = P[g.idx(k) - g.i + g.ie];
        const float t = ((cur - west) + (cur - east)) + ((cur - south) + (cur - north));
        f(k, cur, t);
        south = cur;
        cur = north;
        RD_GROUP_FENCE(k)
    }
}

// sweep_coop() with the plain neighbour sum (see sweep_nsum), for the CG
// iteration on the increment.
template <class F>
__device__ __forceinline__ void sweep_coop_nsum(const float *P, const CoopGeo &g, F &&f)
{
    constexpr int N = kCoopN, R = kCoopR;
    float cur = P[g.idx(0)];
    float south = P[g.idx(0) - N];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const float north = P[g.idx(k) + N];
        const float west = P[g.idx(k) - g.i + g.iw];
        const float east = P[g.idx(k) - g.i + g.ie];
        const float sn = (west + east) + (south + north);
        f(k, cur, sn);
        south = cur;
        cur = north;
        RD_GROUP_FENCE(k)
    }
}

// Publish this member's edge rows of `field` (values v(k) of own cells).
template <class V>
__device__ __forceinline__ void coop_publish(const CoopCtx &x, int field, const CoopGeo &g, V &&v)
{
    if (g.top())
        coop_store(x.halo_row(field, x.m, 0) + lane_off(g.i), v(0));
    if (g.bottom())
        coop_store(x.halo_row(field, x.m, 1) + lane_off(g.i), v(kCoopR - 1));
}

// After a barrier: fill P's halo rows with the neighbours' published edge
// rows of `field` (mirror rows at the domain boundary: the member's own
// edge row, already in P).  The caller synchronises before the sweep.
__device__ __forceinline__ void coop_fetch_halo(const CoopCtx &x, int field, float *P)
{
    constexpr int N = kCoopN;
    const int t = threadIdx.x;
    if (t < N) {
        P[t] = x.m > 0 ? coop_load(x.halo_row(field, x.m - 1, 1) + lane_off(t)) : P[N + t];
    } else if (t < 2 * N) {
        const int c = t - N;
        P[(kCoopStrip + 1) * N + c] = x.m < kCoopG - 1
                                          ? coop_load(x.halo_row(field, x.m + 1, 0) + lane_off(c))
                                          : P[kCoopStrip * N + c];
    }
}

// CG for the increment of one species on the member's strip (the algorithm
// of cg_solve, FP32 compensated, with group barriers for halos and sums).
template <int kSp>
__device__ int cg_coop(const RegArr<float, kCoopR> &hi, const LdsArr<float, kCoopN> &S,
                       RegArr<float, kCoopR> &r, RegArr<float, kCoopR> &q,
                       RegArr<float, kCoopR> &d, float inv_dt, float c, float src, float dl,
                       float gam, double rtol2, int maxit, float *P, const float *lo,
                       const float *H, bool pred, double *red, const CoopGeo &g, CoopCtx &x,
                       int &it_acc, const float *Slo)
{
    constexpr int R = kCoopR, NW = kCoopThreads / kWave;
    const float e0 = uniform(kSp == 0 ? dl + gam : dl);
    const float s0 = uniform(e0 + inv_dt);
    auto e_at = [&](int k) -> float {
        if constexpr (kSp == 0)
            return e0 - gam * (hi[k] * S[k]);
        else
            return e0 + gam * (S[k] * S[k]);
    };
    auto sigma_at = [&](int k) -> float {
        if constexpr (kSp == 0)
            return s0 - gam * (hi[k] * S[k]);
        else
            return s0 + gam * (S[k] * S[k]);
    };
    const float s04 = uniform(s0 + 4.0f * c);  // sigma + 4c: the neighbour-sum form
    auto sigma4_at = [&](int k) -> float {
        if constexpr (kSp == 0)
            return s04 - gam * (hi[k] * S[k]);
        else
            return s04 + gam * (S[k] * S[k]);
    };
    const float *lp = lo + g.off();
    const float *hp = H + g.off();
    // every field of the set-up travels before one barrier
    coop_publish(x, kFieldHi, g, [&](int k) { return hi[k]; });
    coop_publish(x, kFieldLo, g, [&](int k) { return lp[k * kCoopN]; });
    if (pred)
        coop_publish(x, kFieldH, g, [&](int k) { return hp[k * kCoopN]; });
#pragma unroll
    for (int k = 0; k < R; ++k) {
        P[g.idx(k)] = hi[k];
        RD_GROUP_FENCE(k)
    }
    coop_sync(x);
    coop_fetch_halo(x, kFieldHi, P);
    __syncthreads();
    // r0 in FP32 (hi pass, then lo pass).  The resident tiles evaluate it in
    // FP64, which saves CG iterations at rtol 1e-9; here the extra registers
    // of that evaluation made the compiler spill inside the CG loop, which
    // cost more than the iterations saved.
    double bb = 0.0, rr = 0.0;
    const float *slp = Slo + g.off();
    const double e0d = e0, gamd = gam;
    sweep_coop(P, g, [&](int k, float own, float t) {
        const float b = own * inv_dt + src;
        // the reaction coefficient from both fields' hi + lo in FP64,
        // rounded once: 1 - u v cancels, and in FP32 its rounding noise lay
        // above rtol |b|
        const double x64 = (double)own + (double)lp[k * kCoopN];
        const double s64 = (double)S[k] + (double)slp[k * kCoopN];
        const float e = (float)(kSp == 0 ? e0d - gamd * (x64 * s64) : e0d + gamd * (s64 * s64));
        float res = src - e * own - c * t;
        RD_PIN(res);
        r[k] = res;
        bb += (double)b * (double)b;
        RD_PIN(bb);
    });
    __syncthreads();
#pragma unroll
    for (int k = 0; k < R; ++k)
        P[g.idx(k)] = lp[k * kCoopN];
    __syncthreads();
    coop_fetch_halo(x, kFieldLo, P);
    __syncthreads();
    sweep_coop(P, g, [&](int k, float own, float t) {
        float res = r[k] - (e_at(k) * own + c * t);
        RD_PIN(res);
        r[k] = res;
        rr += (double)res * (double)res;
        RD_PIN(rr);
    });
    bool rr_pending = false;
    if (pred) {
        __syncthreads();
#pragma unroll
        for (int k = 0; k < R; ++k)
            P[g.idx(k)] = hp[k * kCoopN];
        __syncthreads();
        coop_fetch_halo(x, kFieldH, P);
        __syncthreads();
        double rw = 0.0, ww = 0.0;
        sweep_coop(P, g, [&](int k, float own, float t) {
            float w = c * t + sigma_at(k) * own;
            RD_PIN(w);
            q[k] = w;
            rw += (double)r[k] * (double)w;
            ww += (double)w * (double)w;
            RD_PIN(rw);
            RD_PIN(ww);
        });
        double v4[4] = {bb, rr, rw, ww};
        coop_sum<NW>(v4, red, x);
        bb = v4[0];
        rw = v4[2];
        ww = v4[3];
        const float w = uniform((float)((ww > 0.0 && finite(rw)) ? rw / ww : 0.0));
#pragma unroll
        for (int k = 0; k < R; ++k) {
            d[k] = w * P[g.idx(k)];
            r[k] = r[k] - w * q[k];
            RD_GROUP_FENCE(k)
        }
        rr_pending = true;  // |r|^2 is summed exactly in the first CG sweep
        // the halo of p = r (the predicted residual) comes from the
        // neighbours' own update: exchanged below with the r rows
    } else {
        double v2[2] = {bb, rr};
        coop_sum<NW>(v2, red, x);
        bb = v2[0];
        rr = v2[1];
#pragma unroll
        for (int k = 0; k < R; ++k)
            d[k] = 0.0f;
    }
    // p0 = r: own rows, and the neighbours' edge rows of r
    coop_publish(x, kFieldR, g, [&](int k) { return r[k]; });
#pragma unroll
    for (int k = 0; k < R; ++k) {
        P[g.idx(k)] = r[k];
        RD_GROUP_FENCE(k)
    }
    coop_sync(x);
    coop_fetch_halo(x, kFieldR, P);

    const double tol2 = rtol2 * bb;
    int st = (finite(bb) && finite(rr)) ? 0 : kStNonfinite;
    int it = 0;
    while (st == 0 && (rr_pending || rr > tol2)) {
        if (*x.fail) {
            st = kStGroupTimeout;
            break;
        }
        if (it >= maxit) {
            st = kStNotConverged;
            break;
        }
        __syncthreads();  // p (own rows and halo) visible
        double pq = 0.0, rp = 0.0;
        sweep_coop_nsum(P, g, [&](int k, float own, float sn) {
            float qq = sigma4_at(k) * own - c * sn;
            RD_PIN(qq);
            q[k] = qq;
            pq += (double)own * (double)qq;
            RD_PIN(pq);
            if (rr_pending) {
                rp += (double)own * (double)own;
                RD_PIN(rp);
            }
        });
        double v2[2] = {pq, rp};
        coop_sum<NW>(v2, red, x);
        pq = v2[0];
        if (rr_pending) {
            rr = v2[1];
            rr_pending = false;
            if (!finite(rr)) {
                st = kStNonfinite;
                break;
            }
            if (!(rr > tol2))
                break;
        }
        if (!finite(pq)) {
            st = kStNonfinite;
            break;
        }
        if (!(pq > 0.0)) {
            st = kStBreakdown;
            break;
        }
        const float a = step_ratio<float>(rr, pq);
        double rn = 0.0;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const float v = r[k] - a * q[k];
            r[k] = v;
            rn += (double)v * (double)v;
            RD_GROUP_FENCE(k)
        }
        coop_publish(x, kFieldR, g, [&](int k) { return r[k]; });
        double v1[1] = {rn};
        coop_sum<NW>(v1, red, x);
        rn = v1[0];
        ++it;
        if (!finite(rn)) {
            st = kStNonfinite;
            break;
        }
        const float bt = step_ratio<float>(rn, rr);
        static_assert(R % kGroup == 0, "whole groups");
        float pg[kGroup];  // own cells of p, a group at a time (as in cg_solve)
#pragma unroll
        for (int k = 0; k < R; ++k) {
            if (k % kGroup == 0) {
#pragma unroll
                for (int j = 0; j < kGroup; ++j)
                    pg[j] = P[g.idx(k + j)];
            }
            const float p = pg[k % kGroup];
            d[k] = d[k] + a * p;
            P[g.idx(k)] = __builtin_fmaf(bt, p, r[k]);
            RD_GROUP_FENCE(k)
        }
        // neighbours' new edge rows of p from their published r and the old p
        {
            constexpr int N = kCoopN;
            const int t = threadIdx.x;
            if (t < N && x.m > 0) {
                P[t] = __builtin_fmaf(bt, P[t],
                                      coop_load(x.halo_row(kFieldR, x.m - 1, 1) + lane_off(t)));
            } else if (t >= N && t < 2 * N && x.m < kCoopG - 1) {
                float *h = P + (kCoopStrip + 1) * N + (t - N);
                *h = __builtin_fmaf(bt, *h,
                                    coop_load(x.halo_row(kFieldR, x.m + 1, 0) + lane_off(t - N)));
            }
        }
        __syncthreads();
        // mirror rows at the domain boundary follow the member's own edge rows
        {
            constexpr int N = kCoopN;
            const int t = threadIdx.x;
            if (t < N && x.m == 0)
                P[t] = P[N + t];
            else if (t >= N && t < 2 * N && x.m == kCoopG - 1)
                P[(kCoopStrip + 1) * N + t - N] = P[kCoopStrip * N + t - N];
        }
        rr = rn;
    }
    if (*x.fail)
        st |= kStGroupTimeout;
    it_acc += it;
    __syncthreads();
    return st;
}

// fold for the member's strip (same arithmetic as fold()).
template <bool kDGlobal>
__device__ __forceinline__ void fold_coop(RegArr<float, kCoopR> &hi, RegArr<float, kCoopR> &d,
                                          float *lo, float *H, const CoopGeo &g,
                                          double *acc = nullptr)
{
    const int o = g.off();
    float l[kCoopR], dd[kCoopR];
#pragma unroll
    for (int k = 0; k < kCoopR; ++k) {
        l[k] = lo[o + k * kCoopN];
        dd[k] = kDGlobal ? H[o + k * kCoopN] : d[k];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < kCoopR; ++k) {
        RD_PIN(l[k]);
        RD_PIN(dd[k]);
    }
#pragma unroll
    for (int k = 0; k < kCoopR; ++k) {
        float s, e;
        two_sum(hi[k], dd[k], s, e);
        const float lk = l[k] + e;
        const float nh = s + lk;
        hi[k] = nh;
        lo[o + k * kCoopN] = lk - (nh - s);
        if (!kDGlobal)
            H[o + k * kCoopN] = dd[k];
        if (acc)
            *acc += (double)dd[k] * (double)dd[k];
    }
}

// One 256^2 item by the group.  Mirrors integrate() + finish_item().
__device__ void solve_item_coop(const SolveArgs &a, int c, const GridDev &gd, float *P,
                                float *stash, double *red, float *slot, CoopCtx &x)
{
    constexpr int N = kCoopN, R = kCoopR, NS = kCoopStrip, NW = kCoopThreads / kWave;
    constexpr size_t strip = (size_t)NS * N;
    const CoopGeo g;
    const double th[4] = {a.theta[4 * c], a.theta[4 * c + 1], a.theta[4 * c + 2],
                          a.theta[4 * c + 3]};
    float *lo_u = slot, *lo_v = slot + strip, *h_u = slot + 2 * strip, *h_v = slot + 3 * strip;
    RegArr<float, R> xu, xv, r, q, d;
    {
        const int o = g.off();
        const size_t base = (size_t)x.m * strip;  // the member's rows of the whole field
        const float *u0 = (const float *)gd.u0 + base + o;
        const float *v0 = (const float *)gd.v0 + base + o;
#pragma unroll
        for (int k = 0; k < R; ++k) {
            xu[k] = u0[k * N];
            xv[k] = v0[k * N];
            lo_u[o + k * N] = u0[(size_t)N * N + k * N];
            lo_v[o + k * N] = v0[(size_t)N * N + k * N];
        }
    }
    const float inv_dt = uniform((float)(1.0 / a.dt));
    const float gam = uniform((float)th[2]);
    const float src_u = uniform((float)(th[2] * th[0]));
    const float src_v = uniform((float)(th[2] * th[1]));
    const float dl = uniform((float)gd.dil);
    const double n2 = (double)N * (double)N;
    const double decay = gd.decay;
    double rho_m2 = 1.0;
    int st = 0, itu = 0, itv = 0, last_u = 0, last_v = 0, steps = 0;
    LdsArr<float, N> sv{stash + g.sidx(0)};
    for (int s = 0; s < a.n_steps; ++s, rho_m2 = uniform(rho_m2 * decay)) {
        const float cu = uniform((float)(rho_m2 * n2));
        const float cv = uniform((float)(th[3] * rho_m2 * n2));
        const bool pred_u = s > 0 && last_u > 0, pred_v = s > 0 && last_v > 0;
        const int itu0 = itu, itv0 = itv;
#pragma unroll
        for (int k = 0; k < R; ++k)
            sv[k] = xv[k];
        st = cg_coop<0>(xu, sv, r, q, d, inv_dt, cu, src_u, dl, gam, a.rtol2, a.maxit, P, lo_u,
                        h_u, pred_u, red, g, x, itu, lo_v);
#pragma unroll
        for (int k = 0; k < R; ++k) {
            xv[k] = sv[k];
            if (!st)
                sv[k] = xu[k];
        }
        if (st)
            break;
        {
            const int o = g.off();
#pragma unroll
            for (int k = 0; k < R; ++k)
                h_u[o + k * N] = d[k];
        }
        st = cg_coop<1>(xv, sv, r, q, d, inv_dt, cv, src_v, dl, gam, a.rtol2, a.maxit, P, lo_v,
                        h_v, pred_v, red, g, x, itv, lo_u);
#pragma unroll
        for (int k = 0; k < R; ++k)
            xu[k] = sv[k];
        if (st)
            break;
        steps = s + 1;
        if (a.steady_tt > 0.0) {
            // steady-state test on the group's sum of squared increments
            double v1[1] = {0.0};
            fold_coop<false>(xv, d, lo_v, h_v, g, &v1[0]);
            fold_coop<true>(xu, d, lo_u, h_u, g, &v1[0]);
            coop_sum<NW>(v1, red, x);
            const double thr = a.steady_tt * (double)N;
            if (v1[0] < thr * thr)
                break;
        } else {
            fold_coop<false>(xv, d, lo_v, h_v, g);
            fold_coop<true>(xu, d, lo_u, h_u, g);
        }
        last_u = uniform(itu - itu0);
        last_v = uniform(itv - itv0);
        if (s + 1 == a.n_steps && a.steady_tt > 0.0)
            st = kStNotSteady;  // the cap came first
    }
    // outputs: each member writes its rows; misfit summed over the group
    const size_t off = (size_t)c * a.out_stride + (size_t)x.m * strip;
    const int o = g.off();
    if (a.u_out) {
#pragma unroll
        for (int k = 0; k < R; ++k)
            ((float *)a.u_out)[off + o + k * N] = xu[k];
    }
    if (a.v_out) {
#pragma unroll
        for (int k = 0; k < R; ++k)
            ((float *)a.v_out)[off + o + k * N] = xv[k];
    }
    if (a.phi) {
        double sum = 0.0;
        if (gd.y) {
            const double *y = gd.y + (size_t)x.m * strip + o;
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const double e = y[k * N] - ((double)xu[k] + (double)lo_u[o + k * N]);
                sum += e * e;
            }
        }
        double v1[1] = {sum};
        coop_sum<NW>(v1, red, x);
        if (threadIdx.x == 0 && x.m == 0)
            a.phi[c] = (st != 0 || !gd.y || !finite(v1[0])) ? __builtin_inf() : v1[0] * gd.inv_2s2;
    }
    if (threadIdx.x == 0 && x.m == 0) {
        a.status[c] = st;
        if (a.steps_out)
            a.steps_out[c] = steps;
        if (a.iters) {
            a.iters[2 * c] = itu;
            a.iters[2 * c + 1] = itv;
        }
    }
}

// Marks queue items failed, starting with the one in *s_item, until the
// queue (or, with prefix_only, its 256^2 prefix) is exhausted.
__device__ void coop_drain(const SolveArgs &a, bool prefix_only, unsigned *queue, int *s_item)
{
    int item = uniform(*s_item);
    __syncthreads();
    while (item < a.n_items) {
        const int c = uniform(a.order ? a.order[item] : item);
        const int gid = uniform(a.grid_id ? a.grid_id[c] : 0);
        const bool bad = (unsigned)gid >= (unsigned)a.n_grids;
        if (prefix_only && (bad || uniform(a.grids[gid].n) != kCoopN))
            break;
        if (threadIdx.x == 0 && (!a.need || a.need[c])) {
            a.status[c] = bad ? kStBadGrid : kStGroupTimeout;
            if (a.phi)
                a.phi[c] = __builtin_inf();
            if (a.iters) {
                a.iters[2 * c] = 0;
                a.iters[2 * c + 1] = 0;
            }
            if (a.steps_out)
                a.steps_out[c] = 0;
        }
        if (threadIdx.x == 0)
            *s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        item = uniform(*s_item);
        __syncthreads();
    }
}

// Groups pull items from a queue of their own (the first word of the
// workspace): member 0 takes the next index and the group exchange hands it
// to the other members.  With `prefix_only` the queue is class-ordered and
// the 256^2 items form its prefix: a group stops at the first item of
// another class (or with an invalid class, which sorts last); a following
// launch serves the rest.
__device__ __forceinline__ void coop_run(const SolveArgs &a, bool prefix_only, float *P, float *stash,
                         double *red, double *gather, int *fail, int *s_item)
{
    // group of this workgroup: ids congruent modulo 8 share an XCD
    const int b = blockIdx.x;
    const int block32 = b / 32, lane32 = b % 32;
    const int member = lane32 / 8;
    const int group = block32 * 8 + lane32 % 8;
    if (threadIdx.x == 0)
        *fail = 0;
    __syncthreads();
    CoopCtx x;
    x.base = (unsigned char *)a.coop + CoopArea::header_bytes + (size_t)group * CoopArea::group_bytes;
    x.m = member;
    x.seq = 0;
    x.fail = fail;
    x.gather = gather;
    x.wait_ticks = a.coop_wait_ticks;
    unsigned *queue = (unsigned *)a.coop;
    float *slot = (float *)((char *)a.gws + (size_t)b * a.gws_stride);
    if (a.coop_stall_ticks && member == 1) {
        // Test hook (host-set): this member arrives late at the group's
        // first exchange, so that the other members' bounded waits give up.
        const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
        while (__builtin_amdgcn_s_memrealtime() - t0 < a.coop_stall_ticks)
            __builtin_amdgcn_s_sleep(8);
    }
    for (;;) {
        if (member == 0 && threadIdx.x == 0)
            *s_item = (int)atomicAdd(queue, 1u);
        __syncthreads();
        // members other than 0 contribute 0: the group sum is member 0's index
        double v[1] = {member == 0 ? (double)*s_item : 0.0};
        coop_exchange<1>(v, x);
        if (*fail) {
            // A member timed out (it cannot happen while every member is
            // resident): the group stops exchanging, and member 0 marks
            // the items it still pulls, its last one included, as failed.
            if (member == 0)
                coop_drain(a, prefix_only, queue, s_item);
            break;
        }
        const int item = (int)(v[0] + 0.5);
        if (item >= a.n_items)
            break;
        const int c = uniform(a.order ? a.order[item] : item);
        const int gid = uniform(a.grid_id ? a.grid_id[c] : 0);
        const bool bad = (unsigned)gid >= (unsigned)a.n_grids;
        if (prefix_only && (bad || uniform(a.grids[gid].n) != kCoopN))
            break;
        if (a.need && !uniform(a.need[c]))
            continue;
        if (bad) {
            if (threadIdx.x == 0 && member == 0) {
                a.status[c] = kStBadGrid;
                if (a.phi)
                    a.phi[c] = __builtin_inf();
                if (a.iters) {
                    a.iters[2 * c] = 0;
                    a.iters[2 * c + 1] = 0;
                }
                if (a.steps_out)
                    a.steps_out[c] = 0;
            }
            continue;
        }
        solve_item_coop(a, c, a.grids[gid], P, stash, red, slot, x);
    }
    // a member whose wait gave up is counted once per launch (host-visible)
    if (*fail && threadIdx.x == 0 && a.coop_timeouts)
        atomicAdd(a.coop_timeouts, 1u);
    __syncthreads();  // every thread has read *fail before the LDS is reused
}

__global__ __launch_bounds__(kCoopThreads) void k_solve_coop(SolveArgs a)
{
    constexpr int N = kCoopN, NS = kCoopStrip, NW = kCoopThreads / kWave;
    __shared__ float P[(NS + 2) * N];
    __shared__ float stash[NS * N];
    __shared__ double red[Slots<NW>::total];
    __shared__ double gather[kCoopG * 4];
    __shared__ int fail;
    __shared__ int s_item;
    coop_run(a, a.coop_wgs > 0, P, stash, red, gather, &fail, &s_item);
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
            else if (n == 256 && !a.coop_wgs)  // else the cooperative launch solved it
                solve_item_class<256, T, Real>(a, c, gd, P, stash, red, slot);
        }
    }
}


// Mixed launch with the cooperative role (FP32, 1024 threads): the first
// a.coop_wgs workgroups (a multiple of 32, all resident: they have the
// lowest ids, so they are dispatched first) serve the 256^2 prefix of the
// class-ordered queue in groups of four, then join the queue of the other
// classes, which the remaining workgroups serve from the start.  Classes
// 32^2 .. 128^2 run resident.
__global__ __launch_bounds__(kCoopThreads) void k_solve_mixed_coop(SolveArgs a)
{
    constexpr int T = kCoopThreads, NW = T / kWave, NM = 128;
    constexpr int kP = (kCoopStrip + 2) * kCoopN;
    static_assert(kP >= NM * NM, "LDS P holds a 128^2 item");
    __shared__ float P[kP];
    __shared__ float stash[NM * NM];
    __shared__ double red[Slots<NW>::total];
    __shared__ double gather[kCoopG * 4];
    __shared__ int fail;
    __shared__ int s_item;
    if ((int)blockIdx.x < a.coop_wgs)
        coop_run(a, true, P, stash, red, gather, &fail, &s_item);
    float *slot = (float *)((char *)a.gws + (size_t)blockIdx.x * a.gws_stride);
    for (int item = next_item(a.queue, &s_item); item < a.n_items;
         item = next_item(a.queue, &s_item)) {
        const int c = uniform(a.order ? a.order[item] : item);
        const int gid = (!a.need || uniform(a.need[c])) ? item_grid(a, c) : -1;
        if (gid >= 0) {
            const GridDev &gd = a.grids[gid];
            const int n = uniform(gd.n);
            if (n == 32)
                solve_item_class<32, T, float>(a, c, gd, P, stash, red, slot);
            else if (n == 64)
                solve_item_class<64, T, float>(a, c, gd, P, stash, red, slot);
            else if (n == 128)
                solve_item_class<128, T, float>(a, c, gd, P, stash, red, slot);
        }
    }
}

// wgs: the most workgroups that are resident at once (every member of a
// group must be, since members wait for each other).  The launch uses whole
// blocks of 32 workgroups (8 groups, one per XCD) and no more groups than
// items.  a.coop_wgs > 0 marks a class-ordered batch whose 256^2 prefix
// this launch serves (the mixed launch that follows serves the rest).
hipError_t launch_solve_coop(const SolveArgs &a, int wgs, hipStream_t s)
{
    const int need = (a.n_items * kCoopG + 31) / 32 * 32;
    const int grid = std::min(wgs / 32 * 32, need);
    if (!a.coop || !a.gws || grid < 32 || grid / kCoopG > a.coop_groups || grid > a.gws_slots ||
        a.gws_stride < (size_t)4 * kCoopStrip * kCoopN * sizeof(float))
        return hipErrorInvalidValue;
    // the queue starts at 0, and stale tags of an earlier launch must not
    // match this launch's
    hipError_t e = launch_fill_u32((unsigned *)a.coop, 0u,
                                   (int)(coop_workspace_bytes(grid / kCoopG) / sizeof(unsigned)), s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_solve_coop, dim3(grid), dim3(kCoopThreads), 0, s, a);
    return hipGetLastError();
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

enum Kind { kNone, kResident, kStreamed, kCoop };

Kind tile_kind(int n, int precision, int cpt)
{
    if (precision == 0) {
        if (n == 32 && (cpt == 4 || cpt == 8 || cpt == 16))
            return kResident;
        if (n == 64 && (cpt == 4 || cpt == 8 || cpt == 16))
            return kResident;
        if (n == 128 && (cpt == 16 || cpt == 32))
            return kResident;
        if (n == 256 && cpt == kCoopR)
            return kCoop;
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
// workgroups at 32^2, 64^2 and 128^2).  At 256^2 in FP32 the cooperative
// tile (16 cells per thread, four workgroups per item) is 9 to 14 times
// faster per item than the streamed one.
int default_cpt(int n, int precision)
{
    if (precision == 0)
        return n == 32 ? 16 : n == 64 ? 16 : n == 128 ? 16 : n == 256 ? kCoopR : 0;
    return n == 32 ? 8 : n == 64 ? 16 : n == 128 ? 32 : n == 256 ? 128 : 0;
}

size_t solve_slot_bytes(int n, int precision, int cpt)
{
    if (tile_kind(n, precision, cpt) == kCoop)  // one member's strip: 4 arrays
        return (size_t)4 * kCoopStrip * kCoopN * sizeof(float);
    // SlotLayout: low parts and two increments per species (6 arrays), and
    // for streamed tiles the strip arrays and p after them (6 more)
    const size_t arrays = tile_kind(n, precision, cpt) == kStreamed ? 12 : 6;
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
    if (tile_kind(n, precision, cpt) == kCoop)
        return occupancy(k_solve_coop, kCoopThreads);
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
    const size_t arrays = mixed_resident(n, precision, threads) ? 6 : 12;
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

hipError_t launch_cost_order(int n, const int *need, const int *cost, int *order, hipStream_t s)
{
    if (n <= 0 || n > kMaxCostOrder)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_cost_order, dim3(1), dim3(1024), 0, s, n, need, cost, order);
    return hipGetLastError();
}

hipError_t launch_note_cost(int n, const int *need, const int *iters, int *cost, hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_note_cost, dim3((n + 255) / 256), dim3(256), 0, s, n, need, iters, cost);
    return hipGetLastError();
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

int mixed_coop_wgs_per_cu()
{
    return occupancy(k_solve_mixed_coop, kCoopThreads);
}

// Mixed batch with 256^2 FP32 items and 1024-thread workgroups: one launch
// of k_solve_mixed_coop (a.coop_wgs leading workgroups in the cooperative
// role).  The caller has class-ordered the queue (a.order).
hipError_t launch_solve_mixed_coop(const SolveArgs &a, int wgs, hipStream_t s)
{
    if (!a.gws || !a.order || !a.coop || wgs > a.gws_slots || a.coop_wgs < 32 ||
        a.coop_wgs % 32 != 0 || a.coop_wgs > wgs || a.coop_wgs / kCoopG > a.coop_groups ||
        a.gws_stride < (size_t)4 * kCoopStrip * kCoopN * sizeof(float))
        return hipErrorInvalidValue;
    hipError_t e = launch_fill_u32((unsigned *)a.coop, 0u,
                                   (int)(coop_workspace_bytes(a.coop_wgs / kCoopG) / sizeof(unsigned)),
                                   s);
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_solve_mixed_coop, dim3(wgs), dim3(kCoopThreads), 0, s, a);
    return hipGetLastError();
}

bool tile_streamed(int n, int precision, int cpt)
{
    return tile_kind(n, precision, cpt) == kStreamed;
}

bool tile_coop(int n, int precision, int cpt)
{
    return tile_kind(n, precision, cpt) == kCoop;
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
    if (tile_kind(n, precision, cpt) == kCoop)
        return launch_solve_coop(a, wgs, s);
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
