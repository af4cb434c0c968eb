// Device helpers shared by the HIP kernels of the library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rd {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Counter-based generator: Philox4x32 with 10 rounds (Salmon, Moraes, Dror,
// Shaw, SC 2011).  Each round multiplies words 0 and 2 by the two round
// multipliers, swaps the halves and folds in the key; the key is bumped by
// the Weyl constants between rounds.
struct U32x4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U32x4 philox10(U32x4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int rnd = 0; rnd < 10; ++rnd) {
        const uint32_t lo0 = 0xD2511F53u * c.x;
        const uint32_t hi0 = __umulhi(0xD2511F53u, c.x);
        const uint32_t lo1 = 0xCD9E8D57u * c.z;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, c.z);
        c = U32x4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// Sampler stream: key = (chain, seed), counter = (step lo, step hi, purpose, block).
__device__ __forceinline__ U32x4 stream_block(uint32_t seed, uint32_t chain, uint64_t step,
                                              uint32_t purpose, uint32_t block)
{
    return philox10(U32x4{(uint32_t)step, (uint32_t)(step >> 32), purpose, block}, chain, seed);
}

// (0,1) double from the top 52 bits of hi:lo, centred in its bin (exact).
__device__ __forceinline__ double unit_open(uint32_t hi, uint32_t lo)
{
    const uint64_t k = ((uint64_t)hi << 20) | (uint64_t)(lo >> 12);
    return ((double)k + 0.5) * 0x1p-52;
}

// Box-Muller pair from one Philox block.
__device__ __forceinline__ void gauss_pair(U32x4 w, double &z0, double &z1)
{
    const double u1 = unit_open(w.x, w.y);
    const double u2 = unit_open(w.z, w.w);
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586476925286766559 * u2;
    double s, c;
    sincos(ang, &s, &c);
    z0 = rad * c;
    z1 = rad * s;
}

// Wave-uniform copies (scalar registers).  Every value that decides a branch
// around a barrier goes through one of these: the compiler then lowers the
// branch as a scalar (uniform) branch.  Without it, loops whose exit depends
// on an LDS-read value are lowered as exec-masked loops, and the control-flow
// structurizer may let some lanes of a wave leave such a loop while the rest
// of the wave passes the next s_barrier (which counts waves, not lanes).
__device__ __forceinline__ int uniform(int x)
{
    return __builtin_amdgcn_readfirstlane(x);
}

__device__ __forceinline__ float uniform(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}

__device__ __forceinline__ double uniform(double x)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// ---------------------------------------------------------------------------
// Reductions.  A wave sums its 64 lanes with DPP moves (no LDS traffic):
// four row_shr steps leave each 16-lane row's sum in its lane 15, then
// row_bcast:15 and row_bcast:31 fold the rows into lane 63.  The order of
// additions is fixed, so the result is deterministic.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_f64(double v)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)b, kCtrl, kRowMask, 0xF, true);
    const int hi =
        __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(b >> 32), kCtrl, kRowMask, 0xF, true);
    return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

constexpr int kLastLane = kWave - 1;

__device__ __forceinline__ double wave_sum_last_lane(double v)
{
    v += dpp_f64<0x111, 0xF>(v);  // row_shr:1
    v += dpp_f64<0x112, 0xF>(v);  // row_shr:2
    v += dpp_f64<0x114, 0xF>(v);  // row_shr:4
    v += dpp_f64<0x118, 0xF>(v);  // row_shr:8  -> lane 15 of each row: row sum
    v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
    v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3 -> lane 63: total
    return v;
}

// Index of this wave in its workgroup, read once into a scalar register at
// the start of a solve and handed to the reductions: recomputed from the
// thread index inside a hot loop it needs a vector register, which the
// register allocator of the large kernels then spills and reloads.
__device__ __forceinline__ int wave_index()
{
    return uniform((int)(threadIdx.x / kWave));
}

__device__ __forceinline__ double readlane_f64(double x, int lane)
{
    const uint64_t b = __builtin_bit_cast(uint64_t, x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), lane);
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// This lane's index in its wave, computed where it is used: the large
// solve kernels keep no VGPR for it across their loops (a loop-invariant
// value derived from the thread index and held across the CG loop is what
// their register allocator spills; a volatile asm is not hoisted).
__device__ __forceinline__ int lane_here()
{
    int l;
    asm volatile("v_mbcnt_lo_u32_b32 %0, -1, 0\n\tv_mbcnt_hi_u32_b32 %0, -1, %0" : "=v"(l));
    return l;
}

// The workgroup totals of M values from the per-wave totals in
// slot[m kWaves + w]: row m of the wave (lanes 16m .. 16m + 15) reads value
// m's kWaves totals in one LDS access and adds them with the four row_shr
// steps of wave_sum_last_lane, so the sum costs one LDS round trip per four
// values (a loop over the slots waits for each load in turn).  The order of
// additions is fixed and the same in every wave; the results are
// wave-uniform (scalar registers).
template <int kWaves, int M>
__device__ __forceinline__ void slots_sum(double (&v)[M], const double *slot)
{
    static_assert(kWaves <= 16, "one 16-lane row per value");
    const int lane = lane_here();
    const int row = lane >> 4, w = lane & 15;
#pragma unroll
    for (int m0 = 0; m0 < M; m0 += 4) {
        double x = 0.0;
        if (m0 + row < M && w < kWaves)
            x = slot[(m0 + row) * kWaves + w];
        x += dpp_f64<0x111, 0xF>(x);  // row_shr:1
        x += dpp_f64<0x112, 0xF>(x);  // row_shr:2
        x += dpp_f64<0x114, 0xF>(x);  // row_shr:4
        x += dpp_f64<0x118, 0xF>(x);  // row_shr:8 -> lane 15 of the row: its sum
#pragma unroll
        for (int m = m0; m < M && m < m0 + 4; ++m)
            v[m] = readlane_f64(x, 16 * (m - m0) + 15);
    }
}

template <int kWaves>
__device__ __forceinline__ double block_sum(double v, double *slot, int wid)
{
    v = wave_sum_last_lane(v);
    const int lane = threadIdx.x & (kWave - 1);
    if (lane == kLastLane)
        slot[wid] = v;
    __syncthreads();
    double s[1];
    slots_sum<kWaves>(s, slot);
    return s[0];
}

template <int kWaves>
__device__ __forceinline__ double block_sum(double v, double *slot)
{
    return block_sum<kWaves>(v, slot, wave_index());
}

template <int kWaves>
__device__ __forceinline__ void block_sum2(double &a, double &b, double *slot)
{
    a = wave_sum_last_lane(a);
    b = wave_sum_last_lane(b);
    const int lane = threadIdx.x & (kWave - 1);
    const int wid = wave_index();
    if (lane == kLastLane) {
        slot[wid] = a;
        slot[kWaves + wid] = b;
    }
    __syncthreads();
    double s[2];
    slots_sum<kWaves>(s, slot);
    a = s[0];
    b = s[1];
}

template <int kWaves, int M>
__device__ __forceinline__ void block_sum_n(double (&v)[M], double *slot, int wid)
{
#pragma unroll
    for (int m = 0; m < M; ++m)
        v[m] = wave_sum_last_lane(v[m]);
    const int lane = threadIdx.x & (kWave - 1);
    if (lane == kLastLane) {
#pragma unroll
        for (int m = 0; m < M; ++m)
            slot[m * kWaves + wid] = v[m];
    }
    __syncthreads();
    slots_sum<kWaves>(v, slot);
}

template <int kWaves, int M>
__device__ __forceinline__ void block_sum_n(double (&v)[M], double *slot)
{
    block_sum_n<kWaves>(v, slot, wave_index());
}

__device__ __forceinline__ bool finite(double x)
{
    return __builtin_isfinite(x);
}



}  // namespace rd
