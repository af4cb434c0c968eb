// Surrogate MLP of the delayed-acceptance sampler: training and inference
// with BF16 matrix-core (MFMA) GEMMs, FP32 accumulation, FP32 master weights.
//
// Network: x = phi scaled to [-1, 1] on the prior box (4 inputs)
//          -> depth x [Linear(width) + GELU] -> Linear(out_side^2),
// output in per-pixel standardised units.  Weights are [out][in] row-major.
//
// GEMM kernel: C[M][N] = sum_k A(m, k) B(k, n) on 64 x 64 tiles, K in steps
// of BK (128 when K allows it, else 32), 256 threads = 4 waves, each wave a
// 32 x 32 quarter made of 2 x 2 v_mfma_f32_16x16x32_bf16 blocks.  Operands
// are staged through LDS in (row, k) order with k contiguous, so each lane
// fetches its 8 k-values with one 16-byte LDS read.  The next K-step's tiles
// are loaded into registers while the current one is multiplied, so a step
// waits for global memory once per BK values of k, not once per 32.  Layouts
// of A and B in global memory are template parameters (forward: H W^T;
// weight gradient: dZ^T H; input gradient: dZ W).
// Epilogues fuse bias, GELU and GELU' so that every activation is written
// once.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "rd_device.hpp"
#include "rd_internal.hpp"
#include "rd_mlp.hpp"

namespace rd {

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 64, kBN = 64, kBK = 32, kBKWide = 128, kLdsPad = 8;

__device__ __forceinline__ float gelu_f(float z)
{
    return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}

__device__ __forceinline__ float gelu_grad_f(float z)
{
    return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
           z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

enum Epi { kEpiStore = 0, kEpiBias = 1, kEpiBiasGelu = 2, kEpiGeluGrad = 3 };

struct GemmArgs {
    const bf16 *A;
    const bf16 *B;
    int M, N, K;
    int lda, ldb;
    const float *bias;    // [N] (kEpiBias, kEpiBiasGelu)
    const float *zin;     // [M][N] pre-activation (kEpiGeluGrad)
    float *c32;           // [M][N] fp32 output
    bf16 *c16;            // [M][N] bf16 output (kEpiBiasGelu: gelu(z); kEpiGeluGrad: dz)
};

// A_KM: A stored [K][M] (A(m,k) = A[k*lda + m]); else [M][K].
// B_KN: B stored [K][N] (B(k,n) = B[k*ldb + n]); else [N][K].
// Each K-step moves a 64 x BK tile of A and of B: BK / 32 chunks of 8
// values per thread and operand.
template <bool A_KM, bool B_KN, int EPI, int BK>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g)
{
    constexpr int kChunks = BK / 32;  // 16-byte global loads per thread and operand
    __shared__ __attribute__((aligned(16))) bf16 As[kBM][BK + kLdsPad];
    __shared__ __attribute__((aligned(16))) bf16 Bs[kBN][BK + kLdsPad];
    const int t = threadIdx.x;
    const int lane = t & 63, wave = t >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int m0 = blockIdx.y * kBM, n0 = blockIdx.x * kBN;
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
            acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // chunk c of thread t: [row][k] layout, 64 rows of BK / 8 chunks; or
    // [k][row] layout, BK k-rows of 8 chunks.
    auto load = [&](const bf16 *X, int ld, int r0, bool km, int k0, bf16x8 (&v)[kChunks]) {
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int idx = t + 256 * c;
            if (!km) {
                const int row = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
                v[c] = *(const bf16x8 *)&X[(size_t)(r0 + row) * ld + k0 + kc];
            } else {
                const int k = idx >> 3, rc = (idx & 7) * 8;
                v[c] = *(const bf16x8 *)&X[(size_t)(k0 + k) * ld + r0 + rc];
            }
        }
    };
    auto stage = [&](bf16 (*S)[BK + kLdsPad], bool km, const bf16x8 (&v)[kChunks]) {
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int idx = t + 256 * c;
            if (!km) {
                const int row = idx / (BK / 8), kc = (idx % (BK / 8)) * 8;
                *(bf16x8 *)&S[row][kc] = v[c];
            } else {
                const int k = idx >> 3, rc = (idx & 7) * 8;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    S[rc + i][k] = v[c][i];
            }
        }
    };
    bf16x8 va[kChunks], vb[kChunks];
    load(g.A, g.lda, m0, A_KM, 0, va);
    load(g.B, g.ldb, n0, B_KN, 0, vb);
    for (int k0 = 0; k0 < g.K; k0 += BK) {
        __syncthreads();  // the previous step's LDS reads are done
        stage(As, A_KM, va);
        stage(Bs, B_KN, vb);
        __syncthreads();
        if (k0 + BK < g.K) {  // next step's tiles, in flight during the MFMAs
            load(g.A, g.lda, m0, A_KM, k0 + BK, va);
            load(g.B, g.ldb, n0, B_KN, k0 + BK, vb);
        }
        // lane l supplies row (l % 16) and k = 8 * (l / 16) .. + 7 of each
        // 32-wide slice
        const int r = lane & 15, kq = (lane >> 4) * 8;
#pragma unroll
        for (int ks = 0; ks < BK; ks += 32) {
            bf16x8 a[2], b[2];
#pragma unroll
            for (int i = 0; i < 2; ++i)
                a[i] = *(const bf16x8 *)&As[wm * 32 + i * 16 + r][ks + kq];
#pragma unroll
            for (int j = 0; j < 2; ++j)
                b[j] = *(const bf16x8 *)&Bs[wn * 32 + j * 16 + r][ks + kq];
#pragma unroll
            for (int i = 0; i < 2; ++i)
#pragma unroll
                for (int j = 0; j < 2; ++j)
                    acc[i][j] =
                        __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        }
    }
    // accumulator block layout: lane l holds column l % 16, rows 4 (l / 16) + 0..3
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int n = n0 + wn * 32 + j * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + wm * 32 + i * 16 + (lane >> 4) * 4 + q;
                const size_t o = (size_t)m * g.N + n;
                float v = acc[i][j][q];
                if (EPI == kEpiStore) {
                    g.c32[o] = v;
                } else if (EPI == kEpiBias) {
                    g.c32[o] = v + g.bias[n];
                } else if (EPI == kEpiBiasGelu) {
                    const float z = v + g.bias[n];
                    g.c32[o] = z;
                    g.c16[o] = (bf16)gelu_f(z);
                } else {  // kEpiGeluGrad: v = dH, times GELU'(z)
                    const float d = v * gelu_grad_f(g.zin[o]);
                    g.c32[o] = d;
                    g.c16[o] = (bf16)d;
                }
            }
        }
    }
}

template <bool A_KM, bool B_KN, int EPI>
static hipError_t gemm(const GemmArgs &g, hipStream_t s)
{
    if (g.M % kBM || g.N % kBN || g.K % kBK || g.K <= 0)
        return hipErrorInvalidValue;
    const dim3 grid(g.N / kBN, g.M / kBM);
    if (g.K % kBKWide == 0)
        hipLaunchKernelGGL((k_gemm<A_KM, B_KN, EPI, kBKWide>), grid, dim3(256), 0, s, g);
    else
        hipLaunchKernelGGL((k_gemm<A_KM, B_KN, EPI, kBK>), grid, dim3(256), 0, s, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Small kernels.

// x = 2 (phi - lo) / (hi - lo) - 1; rows >= n are zero (padding).
__global__ void k_scale_inputs(int n, int npad, const double *phi, SurScale sc, float *x)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad * 4)
        return;
    const int r = i >> 2, c = i & 3;
    x[i] = r < n ? (float)(2.0 * (phi[i] - sc.lo[c]) / (sc.hi[c] - sc.lo[c]) - 1.0) : 0.0f;
}

// First layer (fan-in 4): z = x W^T + b, h = GELU(z).
__global__ void k_layer0_fwd(int npad, int width, const float *x, const float *W, const float *b,
                             float *z, bf16 *h)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad * width)
        return;
    const int r = i / width, n = i % width;
    float s = b[n];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        s = fmaf(x[r * 4 + k], W[n * 4 + k], s);
    z[i] = s;
    h[i] = (bf16)gelu_f(s);
}

// Reductions over the batch rows (weight gradient of the first layer, bias
// gradients): a block takes 64 columns, its 16 waves take every 16th row,
// and the 16 partial sums are added in a fixed order (deterministic).
constexpr int kRowGroups = 16;

// First layer weight gradient: gW[n][k] = sum_r dz[r][n] x[r][k].
__global__ __launch_bounds__(1024) void k_layer0_wgrad(int rows, int width, const float *x,
                                                       const float *dz, float *gW)
{
    __shared__ float part[kRowGroups][64][4];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    float s[4] = {0.f, 0.f, 0.f, 0.f};
    if (n < width) {
        for (int r = grp; r < rows; r += kRowGroups) {
            const float d = dz[(size_t)r * width + n];
#pragma unroll
            for (int k = 0; k < 4; ++k)
                s[k] = fmaf(d, x[r * 4 + k], s[k]);
        }
    }
#pragma unroll
    for (int k = 0; k < 4; ++k)
        part[grp][lane][k] = s[k];
    __syncthreads();
    if (grp == 0 && n < width) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float t = 0.f;
            for (int q = 0; q < kRowGroups; ++q)
                t += part[q][lane][k];
            gW[n * 4 + k] = t;
        }
    }
}

// Column sums (bias gradient): db[n] = sum_r dz[r][n].
__global__ __launch_bounds__(1024) void k_colsum(int rows, int cols, const float *dz, float *db)
{
    __shared__ float part[kRowGroups][64];
    const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
    const int n = blockIdx.x * 64 + lane;
    float s = 0.f;
    if (n < cols)
        for (int r = grp; r < rows; r += kRowGroups)
            s += dz[(size_t)r * cols + n];
    part[grp][lane] = s;
    __syncthreads();
    if (grp == 0 && n < cols) {
        float t = 0.f;
        for (int q = 0; q < kRowGroups; ++q)
            t += part[q][lane];
        db[n] = t;
    }
}

// MSE over `rows` x cols: dy = 2 (y - t) / (rows cols) (zero on padded rows),
// per-row FP64 partial sums of squared errors.
__global__ void k_mse_grad(int rows, int npad, int cols, const float *y, const float *t,
                           float *dy32, bf16 *dy16, double *row_sse)
{
    __shared__ double red[4];
    const int r = blockIdx.x;
    double s = 0.0;
    const float scale = 2.0f / ((float)rows * (float)cols);
    for (int c = threadIdx.x; c < cols; c += blockDim.x) {
        const size_t o = (size_t)r * cols + c;
        float d = 0.f;
        if (r < rows) {
            const float e = y[o] - t[o];
            s += (double)e * (double)e;
            d = scale * e;
        }
        dy32[o] = d;
        dy16[o] = (bf16)d;
    }
    s = block_sum<4>(s, red);
    if (threadIdx.x == 0 && r < rows)
        row_sse[r] = s;
}

__global__ void k_mean_rows(int rows, int cols, const double *row_sse, double *loss)
{
    __shared__ double red[4];
    double s = 0.0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x)
        s += row_sse[r];
    s = block_sum<4>(s, red);
    if (threadIdx.x == 0)
        *loss = s / ((double)rows * (double)cols);
}

// Adam with bias correction; also refreshes the BF16 copy of the parameter.
__global__ void k_adam(int count, float *p, const float *g, float *m, float *v, bf16 *p16,
                       float lr, float b1, float b2, float eps, int t)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count)
        return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / (1.f - powf(b1, (float)t));
    const float vh = vi / (1.f - powf(b2, (float)t));
    const float w = p[i] - lr * mh / (sqrtf(vh) + eps);
    p[i] = w;
    if (p16)
        p16[i] = (bf16)w;
}

__global__ void k_to_bf16(int count, const float *p, bf16 *p16)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count)
        p16[i] = (bf16)p[i];
}

// Uniform(-bound, bound) initialisation from the counter-based generator
// (key = (tensor id, seed), counter = element index).
__global__ void k_init_uniform(int count, float *p, float bound, uint32_t seed, uint32_t tensor)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count)
        return;
    const U32x4 w = philox10(U32x4{(uint32_t)i, 0u, 0u, 0u}, tensor, seed);
    const double u = unit_open(w.x, w.y);
    p[i] = (float)((2.0 * u - 1.0) * bound);
}

// Block means: u [n][N][N] -> out [n][S][S], blocks of (N/S)^2 cells.
template <typename Real>
__global__ void k_downsample(int n, int N, int S, const Real *u, float *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * S * S)
        return;
    const int c = i / (S * S), J = (i / S) % S, I = i % S, f = N / S;
    double s = 0.0;
    for (int jj = 0; jj < f; ++jj)
        for (int ii = 0; ii < f; ++ii)
            s += (double)u[(size_t)c * N * N + (size_t)(J * f + jj) * N + I * f + ii];
    out[i] = (float)(s / (double)(f * f));
}

// Surrogate misfit: Phi~ = |ybar - (mean + sd y)|^2 / (2 sigma1^2), FP64.
__global__ void k_sur_misfit(int n, int cols, const float *y, const float *mean, const float *sd,
                             const double *ybar, double inv_2s2, double *ll)
{
    __shared__ double red[4];
    const int r = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < cols; c += blockDim.x) {
        const double u = (double)mean[c] + (double)sd[c] * (double)y[(size_t)r * cols + c];
        const double e = ybar[c] - u;
        s += e * e;
    }
    s = block_sum<4>(s, red);
    if (threadIdx.x == 0)
        ll[r] = finite(s) ? s * inv_2s2 : __builtin_inf();
}

__global__ void k_destandardise(int n, int cols, const float *y, const float *mean, const float *sd,
                                float *out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n * cols)
        out[i] = mean[i % cols] + sd[i % cols] * y[i];
}

__global__ void k_ybar(int N, int S, const double *y, double *ybar)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S * S)
        return;
    const int J = i / S, I = i % S, f = N / S;
    double s = 0.0;
    for (int jj = 0; jj < f; ++jj)
        for (int ii = 0; ii < f; ++ii)
            s += y[(size_t)(J * f + jj) * N + I * f + ii];
    ybar[i] = s / (double)(f * f);
}

static inline dim3 blocks_for(size_t n, int t = 256)
{
    return dim3((unsigned)((n + t - 1) / t));
}

// ---------------------------------------------------------------------------
// Host side.

struct Surrogate {
    SurrogateDesc d{};
    int L = 0;               // linear layers = depth + 1
    int out = 0;             // out_side^2
    int bpad = 0;            // row capacity (multiple of 64)
    std::vector<int> din, dout;
    std::vector<float *> W, b, gW, gb, mW, vW, mb, vb;
    std::vector<bf16 *> W16;
    std::vector<float *> Z;  // pre-activations [bpad][dout]
    std::vector<bf16 *> H;   // post-activations (bf16) [bpad][dout]
    float *x0 = nullptr;     // [bpad][4]
    float *Y = nullptr;      // [bpad][out]
    float *dz32[2] = {nullptr, nullptr};
    bf16 *dz16[2] = {nullptr, nullptr};
    double *row_sse = nullptr;
    float *mean = nullptr, *sd = nullptr;
    double *ybar = nullptr;
    double inv_2s2 = 0.0;
    bool scaled = false;
    int t = 0;
    std::vector<void *> allocs;
};

static void *salloc(Surrogate *s, size_t bytes, bool *ok)
{
    void *p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 16) != hipSuccess) {
        *ok = false;
        return nullptr;
    }
    s->allocs.push_back(p);
    return p;
}

int32_t surrogate_new(Surrogate **out, const SurrogateDesc &d, uint32_t seed)
{
    *out = nullptr;
    Surrogate *s = new Surrogate();
    s->d = d;
    s->L = d.depth + 1;
    s->out = d.out_side * d.out_side;
    s->bpad = ((d.max_batch + 63) / 64) * 64;
    bool ok = true;
    int maxw = std::max(d.width, s->out);
    for (int l = 0; l < s->L; ++l) {
        const int fi = l == 0 ? 4 : d.width;
        const int fo = l == s->L - 1 ? s->out : d.width;
        s->din.push_back(fi);
        s->dout.push_back(fo);
        const size_t nw = (size_t)fi * fo;
        s->W.push_back((float *)salloc(s, nw * 4, &ok));
        s->b.push_back((float *)salloc(s, fo * 4, &ok));
        s->gW.push_back((float *)salloc(s, nw * 4, &ok));
        s->gb.push_back((float *)salloc(s, fo * 4, &ok));
        s->mW.push_back((float *)salloc(s, nw * 4, &ok));
        s->vW.push_back((float *)salloc(s, nw * 4, &ok));
        s->mb.push_back((float *)salloc(s, fo * 4, &ok));
        s->vb.push_back((float *)salloc(s, fo * 4, &ok));
        s->W16.push_back((bf16 *)salloc(s, nw * 2, &ok));
        s->Z.push_back((float *)salloc(s, (size_t)s->bpad * fo * 4, &ok));
        s->H.push_back((bf16 *)salloc(s, (size_t)s->bpad * fo * 2, &ok));
    }
    s->x0 = (float *)salloc(s, (size_t)s->bpad * 4 * 4, &ok);
    s->Y = (float *)salloc(s, (size_t)s->bpad * s->out * 4, &ok);
    for (int k = 0; k < 2; ++k) {
        s->dz32[k] = (float *)salloc(s, (size_t)s->bpad * maxw * 4, &ok);
        s->dz16[k] = (bf16 *)salloc(s, (size_t)s->bpad * maxw * 2, &ok);
    }
    s->row_sse = (double *)salloc(s, (size_t)s->bpad * 8, &ok);
    s->mean = (float *)salloc(s, s->out * 4, &ok);
    s->sd = (float *)salloc(s, s->out * 4, &ok);
    s->ybar = (double *)salloc(s, s->out * 8, &ok);
    if (!ok) {
        surrogate_destroy(s);
        return -3;
    }
    for (int l = 0; l < s->L; ++l) {
        const int nw = s->din[l] * s->dout[l];
        const float bound = 1.0f / sqrtf((float)s->din[l]);
        hipLaunchKernelGGL(k_init_uniform, blocks_for(nw), dim3(256), 0, nullptr, nw, s->W[l], bound,
                           seed, (uint32_t)(2 * l));
        hipLaunchKernelGGL(k_init_uniform, blocks_for(s->dout[l]), dim3(256), 0, nullptr, s->dout[l],
                           s->b[l], bound, seed, (uint32_t)(2 * l + 1));
        hipLaunchKernelGGL(k_to_bf16, blocks_for(nw), dim3(256), 0, nullptr, nw, s->W[l], s->W16[l]);
        if (hipMemset(s->mW[l], 0, (size_t)nw * 4) != hipSuccess ||
            hipMemset(s->vW[l], 0, (size_t)nw * 4) != hipSuccess ||
            hipMemset(s->mb[l], 0, (size_t)s->dout[l] * 4) != hipSuccess ||
            hipMemset(s->vb[l], 0, (size_t)s->dout[l] * 4) != hipSuccess)
            ok = false;
    }
    if (!ok || hipDeviceSynchronize() != hipSuccess) {
        surrogate_destroy(s);
        return -2;
    }
    *out = s;
    return 0;
}

void surrogate_destroy(Surrogate *s)
{
    if (!s)
        return;
    hipDeviceSynchronize();
    for (void *p : s->allocs)
        hipFree(p);
    delete s;
}

bool surrogate_ready(const Surrogate *s) { return s && s->scaled; }
int surrogate_max_batch(const Surrogate *s) { return s ? s->bpad : 0; }
int surrogate_layers(const Surrogate *s) { return s ? s->L : 0; }

hipError_t surrogate_downsample(Surrogate *s, int n, const void *u, float *out, hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    const size_t cnt = (size_t)n * s->out;
    if (s->d.precision == 0)
        hipLaunchKernelGGL(k_downsample<float>, blocks_for(cnt), dim3(256), 0, st, n, s->d.n,
                           s->d.out_side, (const float *)u, out);
    else
        hipLaunchKernelGGL(k_downsample<double>, blocks_for(cnt), dim3(256), 0, st, n, s->d.n,
                           s->d.out_side, (const double *)u, out);
    return hipGetLastError();
}

// Box of the sampling coordinates that the network's inputs are mapped to
// [-1, 1] over (the prior box by default).
void surrogate_input_box(Surrogate *s, const double lo[4], const double hi[4])
{
    for (int i = 0; i < 4; ++i) {
        s->d.lo[i] = lo[i];
        s->d.hi[i] = hi[i];
    }
}

hipError_t surrogate_scaling(Surrogate *s, const float *mean, const float *sd, double sigma1,
                             hipStream_t st)
{
    hipError_t e;
    if ((e = hipMemcpyAsync(s->mean, mean, s->out * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(s->sd, sd, s->out * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_ybar, blocks_for(s->out), dim3(256), 0, st, s->d.n, s->d.out_side, s->d.y,
                       s->ybar);
    s->inv_2s2 = 0.5 / (sigma1 * sigma1);
    s->scaled = true;
    return hipGetLastError();
}

// Forward pass of `rows` rows (padded to a multiple of 64); result in s->Y.
static hipError_t forward(Surrogate *s, int rows, const double *phi, hipStream_t st)
{
    const int mp = ((rows + 63) / 64) * 64;
    SurScale sc;
    for (int i = 0; i < 4; ++i) {
        sc.lo[i] = s->d.lo[i];
        sc.hi[i] = s->d.hi[i];
    }
    hipLaunchKernelGGL(k_scale_inputs, blocks_for((size_t)mp * 4), dim3(256), 0, st, rows, mp, phi,
                       sc, s->x0);
    hipLaunchKernelGGL(k_layer0_fwd, blocks_for((size_t)mp * s->dout[0]), dim3(256), 0, st, mp,
                       s->dout[0], s->x0, s->W[0], s->b[0], s->Z[0], s->H[0]);
    hipError_t e = hipGetLastError();
    for (int l = 1; l < s->L && e == hipSuccess; ++l) {
        GemmArgs g{};
        g.A = s->H[l - 1];
        g.B = s->W16[l];
        g.M = mp;
        g.N = s->dout[l];
        g.K = s->din[l];
        g.lda = s->din[l];
        g.ldb = s->din[l];
        g.bias = s->b[l];
        if (l < s->L - 1) {
            g.c32 = s->Z[l];
            g.c16 = s->H[l];
            e = gemm<false, false, kEpiBiasGelu>(g, st);
        } else {
            g.c32 = s->Y;
            e = gemm<false, false, kEpiBias>(g, st);
        }
    }
    return e;
}

hipError_t surrogate_train(Surrogate *s, int batch, const double *phi, const float *target,
                           double lr, double *loss, hipStream_t st)
{
    const int mp = ((batch + 63) / 64) * 64;
    hipError_t e = forward(s, batch, phi, st);
    if (e != hipSuccess)
        return e;
    // dY (layer L-1 output gradient) into buffer 0
    hipLaunchKernelGGL(k_mse_grad, dim3(mp), dim3(256), 0, st, batch, mp, s->out, s->Y, target,
                       s->dz32[0], s->dz16[0], s->row_sse);
    if (loss)
        hipLaunchKernelGGL(k_mean_rows, dim3(1), dim3(256), 0, st, batch, s->out, s->row_sse, loss);
    int cur = 0;
    for (int l = s->L - 1; l >= 1 && e == hipSuccess; --l) {
        // weight gradient: gW[n][k] = sum_r dz[r][n] h[r][k]  (A = dz^T, B = h)
        GemmArgs gw{};
        gw.A = s->dz16[cur];
        gw.B = s->H[l - 1];
        gw.M = s->dout[l];
        gw.N = s->din[l];
        gw.K = mp;
        gw.lda = s->dout[l];
        gw.ldb = s->din[l];
        gw.c32 = s->gW[l];
        if ((e = gemm<true, true, kEpiStore>(gw, st)) != hipSuccess)
            break;
        hipLaunchKernelGGL(k_colsum, dim3((s->dout[l] + 63) / 64), dim3(1024), 0, st, mp, s->dout[l],
                           s->dz32[cur], s->gb[l]);
        // input gradient times GELU'(z_{l-1}): dz_{l-1} = (dz W) .* GELU'(z)
        GemmArgs gi{};
        gi.A = s->dz16[cur];
        gi.B = s->W16[l];
        gi.M = mp;
        gi.N = s->din[l];
        gi.K = s->dout[l];
        gi.lda = s->dout[l];
        gi.ldb = s->din[l];
        gi.zin = s->Z[l - 1];
        gi.c32 = s->dz32[1 - cur];
        gi.c16 = s->dz16[1 - cur];
        if ((e = gemm<false, true, kEpiGeluGrad>(gi, st)) != hipSuccess)
            break;
        cur = 1 - cur;
    }
    if (e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_layer0_wgrad, dim3((s->dout[0] + 63) / 64), dim3(1024), 0, st, mp,
                       s->dout[0], s->x0, s->dz32[cur], s->gW[0]);
    hipLaunchKernelGGL(k_colsum, dim3((s->dout[0] + 63) / 64), dim3(1024), 0, st, mp, s->dout[0],
                       s->dz32[cur], s->gb[0]);
    s->t += 1;
    for (int l = 0; l < s->L; ++l) {
        const int nw = s->din[l] * s->dout[l];
        hipLaunchKernelGGL(k_adam, blocks_for(nw), dim3(256), 0, st, nw, s->W[l], s->gW[l], s->mW[l],
                           s->vW[l], s->W16[l], (float)lr, 0.9f, 0.999f, 1e-8f, s->t);
        hipLaunchKernelGGL(k_adam, blocks_for(s->dout[l]), dim3(256), 0, st, s->dout[l], s->b[l],
                           s->gb[l], s->mb[l], s->vb[l], (bf16 *)nullptr, (float)lr, 0.9f, 0.999f,
                           1e-8f, s->t);
    }
    return hipGetLastError();
}

hipError_t surrogate_predict(Surrogate *s, int n, const double *phi, float *out, int raw,
                             hipStream_t st)
{
    if (n <= 0)
        return hipSuccess;
    hipError_t e = forward(s, n, phi, st);
    if (e != hipSuccess)
        return e;
    if (raw)
        return hipMemcpyAsync(out, s->Y, (size_t)n * s->out * 4, hipMemcpyDeviceToDevice, st);
    hipLaunchKernelGGL(k_destandardise, blocks_for((size_t)n * s->out), dim3(256), 0, st, n, s->out,
                       s->Y, s->mean, s->sd, out);
    return hipGetLastError();
}

int32_t surrogate_enqueue_loglik(Surrogate *s, int n, const double *phi, double *ll, hipStream_t st)
{
    if (n <= 0)
        return 0;
    if (!s->scaled)
        return -1;
    if (forward(s, n, phi, st) != hipSuccess)
        return -2;
    hipLaunchKernelGGL(k_sur_misfit, dim3(n), dim3(256), 0, st, n, s->out, s->Y, s->mean, s->sd,
                       s->ybar, s->inv_2s2, ll);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

hipError_t surrogate_copy_params(Surrogate *s, int layer, float *w, float *b, int dir,
                                 hipStream_t st)
{
    const size_t nw = (size_t)s->din[layer] * s->dout[layer];
    hipError_t e;
    if (dir == 2) {
        if ((e = hipMemcpyAsync(w, s->gW[layer], nw * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return e;
        return hipMemcpyAsync(b, s->gb[layer], s->dout[layer] * 4, hipMemcpyDeviceToDevice, st);
    }
    if (dir == 0) {
        if ((e = hipMemcpyAsync(w, s->W[layer], nw * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess)
            return e;
        return hipMemcpyAsync(b, s->b[layer], s->dout[layer] * 4, hipMemcpyDeviceToDevice, st);
    }
    if ((e = hipMemcpyAsync(s->W[layer], w, nw * 4, hipMemcpyDeviceToDevice, st)) != hipSuccess ||
        (e = hipMemcpyAsync(s->b[layer], b, s->dout[layer] * 4, hipMemcpyDeviceToDevice, st)) !=
            hipSuccess)
        return e;
    hipLaunchKernelGGL(k_to_bf16, blocks_for(nw), dim3(256), 0, st, (int)nw, s->W[layer],
                       s->W16[layer]);
    return hipGetLastError();
}

}  // namespace rd
