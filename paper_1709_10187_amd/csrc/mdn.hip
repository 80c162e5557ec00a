// Mixture-density network of the learned escape surrogate: forward, likelihood, backward
// and Adam on BF16 matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation).
//
// Network: x (16) -> 256 -> 256 -> 256 -> 128, exact (erf) GELU on the hidden layers; the
// 128 outputs parameterise a 16-component mixture over (exit face, y1, y2) (component k:
// logit o[k], face logits o[16+2k+f], mean / log-sigma of y1 at o[48+k] / o[64+k], of y2
// at o[80+k] / o[96+k], correlation 0.95 tanh(o[112+k]); log-sigmas clamped to [-6, 4]).
// The loss is the mean negative log-likelihood of the targets.
//
// Every matrix product is one launch of `gemm`: a block of four waves computes a 64x64 FP32
// tile, 32x32 per wave with 32x32x16 MFMA steps, from 64x32 slices of A and B staged in LDS.
// The slices are read from global memory with 16-byte loads along whichever dimension of the
// operand is contiguous (K for activations and transposed weights, M or N for the operands of
// the weight gradients, which are transposed on their way into LDS), so no operand is copied
// or read element by element.  An epilogue adds the bias, applies GELU or its derivative, and
// stores FP32 and / or BF16.  The weight-gradient products contract over the batch (4096 rows
// for 16 output tiles): they split K over blocks, write FP32 partials, and a second kernel
// adds the partials to the gradient in a fixed order (the result does not depend on timing).
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>

#include <algorithm>

#include "rddmc_internal.h"

namespace rddmc {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ uint16_t f2bf(float f)
{   // round to nearest even
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * erfcf(-z * 0.70710678118654752f); }
__device__ __forceinline__ float gelu_grad(float z)
{
    return 0.5f * erfcf(-z * 0.70710678118654752f) + z * 0.39894228040143268f * __expf(-0.5f * z * z);
}

enum Epilogue : int {
    EP_STORE_F32 = 0,      // C = AB (+ bias)
    EP_GELU = 1,           // Z = AB + bias -> f32 Z, bf16 gelu(Z)
    EP_GELU_BACK = 2,      // dH = AB -> bf16 dH * gelu'(Z)   (Z given, f32)
    EP_ACCUM_F32 = 3,      // C += AB
    EP_PARTIAL = 4,        // P[split] = A[., ks] B[ks, .] (K split over blocks; summed by splitk_add)
};

struct GemmArgs {
    const uint16_t *A;     // bf16, element (m, k) at A[m * sam + k * sak]
    const uint16_t *B;     // bf16, element (k, n) at B[k * sbk + n * sbn]
    int64_t sam, sak, sbk, sbn;
    int M, N, K;           // K a multiple of 16; rows / columns past M / N read as zero
    const float *bias;     // [N] or null
    float *C;              // f32 [M, N] row-major (ldc = N)
    uint16_t *Cb;          // bf16 [M, N] row-major
    const float *Z;        // f32 [M, N] for the GELU derivative
    float *P;              // f32 [splits, M, N] partial products (EP_PARTIAL)
    int mode;
    int splits;            // K ranges (multiples of 32) per output tile; 1 unless EP_PARTIAL
};

constexpr int kTile = 64, kKs = 32, kLdsRow = 40;   // block tile, K slice, padded LDS row (bf16)

// Stage the K slice [k0, k0 + 32) of rows [r0, r0 + 64) of an operand into L[row][k] (bf16,
// rows padded to 40): element (r, k) lives at X[r * sr + k * sk].  K-contiguous operands
// (sk == 1) are read 8 k at a time along a row, row-contiguous ones (sr == 1) 8 rows at a
// time along a k, anything else element by element; out-of-range elements read as zero.
__device__ __forceinline__ void stage(uint16_t *__restrict__ L, const uint16_t *__restrict__ X, int64_t sr,
                                      int64_t sk, int rows, int K, int r0, int k0, int t)
{
    if (sk == 1) {
        const int r = t >> 2, c = (t & 3) << 3;
        uint4 v = make_uint4(0u, 0u, 0u, 0u);
        const int gr = r0 + r, gk = k0 + c;
        if (gr < rows && gk + 8 <= K) {
            v = *reinterpret_cast<const uint4 *>(X + (int64_t)gr * sr + gk);
        } else if (gr < rows) {
            uint16_t h[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) h[e] = gk + e < K ? X[(int64_t)gr * sr + gk + e] : (uint16_t)0;
            v = make_uint4(h[0] | ((uint32_t)h[1] << 16), h[2] | ((uint32_t)h[3] << 16), h[4] | ((uint32_t)h[5] << 16),
                           h[6] | ((uint32_t)h[7] << 16));
        }
        *reinterpret_cast<uint4 *>(L + r * kLdsRow + c) = v;
    } else if (sr == 1) {
        const int kk = t >> 3, c = (t & 7) << 3;
        const int gk = k0 + kk, gr = r0 + c;
        uint16_t h[8];
        if (gk < K && gr + 8 <= rows) {
            const uint4 v = *reinterpret_cast<const uint4 *>(X + (int64_t)gk * sk + gr);
            h[0] = (uint16_t)v.x; h[1] = (uint16_t)(v.x >> 16); h[2] = (uint16_t)v.y; h[3] = (uint16_t)(v.y >> 16);
            h[4] = (uint16_t)v.z; h[5] = (uint16_t)(v.z >> 16); h[6] = (uint16_t)v.w; h[7] = (uint16_t)(v.w >> 16);
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) h[e] = (gk < K && gr + e < rows) ? X[(int64_t)gk * sk + gr + e] : (uint16_t)0;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e) L[(c + e) * kLdsRow + kk] = h[e];
    } else {
        for (int q = t; q < kTile * kKs; q += 256) {
            const int r = q / kKs, kk = q % kKs;
            const int gr = r0 + r, gk = k0 + kk;
            L[r * kLdsRow + kk] = (gr < rows && gk < K) ? X[(int64_t)gr * sr + (int64_t)gk * sk] : (uint16_t)0;
        }
    }
}

// Block (tile_m, tile_n, split) of 256 lanes: wave w owns rows m0 + 32 (w >> 1), columns
// n0 + 32 (w & 1).  Lane l supplies A row (l % 32), k-slice [(l / 32) * 8, +8) of each 16-deep
// step from LDS, likewise B column (l % 32); its 16 accumulators hold rows
// 8 (r / 4) + 4 (l / 32) + (r % 4) of the wave's sub-tile, column l % 32.
__global__ __launch_bounds__(256) void gemm(GemmArgs g)
{
    __shared__ __attribute__((aligned(16))) uint16_t As[kTile * kLdsRow];
    __shared__ __attribute__((aligned(16))) uint16_t Bs[kTile * kLdsRow];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int tiles_n = (g.N + kTile - 1) / kTile, tiles_m = (g.M + kTile - 1) / kTile;
    const int tile = blockIdx.x % (tiles_m * tiles_n), split = blockIdx.x / (tiles_m * tiles_n);
    const int m0 = (tile / tiles_n) * kTile, n0 = (tile % tiles_n) * kTile;
    // this block's K range: whole slices, the last split takes the remainder
    const int nks = (g.K + kKs - 1) / kKs;
    const int per = (nks + g.splits - 1) / g.splits;
    const int ks_lo = split * per, ks_hi = min(nks, ks_lo + per);
    const int r32 = lane & 31, kh = (lane >> 5) << 3;
    const int wm = (w >> 1) << 5, wn = (w & 1) << 5;
    f32x16 acc;
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[i] = 0.0f;
    for (int ks = ks_lo; ks < ks_hi; ++ks) {
        const int k0 = ks * kKs;
        // A rows are M, B "rows" are N with element (n, k) at B[n * sbn + k * sbk]
        stage(As, g.A, g.sam, g.sak, g.M, g.K, m0, k0, t);
        stage(Bs, g.B, g.sbn, g.sbk, g.N, g.K, n0, k0, t);
        __syncthreads();
#pragma unroll
        for (int h = 0; h < kKs; h += 16) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(As + (wm + r32) * kLdsRow + h + kh);
            const bf16x8 b = *reinterpret_cast<const bf16x8 *>(Bs + (wn + r32) * kLdsRow + h + kh);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
        }
        __syncthreads();
    }
    const int col = n0 + wn + r32;
    if (col >= g.N) return;
    if (g.mode == EP_PARTIAL) {
        float *P = g.P + (int64_t)split * g.M * g.N;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = m0 + wm + ((r >> 2) << 3) + ((lane >> 5) << 2) + (r & 3);
            if (row < g.M) P[(int64_t)row * g.N + col] = acc[r];
        }
        return;
    }
    const float bv = g.bias ? g.bias[col] : 0.0f;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int row = m0 + wm + ((r >> 2) << 3) + ((lane >> 5) << 2) + (r & 3);
        if (row >= g.M) continue;
        const int64_t o = (int64_t)row * g.N + col;
        const float v = acc[r] + bv;
        if (g.mode == EP_STORE_F32) {
            if (g.C) g.C[o] = v;
            if (g.Cb) g.Cb[o] = f2bf(v);
        } else if (g.mode == EP_GELU) {
            g.C[o] = v;
            g.Cb[o] = f2bf(gelu(v));
        } else if (g.mode == EP_GELU_BACK) {
            g.Cb[o] = f2bf(v * gelu_grad(g.Z[o]));
        } else {
            g.C[o] += v;
        }
    }
}

// C[i] += sum over splits of P[split][i], splits in order.
__global__ void splitk_add(const float *__restrict__ P, int splits, int64_t n, float *__restrict__ C)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float v = 0.0f;
    for (int q = 0; q < splits; ++q) v += P[(int64_t)q * n + i];
    C[i] += v;
}

// ---- parameter layout ---------------------------------------------------------------
constexpr int kIn = 16, kHid = 256, kOut = 128, kComp = 16;
constexpr int kMaxSplits = 16;     // K splits of a weight-gradient product
constexpr int64_t kW1 = 0, kB1 = kW1 + kIn * kHid, kW2 = kB1 + kHid, kB2 = kW2 + kHid * kHid, kW3 = kB2 + kHid,
                  kB3 = kW3 + kHid * kHid, kW4 = kB3 + kHid, kB4 = kW4 + kHid * kOut, kNParams = kB4 + kOut;
constexpr int64_t kLayerW[4] = {kW1, kW2, kW3, kW4};
constexpr int64_t kLayerB[4] = {kB1, kB2, kB3, kB4};
constexpr int kLayerIn[4] = {kIn, kHid, kHid, kHid};
constexpr int kLayerOut[4] = {kHid, kHid, kHid, kOut};

// Parameter buffer: f32 theta, Adam m, Adam v, grad (kNParams each), then bf16 copies of
// every W ([in, out]) and of its transpose ([out, in]).
struct ParamView {
    float *theta, *m, *v, *grad;
    uint16_t *w, *wt;     // bf16, kNParams entries each (bias slots unused)
};

__host__ __device__ inline ParamView param_view(void *base)
{
    ParamView p;
    float *f = static_cast<float *>(base);
    p.theta = f;
    p.m = f + kNParams;
    p.v = f + 2 * kNParams;
    p.grad = f + 3 * kNParams;
    p.w = reinterpret_cast<uint16_t *>(f + 4 * kNParams);
    p.wt = p.w + kNParams;
    return p;
}
constexpr uint64_t kParamBytes = 4ull * 4 * kNParams + 2ull * 2 * kNParams;

// Work buffer for a batch of up to `cap` samples (cap a multiple of 32).
struct WorkView {
    uint16_t *xb;                  // [cap, 16]
    float *z[3];                   // [cap, 256]
    uint16_t *h[3];                // [cap, 256]
    float *o;                      // [cap, 128]
    uint16_t *dout;                // [cap, 128]
    uint16_t *dz[2];               // [cap, 256] ping-pong
    float *part;                   // [kMaxSplits, 256, 256] split-K partials of a weight gradient
    float *loss;                   // [1]
};

__host__ __device__ inline WorkView work_view(void *base, int64_t cap)
{
    WorkView w;
    uint8_t *p = static_cast<uint8_t *>(base);
    auto take = [&](uint64_t bytes) {
        uint8_t *q = p;
        p += (bytes + 255) & ~255ull;
        return q;
    };
    w.xb = reinterpret_cast<uint16_t *>(take(2ull * cap * kIn));
    for (int l = 0; l < 3; ++l) w.z[l] = reinterpret_cast<float *>(take(4ull * cap * kHid));
    for (int l = 0; l < 3; ++l) w.h[l] = reinterpret_cast<uint16_t *>(take(2ull * cap * kHid));
    w.o = reinterpret_cast<float *>(take(4ull * cap * kOut));
    w.dout = reinterpret_cast<uint16_t *>(take(2ull * cap * kOut));
    for (int l = 0; l < 2; ++l) w.dz[l] = reinterpret_cast<uint16_t *>(take(2ull * cap * kHid));
    w.part = reinterpret_cast<float *>(take(4ull * kMaxSplits * kHid * kHid));
    w.loss = reinterpret_cast<float *>(take(256));
    return w;
}

__host__ inline uint64_t work_bytes_for(int64_t cap)
{
    WorkView w = work_view(nullptr, cap);
    return reinterpret_cast<uint64_t>(w.loss) + 256;
}

// ---- small kernels --------------------------------------------------------------------
// bf16 copy of n values, zero up to n_pad
__global__ void to_bf16_padded(const float *x, uint16_t *y, int64_t n, int64_t n_pad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n_pad) y[i] = i < n ? f2bf(x[i]) : (uint16_t)0;
}

// bf16 copies of every weight matrix and its transpose
__global__ void refresh_bf16(ParamView p)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    for (int l = 0; l < 4; ++l) {
        const int64_t w0 = kLayerW[l], n = (int64_t)kLayerIn[l] * kLayerOut[l];
        if (i >= w0 && i < w0 + n) {
            const int64_t r = (i - w0) / kLayerOut[l], c = (i - w0) % kLayerOut[l];
            const uint16_t b = f2bf(p.theta[i]);
            p.w[i] = b;
            p.wt[w0 + c * kLayerIn[l] + r] = b;
        }
    }
}

__global__ void zero_f32(float *x, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0f;
}

// Glorot-uniform weights and zero biases from a Philox-free hash of (seed, index): the
// initial point only needs to be reproducible.
__global__ void init_params(ParamView p, uint64_t seed)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    float val = 0.0f;
    for (int l = 0; l < 4; ++l) {
        const int64_t w0 = kLayerW[l], n = (int64_t)kLayerIn[l] * kLayerOut[l];
        if (i >= w0 && i < w0 + n) {
            uint64_t z = seed * 0x9E3779B97F4A7C15ull + (uint64_t)i * 0xD1B54A32D192ED03ull + 0x632BE59BD9B4E019ull;
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            z ^= z >> 31;
            const float u = ((float)(z >> 40) + 0.5f) * 5.9604644775390625e-8f;
            const float lim = sqrtf(6.0f / (float)(kLayerIn[l] + kLayerOut[l]));
            val = (2.0f * u - 1.0f) * lim;
        }
    }
    p.theta[i] = val;
    p.m[i] = 0.0f;
    p.v[i] = 0.0f;
    p.grad[i] = 0.0f;
}

// Mixture likelihood of one sample and d(mean NLL)/d(o) (stored bf16, scaled by 1/n).
__global__ void nll_kernel(const float *__restrict__ o, const float *__restrict__ y, int n, int n_pad,
                           uint16_t *__restrict__ dout, float *__restrict__ loss_sum)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n_pad) return;
    uint16_t *g = dout + (int64_t)i * kOut;
    if (i >= n) {   // padding rows contribute nothing
        for (int c = 0; c < kOut; ++c) g[c] = 0;
        return;
    }
    const float *q = o + (int64_t)i * kOut;
    const int f = (int)y[3 * i];
    const float y1 = y[3 * i + 1], y2 = y[3 * i + 2];
    float lc[kComp];
    float amax = -INFINITY;
    for (int k = 0; k < kComp; ++k) amax = fmaxf(amax, q[k]);
    float asum = 0.0f;
    for (int k = 0; k < kComp; ++k) asum += __expf(q[k] - amax);
    const float log_asum = amax + __logf(asum);
    float lmax = -INFINITY;
    for (int k = 0; k < kComp; ++k) {
        const float f0 = q[16 + 2 * k], f1 = q[17 + 2 * k];
        const float fm = fmaxf(f0, f1);
        const float lse_f = fm + __logf(__expf(f0 - fm) + __expf(f1 - fm));
        const float s1 = fminf(fmaxf(q[64 + k], -6.0f), 4.0f), s2 = fminf(fmaxf(q[96 + k], -6.0f), 4.0f);
        const float rho = 0.95f * tanhf(q[112 + k]);
        const float z1 = (y1 - q[48 + k]) * __expf(-s1), z2 = (y2 - q[80 + k]) * __expf(-s2);
        const float om = 1.0f - rho * rho;
        const float qq = (z1 * z1 - 2.0f * rho * z1 * z2 + z2 * z2) / om;
        lc[k] = (q[k] - log_asum) + ((f ? f1 : f0) - lse_f) +
                (-1.8378770664093453f - s1 - s2 - 0.5f * __logf(om) - 0.5f * qq);
        lmax = fmaxf(lmax, lc[k]);
    }
    float lsum = 0.0f;
    for (int k = 0; k < kComp; ++k) lsum += __expf(lc[k] - lmax);
    const float ll = lmax + __logf(lsum);
    atomicAdd(loss_sum, -ll / (float)n);      // the mean NLL
    const float inv_n = 1.0f / (float)n;
    for (int k = 0; k < kComp; ++k) {
        const float w = __expf(lc[k] - ll);
        const float pi = __expf(q[k] - log_asum);
        g[k] = f2bf((pi - w) * inv_n);
        const float f0 = q[16 + 2 * k], f1 = q[17 + 2 * k];
        const float fm = fmaxf(f0, f1);
        const float e0 = __expf(f0 - fm), e1 = __expf(f1 - fm);
        const float p0 = e0 / (e0 + e1), p1 = e1 / (e0 + e1);
        g[16 + 2 * k] = f2bf(w * (p0 - (f == 0 ? 1.0f : 0.0f)) * inv_n);
        g[17 + 2 * k] = f2bf(w * (p1 - (f == 1 ? 1.0f : 0.0f)) * inv_n);
        const float s1r = q[64 + k], s2r = q[96 + k];
        const float s1 = fminf(fmaxf(s1r, -6.0f), 4.0f), s2 = fminf(fmaxf(s2r, -6.0f), 4.0f);
        const float rr = tanhf(q[112 + k]);
        const float rho = 0.95f * rr;
        const float e1s = __expf(-s1), e2s = __expf(-s2);
        const float z1 = (y1 - q[48 + k]) * e1s, z2 = (y2 - q[80 + k]) * e2s;
        const float om = 1.0f - rho * rho;
        const float dq1 = (2.0f * z1 - 2.0f * rho * z2) / om, dq2 = (2.0f * z2 - 2.0f * rho * z1) / om;
        const float qq = (z1 * z1 - 2.0f * rho * z1 * z2 + z2 * z2) / om;
        const float dqr = (-2.0f * z1 * z2) / om + qq * (2.0f * rho) / om;
        const float in1 = (s1r > -6.0f && s1r < 4.0f) ? 1.0f : 0.0f;
        const float in2 = (s2r > -6.0f && s2r < 4.0f) ? 1.0f : 0.0f;
        g[48 + k] = f2bf(-w * 0.5f * dq1 * e1s * inv_n);
        g[64 + k] = f2bf(-w * (-1.0f + 0.5f * dq1 * z1) * in1 * inv_n);
        g[80 + k] = f2bf(-w * 0.5f * dq2 * e2s * inv_n);
        g[96 + k] = f2bf(-w * (-1.0f + 0.5f * dq2 * z2) * in2 * inv_n);
        g[112 + k] = f2bf(-w * (rho / om - 0.5f * dqr) * 0.95f * (1.0f - rr * rr) * inv_n);
    }
}

// column sums of a bf16 [M, N] matrix, added into out[N]
// Column sums of a bf16 [M, N] matrix in two passes: block (column chunk of 64, row chunk of
// `rows`) has 4 lanes per column each summing a quarter of the chunk's rows, reduced in LDS
// to partial[row chunk][column]; colsum_finish adds the row chunks' partials to out in order.
// At most kMaxSplits * kHid * kHid / N row chunks (the partial buffer), of at least 256 rows.
__global__ __launch_bounds__(256) void colsum_partial(const uint16_t *__restrict__ d, int M, int N, int rows,
                                                     float *__restrict__ part)
{
    __shared__ float red[4][64];
    const int cl = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int c = blockIdx.x * 64 + cl;
    const int r0 = blockIdx.y * rows;
    float s = 0.0f;
    if (c < N)
        for (int r = r0 + g; r < min(M, r0 + rows); r += 4) s += bf2f(d[(int64_t)r * N + c]);
    red[g][cl] = s;
    __syncthreads();
    if (g == 0 && c < N) part[(int64_t)blockIdx.y * N + c] = ((red[0][cl] + red[1][cl]) + red[2][cl]) + red[3][cl];
}

__global__ void colsum_finish(const float *__restrict__ part, int chunks, int N, float *__restrict__ out)
{
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= N) return;
    float s = 0.0f;
    for (int q = 0; q < chunks; ++q) s += part[(int64_t)q * N + c];
    out[c] += s;
}

__global__ void adam_kernel(ParamView p, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kNParams) return;
    const float g = p.grad[i];
    const float m = b1 * p.m[i] + (1.0f - b1) * g;
    const float v = b2 * p.v[i] + (1.0f - b2) * g * g;
    p.m[i] = m;
    p.v[i] = v;
    p.theta[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

// ---- host orchestration -----------------------------------------------------------------
hipError_t launch_gemm(const GemmArgs &g, hipStream_t s)
{
    const int tiles = ((g.M + kTile - 1) / kTile) * ((g.N + kTile - 1) / kTile);
    gemm<<<(unsigned)(tiles * g.splits), 256, 0, s>>>(g);
    if (g.mode == EP_PARTIAL) {
        const int64_t n = (int64_t)g.M * g.N;
        splitk_add<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(g.P, g.splits, n, g.C);
    }
    return hipGetLastError();
}

GemmArgs gemm_args(const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk, int64_t sbn, int M,
                   int N, int K)
{
    GemmArgs g{};
    g.A = A;
    g.sam = sam;
    g.sak = sak;
    g.B = B;
    g.sbk = sbk;
    g.sbn = sbn;
    g.M = M;
    g.N = N;
    g.K = K;
    g.splits = 1;
    return g;
}

// forward of `mp` (multiple of 32) rows whose bf16 inputs are in w.xb
hipError_t forward(const ParamView &p, const WorkView &w, int mp, hipStream_t s)
{
    hipError_t e;
    const uint16_t *in = w.xb;
    for (int l = 0; l < 4; ++l) {
        const int K = kLayerIn[l], N = kLayerOut[l];
        // B = W [K, N]: element (k, n) read from the transposed copy at n * K + k
        GemmArgs g = gemm_args(in, K, 1, p.wt + kLayerW[l], 1, K, mp, N, K);
        g.bias = p.theta + kLayerB[l];
        if (l < 3) {
            g.mode = EP_GELU;
            g.C = w.z[l];
            g.Cb = w.h[l];
            in = w.h[l];
        } else {
            g.mode = EP_STORE_F32;
            g.C = w.o;
        }
        if ((e = launch_gemm(g, s)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// loss and gradient (into p.grad, overwritten) of n samples (padded to mp rows)
hipError_t loss_grad(const ParamView &p, const WorkView &w, const float *d_x, const float *d_y, int n, int mp,
                     hipStream_t s)
{
    hipError_t e;
    to_bf16_padded<<<(unsigned)(((int64_t)mp * kIn + 255) / 256), 256, 0, s>>>(d_x, w.xb, (int64_t)n * kIn,
                                                                             (int64_t)mp * kIn);
    if ((e = forward(p, w, mp, s)) != hipSuccess) return e;
    zero_f32<<<1, 64, 0, s>>>(w.loss, 1);
    zero_f32<<<(unsigned)((kNParams + 255) / 256), 256, 0, s>>>(p.grad, kNParams);
    nll_kernel<<<(unsigned)((mp + 127) / 128), 128, 0, s>>>(w.o, d_y, n, mp, w.dout, w.loss);
    // layer 4: dW4 = h3^T dout, db4 = colsum(dout), dz3 = (dout W4^T) * gelu'(z3)
    const uint16_t *dcur = w.dout;
    int dn = kOut;
    int pp = 0;
    for (int l = 3; l >= 0; --l) {
        const int K = kLayerIn[l], N = kLayerOut[l];
        const uint16_t *hin = l > 0 ? w.h[l - 1] : w.xb;
        // dW[K, N] += hin^T (K x mp) * dcur (mp x N)
        GemmArgs gw = gemm_args(hin, 1, K, dcur, dn, 1, K, N, mp);
        gw.mode = EP_PARTIAL;
        gw.splits = std::max(1, std::min(kMaxSplits, mp / 256));
        gw.P = w.part;
        gw.C = p.grad + kLayerW[l];
        if ((e = launch_gemm(gw, s)) != hipSuccess) return e;
        {
            const int max_chunks = (int)(kMaxSplits * kHid * kHid / N);
            const int rows = std::max(256, (mp + max_chunks - 1) / max_chunks);
            const int chunks = (mp + rows - 1) / rows;
            colsum_partial<<<dim3((N + 63) / 64, chunks), 256, 0, s>>>(dcur, mp, N, rows, w.part);
            colsum_finish<<<(N + 127) / 128, 128, 0, s>>>(w.part, chunks, N, p.grad + kLayerB[l]);
        }
        if (l == 0) break;
        // dz_{l-1}[mp, K] = (dcur [mp, N] * W^T [N, K]) * gelu'(z_{l-1}); B element (o, i) = W[i, o]
        GemmArgs gd = gemm_args(dcur, dn, 1, p.w + kLayerW[l], 1, N, mp, K, N);
        gd.mode = EP_GELU_BACK;
        gd.Z = w.z[l - 1];
        gd.Cb = w.dz[pp];
        if ((e = launch_gemm(gd, s)) != hipSuccess) return e;
        dcur = w.dz[pp];
        dn = K;
        pp ^= 1;
    }
    return hipGetLastError();
}

}  // namespace

uint64_t mdn_param_bytes() { return kParamBytes; }
uint64_t mdn_work_bytes(int64_t cap) { return work_bytes_for(cap); }
int64_t mdn_n_params() { return kNParams; }

hipError_t mdn_init(void *d_params, uint64_t seed, hipStream_t s)
{
    ParamView p = param_view(d_params);
    init_params<<<(unsigned)((kNParams + 255) / 256), 256, 0, s>>>(p, seed);
    refresh_bf16<<<(unsigned)((kNParams + 255) / 256), 256, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t mdn_refresh(void *d_params, hipStream_t s)
{
    ParamView p = param_view(d_params);
    refresh_bf16<<<(unsigned)((kNParams + 255) / 256), 256, 0, s>>>(p);
    return hipGetLastError();
}

hipError_t mdn_forward(void *d_params, void *d_work, int64_t cap, const float *d_x, int n, float *d_out,
                       hipStream_t s)
{
    ParamView p = param_view(d_params);
    WorkView w = work_view(d_work, cap);
    const int mp = (n + 31) & ~31;
    hipError_t e;
    to_bf16_padded<<<(unsigned)(((int64_t)mp * kIn + 255) / 256), 256, 0, s>>>(d_x, w.xb, (int64_t)n * kIn,
                                                                             (int64_t)mp * kIn);
    if ((e = forward(p, w, mp, s)) != hipSuccess) return e;
    if (d_out && (e = hipMemcpyAsync(d_out, w.o, 4ull * n * kOut, hipMemcpyDeviceToDevice, s)) != hipSuccess)
        return e;
    return hipGetLastError();
}

hipError_t mdn_loss_grad(void *d_params, void *d_work, int64_t cap, const float *d_x, const float *d_y, int n,
                         float *d_loss, hipStream_t s)
{
    ParamView p = param_view(d_params);
    WorkView w = work_view(d_work, cap);
    const int mp = (n + 31) & ~31;
    hipError_t e = loss_grad(p, w, d_x, d_y, n, mp, s);
    if (e != hipSuccess) return e;
    if (d_loss && (e = hipMemcpyAsync(d_loss, w.loss, 4, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    return hipGetLastError();
}

hipError_t mdn_adam(void *d_params, int64_t step, float lr, hipStream_t s)
{
    ParamView p = param_view(d_params);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    adam_kernel<<<(unsigned)((kNParams + 255) / 256), 256, 0, s>>>(p, lr, b1, b2, eps, c1, c2);
    refresh_bf16<<<(unsigned)((kNParams + 255) / 256), 256, 0, s>>>(p);
    return hipGetLastError();
}

// raw network outputs of the current batch (work buffer), for the surrogate table kernel
const float *mdn_outputs(void *d_work, int64_t cap) { return work_view(d_work, cap).o; }

}  // namespace rddmc
