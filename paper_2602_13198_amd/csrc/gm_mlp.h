// gm_mlp.h -- the small network of the learned form: 6 -> 64 -> 64 -> 2
// with tanh hidden layers, evaluated and trained with matrix-core (MFMA)
// instructions: BF16 operands, FP32 accumulation, FP32 master weights.
//
// Every wave owns a tile of 16 rows.  Each layer is a set of 16x16x16 BF16
// MFMAs (v_mfma_f32_16x16x16_bf16); between layers the activations go
// through LDS to turn the accumulator layout into the operand layout.  The
// backward pass forms the weight gradients H^T dZ with the 16 rows of the
// tile as the MFMA reduction dimension.  Within a block each gradient entry
// receives exactly one addition per wave (two waves) onto zero, and IEEE
// addition is commutative, so the block's partial does not depend on the
// order of the waves' LDS atomics; blocks write their partials, which a
// second kernel sums in a fixed order, so the gradient is deterministic; in
// a training step that kernel then applies the Adam step to the FP32 weights
// and refreshes their BF16 copies.
//
// Operand layouts of the 16x16x16 BF16 MFMA (lane l, element j = 0..3):
//   A (16 x K16):  row l % 16, k = 4 (l / 16) + j
//   B (K16 x 16):  col l % 16, k = 4 (l / 16) + j
//   D (16 x 16):   col l % 16, row 4 (l / 16) + j
#pragma once

#include "gm_common.h"

namespace gm {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kMlpIn = 6, kMlpH = 64, kMlpOut = 2;
constexpr int kMlpXStride = 8;            // floats per input row (6 features, 2 pad)
// parameter offsets in the FP32 master vector
constexpr int kW1 = 0;                          // [6][64]
constexpr int kB1 = kW1 + kMlpIn * kMlpH;       // [64]
constexpr int kW2 = kB1 + kMlpH;                // [64][64]
constexpr int kB2 = kW2 + kMlpH * kMlpH;        // [64]
constexpr int kW3 = kB2 + kMlpH;                // [64][2]
constexpr int kB3 = kW3 + kMlpH * kMlpOut;      // [2]
constexpr int kMlpParams = kB3 + kMlpOut;       // 4738
// BF16 copies, zero-padded to MFMA shapes
constexpr int kW1b = 0;                         // [16][64]  (k = feature)
constexpr int kW2b = kW1b + 16 * kMlpH;         // [64][64]
constexpr int kW3b = kW2b + kMlpH * kMlpH;      // [64][16]  (n = output)
constexpr int kMlpBf16 = kW3b + kMlpH * 16;

constexpr int kMlpWaves = 4;                    // waves (tiles of 16 rows) per inference block
constexpr int kMlpGradWaves = 2;                // per training block (LDS: 4 tiles per wave)
constexpr int kMlpGradRows = 16 * kMlpGradWaves;

GM_D short f2bf(float x)
{
    // round to nearest even
    uint32_t u = __float_as_uint(x);
    uint32_t r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (short)(r >> 16);
}

GM_D f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

struct MlpArgs {
    const float *X;        // [n][8]
    const float *T;        // [n][2] targets (training)
    const float *C;        // [n][2] loss weights (training)
    float *Y;              // [n][2] outputs (inference)
    long long n;
    const float *P;        // FP32 master parameters
    const short *Pb;       // BF16 padded weights
    float *gpart;          // [n_blocks][kMlpParams + 1] partial gradients (+ loss)
    float loss_scale;      // 1 / sum of the loss weights
    int loss_kind;         // 0: C (y - T)^2; 1: log-link Poisson deviance C (e^y - T y)
};

// Per-wave LDS scratch: a 16 x 64 tile (+1 pad column) of floats.
constexpr int kTileLd = 65;

GM_D void tile_store_D(float *t, int col0, f32x4 d)
{
    int l = lane_id();
#pragma unroll
    for (int j = 0; j < 4; ++j) t[(4 * (l >> 4) + j) * kTileLd + col0 + (l & 15)] = d[j];
}

// A operand (rows of the tile, k block kb of the 64 columns)
GM_D bf16x4 tile_load_A(const float *t, int kb)
{
    int l = lane_id();
    bf16x4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = f2bf(t[(l & 15) * kTileLd + 16 * kb + 4 * (l >> 4) + j]);
    return a;
}

// A operand of the transposed tile: rows = columns c0.. of the tile, k = tile rows
GM_D bf16x4 tile_load_AT(const float *t, int c0)
{
    int l = lane_id();
    bf16x4 a;
#pragma unroll
    for (int j = 0; j < 4; ++j) a[j] = f2bf(t[(4 * (l >> 4) + j) * kTileLd + c0 + (l & 15)]);
    return a;
}

// B operand from a tile with k = tile rows, n = columns c0..
GM_D bf16x4 tile_load_B(const float *t, int c0)
{
    int l = lane_id();
    bf16x4 b;
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = f2bf(t[(4 * (l >> 4) + j) * kTileLd + c0 + (l & 15)]);
    return b;
}

// B operand from a BF16 weight matrix W[k][n] with leading dimension ld
GM_D bf16x4 w_load_B(const short *W, int ld, int k0, int n0)
{
    int l = lane_id();
    bf16x4 b;
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = W[(k0 + 4 * (l >> 4) + j) * ld + n0 + (l & 15)];
    return b;
}

// B operand from the transpose of W[n][k] (ld = row length of W)
GM_D bf16x4 w_load_BT(const short *W, int ld, int k0, int n0)
{
    int l = lane_id();
    bf16x4 b;
#pragma unroll
    for (int j = 0; j < 4; ++j) b[j] = W[(n0 + (l & 15)) * ld + k0 + 4 * (l >> 4) + j];
    return b;
}

// Forward pass of one 16-row tile whose input features come from
// feat(row, k) (k < kMlpIn, row < n); leaves H1 and H2 (post-tanh) in LDS
// tiles h1, h2 and returns the output accumulator (cols 0, 1 valid).
template <class Feat>
GM_D f32x4 mlp_tile_forward_f(const MlpArgs &M, long long r0, float *h1, float *h2, Feat feat)
{
    const int l = lane_id();
    // layer 1: X [16 x 16 (6 used)] x W1 [16 x 64]
    bf16x4 ax;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        int k = 4 * (l >> 4) + j;
        long long r = r0 + (l & 15);
        float v = (k < kMlpIn && r < M.n) ? feat(r, k) : 0.0f;
        ax[j] = f2bf(v);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
        d = mfma16(ax, w_load_B(M.Pb + kW1b, kMlpH, 0, 16 * t), d);
        float bias = M.P[kB1 + 16 * t + (l & 15)];
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = tanhf(d[j] + bias);
        tile_store_D(h1, 16 * t, d);
    }
    __builtin_amdgcn_wave_barrier();
    // layer 2: H1 [16 x 64] x W2 [64 x 64]
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int s = 0; s < 4; ++s) d = mfma16(tile_load_A(h1, s), w_load_B(M.Pb + kW2b, kMlpH, 16 * s, 16 * t), d);
        float bias = M.P[kB2 + 16 * t + (l & 15)];
#pragma unroll
        for (int j = 0; j < 4; ++j) d[j] = tanhf(d[j] + bias);
        tile_store_D(h2, 16 * t, d);
    }
    __builtin_amdgcn_wave_barrier();
    // layer 3: H2 [16 x 64] x W3 [64 x 16 (2 used)]
    f32x4 y = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int s = 0; s < 4; ++s) y = mfma16(tile_load_A(h2, s), w_load_B(M.Pb + kW3b, 16, 16 * s, 0), y);
    float bias = (l & 15) < kMlpOut ? M.P[kB3 + (l & 15)] : 0.0f;
#pragma unroll
    for (int j = 0; j < 4; ++j) y[j] += bias;
    return y;
}

GM_D f32x4 mlp_tile_forward(const MlpArgs &M, long long r0, float *h1, float *h2)
{
    return mlp_tile_forward_f(M, r0, h1, h2, [&](long long r, int k) { return M.X[r * kMlpXStride + k]; });
}

__global__ __launch_bounds__(64 * kMlpWaves) void mlp_forward_kernel(MlpArgs M)
{
    __shared__ float lds[kMlpWaves][2][16 * kTileLd];
    const int w = threadIdx.x >> 6, l = lane_id();
    const long long r0 = ((long long)blockIdx.x * kMlpWaves + w) * 16;
    if (r0 >= M.n) return;                       // whole wave idle: no barrier below is block-wide
    f32x4 y = mlp_tile_forward(M, r0, lds[w][0], lds[w][1]);
    const int n = l & 15;
    if (n < kMlpOut) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            long long r = r0 + 4 * (l >> 4) + j;
            if (r < M.n) M.Y[r * kMlpOut + n] = y[j];
        }
    }
}

// Forward + backward of a weighted loss over the rows of this block,
//   L = loss_scale * sum_rows sum_o C[r][o] l(y[r][o], T[r][o]),
// l = (y - T)^2 or the Poisson deviance e^y - T y (minimised by
// y = ln E[T], also for targets that are mostly zero); writes the block's
// partial gradient and loss to gpart[block].
__global__ __launch_bounds__(64 * kMlpGradWaves) void mlp_grad_kernel(MlpArgs M)
{
    __shared__ float lds[kMlpGradWaves][4][16 * kTileLd];    // h1, h2, dz2, dz1 per wave
    __shared__ float gacc[kMlpParams + 1];
    for (int i = threadIdx.x; i < kMlpParams + 1; i += blockDim.x) gacc[i] = 0.0f;
    __syncthreads();
    const int w = threadIdx.x >> 6, l = lane_id();
    const long long r0 = ((long long)blockIdx.x * kMlpGradWaves + w) * 16;
    float *h1 = lds[w][0], *h2 = lds[w][1], *dz2 = lds[w][2], *dz1 = lds[w][3];
    if (r0 < M.n) {
        f32x4 y = mlp_tile_forward(M, r0, h1, h2);
        // dL/dy in accumulator layout (col n = output, row = tile row); rows
        // past the end have zero weight
        const int n = l & 15;
        f32x4 dy = {0.0f, 0.0f, 0.0f, 0.0f};
        float lsum = 0.0f;
        if (n < kMlpOut) {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                long long r = r0 + 4 * (l >> 4) + j;
                if (r < M.n) {
                    const float c = M.C[r * kMlpOut + n], t = M.T[r * kMlpOut + n];
                    if (M.loss_kind == 1) {
                        const float ey = expf(y[j]);
                        dy[j] = M.loss_scale * c * (ey - t);
                        lsum += M.loss_scale * c * (ey - t * y[j]);
                    } else {
                        const float e = y[j] - t;
                        dy[j] = 2.0f * M.loss_scale * c * e;
                        lsum += M.loss_scale * c * e * e;
                    }
                }
            }
        }
        // dy through LDS (the dz1 tile is free until later)
        tile_store_D(dz1, 0, dy);
        __builtin_amdgcn_wave_barrier();
        // dW3 [64 x 16] = H2^T [64 x 16 rows] dY [16 rows x 16]
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f32x4 g = {0.0f, 0.0f, 0.0f, 0.0f};
            g = mfma16(tile_load_AT(h2, 16 * mt), tile_load_B(dz1, 0), g);
            if (n < kMlpOut) {
#pragma unroll
                for (int j = 0; j < 4; ++j) atomicAdd(&gacc[kW3 + (16 * mt + 4 * (l >> 4) + j) * kMlpOut + n], g[j]);
            }
        }
        {
            // db3: the wave's four row groups summed by shuffles in a fixed
            // order, then one addition per wave
            float s = dy[0] + dy[1] + dy[2] + dy[3];
            s += __shfl_xor(s, 16);
            s += __shfl_xor(s, 32);
            if (l < kMlpOut) atomicAdd(&gacc[kB3 + l], s);
        }
        // dH2 [16 x 64] = dY [16 x 16] W3^T [16 x 64]; dZ2 = dH2 (1 - h2^2)
        bf16x4 ady = tile_load_A(dz1, 0);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
            d = mfma16(ady, w_load_BT(M.Pb + kW3b, 16, 0, 16 * t), d);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float hv = h2[(4 * (l >> 4) + j) * kTileLd + 16 * t + n];
                d[j] *= 1.0f - hv * hv;
            }
            tile_store_D(dz2, 16 * t, d);
        }
        __builtin_amdgcn_wave_barrier();
        // dW2 [64 x 64] = H1^T dZ2, db2 = column sums of dZ2
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            bf16x4 a = tile_load_AT(h1, 16 * mt);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                f32x4 g = {0.0f, 0.0f, 0.0f, 0.0f};
                g = mfma16(a, tile_load_B(dz2, 16 * t), g);
#pragma unroll
                for (int j = 0; j < 4; ++j) atomicAdd(&gacc[kW2 + (16 * mt + 4 * (l >> 4) + j) * kMlpH + 16 * t + n], g[j]);
            }
        }
        {
            float s = 0.0f;                     // lane l: column l
            for (int i = 0; i < 16; ++i) s += dz2[i * kTileLd + l];
            atomicAdd(&gacc[kB2 + l], s);
        }
        // dH1 [16 x 64] = dZ2 [16 x 64] W2^T; dZ1 = dH1 (1 - h1^2)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 d = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < 4; ++s) d = mfma16(tile_load_A(dz2, s), w_load_BT(M.Pb + kW2b, kMlpH, 16 * s, 16 * t), d);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                float hv = h1[(4 * (l >> 4) + j) * kTileLd + 16 * t + n];
                d[j] *= 1.0f - hv * hv;
            }
            // dz1's first 16 columns held dY, which is no longer needed
            tile_store_D(dz1, 16 * t, d);
        }
        __builtin_amdgcn_wave_barrier();
        // dW1 [16 (6 used) x 64] = X^T dZ1, db1 = column sums of dZ1
        bf16x4 axt;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            long long r = r0 + 4 * (l >> 4) + j;
            int k = l & 15;
            float v = (k < kMlpIn && r < M.n) ? M.X[r * kMlpXStride + k] : 0.0f;
            axt[j] = f2bf(v);
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            f32x4 g = {0.0f, 0.0f, 0.0f, 0.0f};
            g = mfma16(axt, tile_load_B(dz1, 16 * t), g);
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                int k = 4 * (l >> 4) + j;
                if (k < kMlpIn) atomicAdd(&gacc[kW1 + k * kMlpH + 16 * t + n], g[j]);
            }
        }
        {
            float s = 0.0f;
            for (int i = 0; i < 16; ++i) s += dz1[i * kTileLd + l];
            atomicAdd(&gacc[kB1 + l], s);
        }
        // loss
        for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
        if (l == 0) atomicAdd(&gacc[kMlpParams], lsum);
    }
    __syncthreads();
    float *out = M.gpart + (size_t)blockIdx.x * (kMlpParams + 1);
    for (int i = threadIdx.x; i < kMlpParams + 1; i += blockDim.x) out[i] = gacc[i];
}

// Refresh the BF16 padded copies of the weights from the FP32 master.
GM_D void write_bf16_param(short *Pb, int i, float v)
{
    if (i >= kW1 && i < kB1) {
        int k = (i - kW1) / kMlpH, n = (i - kW1) % kMlpH;
        Pb[kW1b + k * kMlpH + n] = f2bf(v);
    } else if (i >= kW2 && i < kB2) {
        Pb[kW2b + (i - kW2)] = f2bf(v);
    } else if (i >= kW3 && i < kB3) {
        int k = (i - kW3) / kMlpOut, n = (i - kW3) % kMlpOut;
        Pb[kW3b + k * 16 + n] = f2bf(v);
    }
}

struct AdamArgs {
    float *P, *m, *v;
    const float *g;
    short *Pb;
    float lr, beta1, beta2, eps, bc1, bc2;   // bc = 1 - beta^t
};

// One parameter's Adam step with gradient g (FP32 master, moments, BF16 copy).
GM_D void adam_update(const AdamArgs &A, int i, float g)
{
    float m = A.beta1 * A.m[i] + (1.0f - A.beta1) * g;
    float v = A.beta2 * A.v[i] + (1.0f - A.beta2) * g * g;
    A.m[i] = m;
    A.v[i] = v;
    float p = A.P[i] - A.lr * (m / A.bc1) / (sqrtf(v / A.bc2) + A.eps);
    A.P[i] = p;
    write_bf16_param(A.Pb, i, p);
}

// Sum the blocks' partial gradients.  A block takes 64 consecutive entries
// (lane = entry); its wave w sums the partials of blocks w, w + 4, w + 8, ...
// in that order, eight loads in flight, and the four waves' sums are added
// in wave order -- a fixed association, so the gradient does not depend on
// scheduling, and 4 x 75 waves share the partials' reads instead of one
// thread per entry walking all of them.
constexpr int kMlpReduceEntries = 64;
constexpr int kMlpReduceBlocks = (kMlpParams + 1 + kMlpReduceEntries - 1) / kMlpReduceEntries;

__global__ __launch_bounds__(256) void mlp_reduce_kernel(const float *gpart, int n_blocks, float *g)
{
    __shared__ float part[4][kMlpReduceEntries];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int i = blockIdx.x * kMlpReduceEntries + l;
    float s = 0.0f;
    if (i <= kMlpParams) {
#pragma unroll 8
        for (int b = w; b < n_blocks; b += 4) s += gpart[(size_t)b * (kMlpParams + 1) + i];
    }
    part[w][l] = s;
    __syncthreads();
    if (w == 0 && i <= kMlpParams) g[i] = ((part[0][l] + part[1][l]) + part[2][l]) + part[3][l];
}

// The same sum followed, for the block's entries, by their Adam step
// (adam_update): one launch per training step for both.
__global__ __launch_bounds__(256) void mlp_reduce_adam_kernel(const float *gpart, int n_blocks, float *g, AdamArgs A)
{
    __shared__ float part[4][kMlpReduceEntries];
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    const int i = blockIdx.x * kMlpReduceEntries + l;
    float s = 0.0f;
    if (i <= kMlpParams) {
#pragma unroll 8
        for (int b = w; b < n_blocks; b += 4) s += gpart[(size_t)b * (kMlpParams + 1) + i];
    }
    part[w][l] = s;
    __syncthreads();
    if (w == 0 && i <= kMlpParams) {
        const float gi = ((part[0][l] + part[1][l]) + part[2][l]) + part[3][l];
        g[i] = gi;
        if (i < kMlpParams) adam_update(A, i, gi);
    }
}



// Write every BF16 entry (padding as zero) from the FP32 master: one thread
// per BF16 entry, so no two threads write the same place.
__global__ __launch_bounds__(256) void mlp_sync_bf16_kernel(const float *P, short *Pb)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kMlpBf16) return;
    float v = 0.0f;
    if (i < kW2b) {
        int k = (i - kW1b) / kMlpH, n = (i - kW1b) % kMlpH;
        if (k < kMlpIn) v = P[kW1 + k * kMlpH + n];
    } else if (i < kW3b) {
        v = P[kW2 + (i - kW2b)];
    } else {
        int k = (i - kW3b) / 16, n = (i - kW3b) % 16;
        if (n < kMlpOut) v = P[kW3 + k * kMlpOut + n];
    }
    Pb[i] = f2bf(v);
}

}  // namespace gm
