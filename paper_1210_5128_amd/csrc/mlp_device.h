// Device code of the learned swap proposal's network: per-node features
// (8) -> 128 -> 128 -> 1 logit on the matrix cores (v_mfma_f32_16x16x32_bf16,
// gfx950's K = 32 BF16 instruction), FP32 accumulation, FP32 biases.
//
// Precision: the weights are BF16 (W1, W2, w3 rounded to nearest even from
// the FP32 master copy).  Activations are not rounded to BF16: every
// activation operand x enters the matrix cores as two BF16 numbers, hi =
// bf16(x) and lo = bf16(x - hi), whose sum carries 16 significant bits
// (relative error <= 2^-17), and both halves are multiplied by the same
// weight.  The sums over rows in the backward pass (weight gradients) cancel
// strongly -- the loss gradient w.r.t. the logits sums to zero over the nodes
// -- so a single BF16 rounding of the activations (2^-9) would show up
// amplified in the gradients; with the split it stays below FP32 accumulation
// noise.
//
// MFMA 16x16x32 operand layout (one wavefront, lane l, g = l / 16):
//   A (16 x 32, row i, column k):  lane holds A[l % 16][8 g + j], j = 0..7
//   B (32 x 16, row k, column c):  lane holds B[8 g + j][l % 16]
//   D (16 x 16):                   lane holds D[4 g + r][l % 16],  r = 0..3
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bnos {

constexpr int kH = 128;          // hidden width
constexpr int kF = 8;            // features per node
constexpr int kRows = 64;        // rows (nodes) of one sample, padded
constexpr int kHP = kH + 8;      // LDS row pitch of hidden activations (bf16): breaks the 256-byte row stride
constexpr int kNParam = kH * kF + kH + kH * kH + kH + kH + 1;   // 17,793
// offsets in the flat parameter vector W1 [128][8], b1, W2 [128][128], b2, w3, b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kF;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef uint32_t v4u __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// float -> bf16 bits, round to nearest even (finite inputs)
__device__ __host__ __forceinline__ uint16_t f2bf(float x)
{
    uint32_t u;
    __builtin_memcpy(&u, &x, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __host__ __forceinline__ float bf2f(uint16_t b)
{
    uint32_t u = (uint32_t)b << 16;
    float x;
    __builtin_memcpy(&x, &u, 4);
    return x;
}

// x = hi + lo + O(2^-17 |x|); x - hi is exact in FP32.
__device__ __forceinline__ void split_bf(float x, uint16_t &hi, uint16_t &lo)
{
    hi = f2bf(x);
    lo = f2bf(x - bf2f(hi));
}

// What the kernels read: BF16 weights (W2 also transposed, for the backward
// pass), w3 as the BF16-rounded floats, FP32 biases, feature normalisation.
struct MlpView {
    const uint16_t *W1b;     // [128][8]
    const uint16_t *W2b;     // [128][128]  W2[u][k]
    const uint16_t *W2tb;    // [128][128]  W2[u][k] at [k][u]
    const float *w3r;        // [128] bf16-rounded values
    const float *b1, *b2, *b3;
    const float *norm;       // [16]: mu[8], 1/sd[8]
};

__device__ __forceinline__ v4f mfma32(v4u a, v4u b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(v8bf, a), __builtin_bit_cast(v8bf, b), c, 0,
                                                   0, 0);
}

// Eight consecutive bf16 values (16-byte aligned) as one operand register set.
__device__ __forceinline__ v4u ld8(const uint16_t *p) { return *reinterpret_cast<const v4u *>(p); }

// Eight bf16 values p[0], p[s], ..., p[7 s] (a column of a row-major array).
__device__ __forceinline__ v4u ld8_strided(const uint16_t *p, int s)
{
    v4u v;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = (uint32_t)p[(2 * j) * s] | ((uint32_t)p[(2 * j + 1) * s] << 16);
    return v;
}

// LDS of one forward pass (16-byte aligned: operands are read with 16-byte LDS loads).
struct alignas(16) MlpLds {
    uint16_t z[kRows][16];          // normalised features: hi in columns 0..7, lo in 8..15
    uint16_t h1[2][kRows][kHP];     // relu(layer 1): [0] hi, [1] lo
    float part[kRows][8];           // per column-tile partial logits
    float logit[kRows];
};

// Forward pass of one sample (rows <= 64 nodes) by a block of 1-32 wavefronts.
// zraw: raw features [rows][8] (LDS or global).  If h2 != null, relu(layer 2)
// is also stored there ([64][128] floats, for the backward pass).  The
// logits land in L.logit[0..rows).  Fixed reduction orders: deterministic.
__device__ __forceinline__ void mlp_forward_block(const MlpView &P, const float *zraw, int rows, MlpLds &L,
                                                  float *h2)
{
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int nw = blockDim.x >> 6;
    for (int e = tid; e < kRows * kF; e += blockDim.x) {
        const int r = e / kF, k = e % kF;
        float v = 0.f;
        if (r < rows) v = (zraw[r * kF + k] - P.norm[k]) * P.norm[kF + k];
        split_bf(v, L.z[r][k], L.z[r][kF + k]);
    }
    __syncthreads();
    const int li = lane & 15, g = lane >> 4;
    // layer 1: 4 row tiles x 8 column tiles, one K = 32 step: A = [z_hi | z_lo | 0 | 0],
    // B = [W1^T; W1^T; 0; 0], so the product is (z_hi + z_lo) W1^T
    for (int tile = wave; tile < 32; tile += nw) {
        const int rt = tile >> 3, ct = tile & 7;
        v4u a = {0u, 0u, 0u, 0u}, b = {0u, 0u, 0u, 0u};
        if (g < 2) {
            a = ld8(&L.z[rt * 16 + li][8 * g]);
            b = ld8(P.W1b + (ct * 16 + li) * kF);
        }
        const v4f d = mfma32(a, b, (v4f){0.f, 0.f, 0.f, 0.f});
        const int u = ct * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float x = d[r] + P.b1[u];
            split_bf(x > 0.f ? x : 0.f, L.h1[0][rt * 16 + 4 * g + r][u], L.h1[1][rt * 16 + 4 * g + r][u]);
        }
    }
    __syncthreads();
    // layer 2: K = 128 inputs, taken twice (hi, then lo), each against W2; then
    // the layer-3 dot products per column tile
    for (int tile = wave; tile < 32; tile += nw) {
        const int rt = tile >> 3, ct = tile & 7;
        v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int part = s >> 2, kb = (s & 3) * 32 + 8 * g;
            d = mfma32(ld8(&L.h1[part][rt * 16 + li][kb]), ld8(P.W2b + (ct * 16 + li) * kH + kb), d);
        }
        const int u = ct * 16 + li;
        float q[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float x = d[r] + P.b2[u];
            x = x > 0.f ? x : 0.f;
            if (h2) h2[(rt * 16 + 4 * g + r) * kH + u] = x;
            q[r] = x * P.w3r[u];
        }
        // sum over the 16 columns of the tile (lanes with equal l/16), fixed butterfly
#pragma unroll
        for (int off = 1; off < 16; off <<= 1)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const float o = __shfl_xor(q[r], off, 64);
                q[r] = (li & off) ? (o + q[r]) : (q[r] + o);
            }
        if (li == 0)
#pragma unroll
            for (int r = 0; r < 4; ++r) L.part[rt * 16 + 4 * g + r][ct] = q[r];
    }
    __syncthreads();
    if (tid < kRows) {
        float s = P.b3[0];
#pragma unroll
        for (int ct = 0; ct < 8; ++ct) s += L.part[tid][ct];
        L.logit[tid] = s;
    }
    __syncthreads();
}

// ln q({a,b}) from logits (FP64 softmax of the FP32 logits), eps mixing weight.
__device__ __forceinline__ double pair_logq_dev(const float *logit, int n, int a, int b, double eps)
{
    double mx = -1e300;
    for (int i = 0; i < n; ++i) mx = logit[i] > mx ? logit[i] : mx;
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += exp((double)logit[i] - mx);
    const double pa = exp((double)logit[a] - mx) / s, pb = exp((double)logit[b] - mx) / s;
    const double Q = pa * pb * (1.0 / (1.0 - pa) + 1.0 / (1.0 - pb));
    return log((1.0 - eps) * Q + eps * 2.0 / ((double)n * (n - 1)));
}

// host side (mlp.hip)
MlpView mlp_view(const void *mlp_handle);
bool mlp_handle_live(const void *mlp_handle);

}  // namespace bnos
