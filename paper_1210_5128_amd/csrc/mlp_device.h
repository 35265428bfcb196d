// Device code of the learned swap proposal's network: per-node features
// (8) -> 128 -> 128 -> 1 logit, BF16 weights and activations on the matrix
// cores (v_mfma_f32_16x16x16_bf16), FP32 accumulation, FP32 biases.
//
// MFMA 16x16x16 operand layout (one wavefront, lane l):
//   A (16 x 16, row i, column k):  lane holds A[l % 16][4*(l/16) + j], j = 0..3
//   B (16 x 16, row k, column j'): lane holds B[4*(l/16) + j][l % 16]
//   D (16 x 16):                   lane holds D[4*(l/16) + r][l % 16],  r = 0..3
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bnos {

constexpr int kH = 128;          // hidden width
constexpr int kF = 8;            // features per node
constexpr int kFP = 16;          // features padded to the MFMA K
constexpr int kRows = 64;        // rows (nodes) of one sample, padded
constexpr int kNParam = kH * kF + kH + kH * kH + kH + kH + 1;   // 17,793
// offsets in the flat parameter vector W1 [128][8], b1, W2 [128][128], b2, w3, b3
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kH * kF;
constexpr int kOffW2 = kOffB1 + kH;
constexpr int kOffB2 = kOffW2 + kH * kH;
constexpr int kOffW3 = kOffB2 + kH;
constexpr int kOffB3 = kOffW3 + kH;

typedef short v4s __attribute__((ext_vector_type(4)));
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

// What the kernels read: BF16 copies of W1 (K padded to 16), W2 and w3
// (stored as the rounded floats), FP32 biases, feature normalisation.
struct MlpView {
    const uint16_t *W1b;     // [128][16]
    const uint16_t *W2b;     // [128][128]
    const float *w3r;        // [128] bf16-rounded values
    const float *b1, *b2, *b3;
    const float *norm;       // [16]: mu[8], 1/sd[8]
};

__device__ __forceinline__ v4f mfma16(v4s a, v4s b, v4f c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// LDS of one forward pass.
struct MlpLds {
    uint16_t z[kRows][kFP];      // normalised features, bf16
    uint16_t h1[kRows][kH];      // relu(layer 1), bf16
    float part[kRows][8];        // per column-tile partial logits
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
    for (int e = tid; e < kRows * kFP; e += blockDim.x) {
        const int r = e / kFP, k = e % kFP;
        float v = 0.f;
        if (r < rows && k < kF) v = (zraw[r * kF + k] - P.norm[k]) * P.norm[kF + k];
        L.z[r][k] = f2bf(v);
    }
    __syncthreads();
    const int li = lane & 15, lk = 4 * (lane >> 4);
    // layer 1: 4 row tiles x 8 column tiles, K = 16
    for (int tile = wave; tile < 32; tile += nw) {
        const int rt = tile >> 3, ct = tile & 7;
        v4s a, b;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            a[j] = (short)L.z[rt * 16 + li][lk + j];
            b[j] = (short)P.W1b[(ct * 16 + li) * kFP + lk + j];
        }
        v4f d = mfma16(a, b, (v4f){0.f, 0.f, 0.f, 0.f});
        const int u = ct * 16 + li;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float x = d[r] + P.b1[u];
            L.h1[rt * 16 + lk + r][u] = f2bf(x > 0.f ? x : 0.f);
        }
    }
    __syncthreads();
    // layer 2 (K = 128) and the layer-3 dot products per column tile
    for (int tile = wave; tile < 32; tile += nw) {
        const int rt = tile >> 3, ct = tile & 7;
        v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < kH / 16; ++ks) {
            v4s a, b;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                a[j] = (short)L.h1[rt * 16 + li][ks * 16 + lk + j];
                b[j] = (short)P.W2b[(ct * 16 + li) * kH + ks * 16 + lk + j];
            }
            d = mfma16(a, b, d);
        }
        const int u = ct * 16 + li;
        float q[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            float x = d[r] + P.b2[u];
            x = x > 0.f ? x : 0.f;
            if (h2) h2[(rt * 16 + lk + r) * kH + u] = x;
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
            for (int r = 0; r < 4; ++r) L.part[rt * 16 + lk + r][ct] = q[r];
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
