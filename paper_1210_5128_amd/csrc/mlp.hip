// The learned swap proposal's network on the device: parameters (FP32
// master + BF16 copies), forward pass, loss gradient by hand-written
// MFMA backward GEMMs, deterministic reductions and Adam.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "bnos_internal.h"
#include "mlp_device.h"

namespace bnos {

struct MlpT {
    uint32_t magic = 0;
    int device = 0;
    float *d_master = nullptr;   // [kNParam]
    float *d_m = nullptr;        // Adam first moment
    float *d_v = nullptr;        // Adam second moment
    uint16_t *d_W1b = nullptr;   // [128][8]
    uint16_t *d_W2b = nullptr;   // [128][128]
    uint16_t *d_W2tb = nullptr;  // [128][128], transposed
    float *d_w3r = nullptr;      // [128]
    float *d_norm = nullptr;     // [16]: mu, 1/sd
    double *d_normpart = nullptr;   // [kNormBlocks][16]: per-block feature sums
    float h_mu[kF], h_sd[kF];
    int64_t adam_t = 0;
};

constexpr uint32_t kMlpMagic = 0x3E7A11CEu;
static std::mutex g_mlp_mu;
static std::set<const MlpT *> g_mlps;

static bool mlp_live(const MlpT *m)
{
    std::lock_guard<std::mutex> lk(g_mlp_mu);
    return m && g_mlps.count(m) && m->magic == kMlpMagic;
}

MlpView mlp_view(const void *h)
{
    const MlpT *m = reinterpret_cast<const MlpT *>(h);
    MlpView P;
    P.W1b = m->d_W1b;
    P.W2b = m->d_W2b;
    P.W2tb = m->d_W2tb;
    P.w3r = m->d_w3r;
    P.b1 = m->d_master + kOffB1;
    P.b2 = m->d_master + kOffB2;
    P.b3 = m->d_master + kOffB3;
    P.norm = m->d_norm;
    return P;
}

bool mlp_handle_live(const void *h) { return mlp_live(reinterpret_cast<const MlpT *>(h)); }

// ------------------------------------------------------------------ kernels

// BF16 copies of the weights from the FP32 master (W2 also transposed).
__global__ void k_mlp_refresh(const float *__restrict__ master, uint16_t *__restrict__ W1b,
                              uint16_t *__restrict__ W2b, uint16_t *__restrict__ W2tb, float *__restrict__ w3r)
{
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < kH * kF) {
        W1b[g] = f2bf(master[kOffW1 + g]);
    } else if (g < kH * kF + kH * kH) {
        const int e = g - kH * kF;
        const uint16_t b = f2bf(master[kOffW2 + e]);
        W2b[e] = b;
        W2tb[(e % kH) * kH + e / kH] = b;
    } else if (g < kH * kF + kH * kH + kH) {
        const int e = g - kH * kF - kH * kH;
        w3r[e] = bf2f(f2bf(master[kOffW3 + e]));
    }
}

// Block per sample: logits of its n nodes from raw features [R][n][8].
__global__ __launch_bounds__(1024) void k_mlp_forward(MlpView P, const float *__restrict__ feats, int n,
                                                      float *__restrict__ logits)
{
    __shared__ MlpLds L;
    const int s = blockIdx.x;
    mlp_forward_block(P, feats + (int64_t)s * n * kF, n, L, nullptr);
    if (threadIdx.x < n) logits[(int64_t)s * n + threadIdx.x] = L.logit[threadIdx.x];
}

// Per-feature mean and population standard deviation over `rows` rows (FP64,
// fixed reduction trees, so the result does not depend on scheduling); sd
// below 1e-6 is replaced by 1.  Block b of kNormBlocks sums rows b, b + G, ...
// (G = grid threads) per thread, then a tree over its threads; the last
// kernel adds the block sums in block order.
constexpr int kNormBlocks = 256;
constexpr int kNormThreads = 256;
__global__ __launch_bounds__(kNormThreads) void k_feat_norm_part(const float *__restrict__ feats, int64_t rows,
                                                                  double *__restrict__ part)
{
    __shared__ double s1[kF][kNormThreads], s2[kF][kNormThreads];
    double a[kF], b[kF];
#pragma unroll
    for (int k = 0; k < kF; ++k) a[k] = b[k] = 0.0;
    const float4 *f4 = reinterpret_cast<const float4 *>(feats);
    const int64_t stride = (int64_t)gridDim.x * kNormThreads;
    for (int64_t r = (int64_t)blockIdx.x * kNormThreads + threadIdx.x; r < rows; r += stride) {
        const float4 lo = f4[2 * r], hi = f4[2 * r + 1];
        const float v[kF] = {lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
#pragma unroll
        for (int k = 0; k < kF; ++k) {
            a[k] += (double)v[k];
            b[k] += (double)v[k] * (double)v[k];
        }
    }
#pragma unroll
    for (int k = 0; k < kF; ++k) {
        s1[k][threadIdx.x] = a[k];
        s2[k][threadIdx.x] = b[k];
    }
    __syncthreads();
    for (int w = kNormThreads / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w)
#pragma unroll
            for (int k = 0; k < kF; ++k) {
                s1[k][threadIdx.x] += s1[k][threadIdx.x + w];
                s2[k][threadIdx.x] += s2[k][threadIdx.x + w];
            }
        __syncthreads();
    }
    if (threadIdx.x < kF) {
        part[(int64_t)blockIdx.x * 2 * kF + threadIdx.x] = s1[threadIdx.x][0];
        part[(int64_t)blockIdx.x * 2 * kF + kF + threadIdx.x] = s2[threadIdx.x][0];
    }
}

__global__ void k_feat_norm_final(const double *__restrict__ part, int blocks, int64_t rows,
                                  float *__restrict__ norm)
{
    const int k = threadIdx.x;
    if (k >= kF) return;
    double t1 = 0.0, t2 = 0.0;
    for (int b = 0; b < blocks; ++b) {
        t1 += part[(int64_t)b * 2 * kF + k];
        t2 += part[(int64_t)b * 2 * kF + kF + k];
    }
    const double mu = rows ? t1 / (double)rows : 0.0;
    const double var = rows ? t2 / (double)rows - mu * mu : 1.0;
    double sd = var > 0 ? sqrt(var) : 0.0;
    if (!(sd > 1e-6)) sd = 1.0;
    norm[k] = (float)mu;
    norm[kF + k] = (float)(1.0 / sd);
}

struct alignas(16) GradLds {
    MlpLds f;
    float zraw[kRows * kF];
    float h2[kRows][kH];            // relu(layer 2); later reused for dpre1
    uint16_t d2[2][kRows][kHP];     // dL/dpre2 as hi / lo bf16 operands
    float dl[kRows];
    float gw3[kH], gb2[kH], gb1[kH];
    double loss;
    float gb3;
};

// Sample index of position j of the epoch's visiting order (affine bijection).
__device__ __forceinline__ int64_t visit(int64_t j, int64_t count, int64_t stride, int64_t offset)
{
    // j < 2^31 and stride < count <= 2^31: the product fits in 64 bits
    return (int64_t)(((uint64_t)j * (uint64_t)stride + (uint64_t)offset) % (uint64_t)count);
}

// Block per chunk of `spb` samples: forward, gradient of -ln q(pair) w.r.t.
// the logits, backward through both layers with MFMA GEMMs (the weight
// gradients accumulate in matrix-core accumulators across the chunk), then
// one partial gradient (+ loss sum at index kNParam) per block.  Every
// activation operand is a hi/lo BF16 pair (see mlp_device.h); products of two
// activations take hi*hi + hi*lo + lo*hi.
constexpr int kGradWaves = 8;
constexpr int kW2TilesPerWave = 64 / kGradWaves;

__global__ __launch_bounds__(kGradWaves * 64) void k_mlp_grad(MlpView P, const float *__restrict__ feats,
                                                   const int32_t *__restrict__ pairs, int64_t count, int64_t first,
                                                   int64_t nsamples, int64_t stride, int64_t offset, int n, int spb,
                                                   double eps, float *__restrict__ part)
{
    __shared__ GradLds G;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int li = lane & 15, g = lane >> 4;
    v4f accW2[kW2TilesPerWave];     // gW2 tiles (ut, kt) = (wave*T+q) / 8, % 8
    v4f accW1 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int q = 0; q < kW2TilesPerWave; ++q) accW2[q] = (v4f){0.f, 0.f, 0.f, 0.f};
    if (tid < kH) {
        G.gw3[tid] = 0.f;
        G.gb2[tid] = 0.f;
        G.gb1[tid] = 0.f;
    }
    if (tid == 0) {
        G.loss = 0.0;
        G.gb3 = 0.f;
    }
    const int64_t j0 = (int64_t)blockIdx.x * spb;
    for (int si = 0; si < spb; ++si) {
        const int64_t j = j0 + si;
        if (j >= nsamples) break;                        // uniform
        const int64_t smp = visit(first + j, count, stride, offset);
        for (int e = tid; e < n * kF; e += blockDim.x) G.zraw[e] = feats[smp * n * kF + e];
        __syncthreads();
        mlp_forward_block(P, G.zraw, n, G.f, &G.h2[0][0]);
        // dL/dlogit for L = -ln q({a,b})
        if (wave == 0) {
            const int a = pairs[smp * 2], b = pairs[smp * 2 + 1];
            const double l = lane < n ? (double)G.f.logit[lane] : -1e300;
            double mx = l;
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
            double e = lane < n ? exp(l - mx) : 0.0;
            double se = e;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const double o = __shfl_xor(se, off, 64);
                se = (lane & off) ? (o + se) : (se + o);
            }
            const double p = e / se;
            const double pa = __shfl(p, a, 64), pb = __shfl(p, b, 64);
            const double Q = pa * pb * (1.0 / (1.0 - pa) + 1.0 / (1.0 - pb));
            const double q = (1.0 - eps) * Q + eps * 2.0 / ((double)n * (n - 1));
            const double ga = pa * pb * (1.0 / ((1.0 - pa) * (1.0 - pa)) + 1.0 / (1.0 - pb));
            const double gb = pb * pa * (1.0 / ((1.0 - pb) * (1.0 - pb)) + 1.0 / (1.0 - pa));
            double dQ = -p * (ga + gb) + (lane == a ? ga : 0.0) + (lane == b ? gb : 0.0);
            G.dl[lane] = lane < n ? (float)(-(1.0 - eps) * dQ / q) : 0.f;
            if (lane == 0) G.loss += -log(q);
        }
        __syncthreads();
        // dL/dpre2 = relu'(pre2) * dl * w3 (hi/lo operands); bias / w3 / b3 gradients (rows in order)
        for (int e = tid; e < kRows * kH; e += blockDim.x) {
            const int r = e / kH, u = e % kH;
            const float d = G.h2[r][u] > 0.f ? G.dl[r] * P.w3r[u] : 0.f;
            split_bf(d, G.d2[0][r][u], G.d2[1][r][u]);
        }
        if (tid < kH) {
            float s3 = 0.f, s2 = 0.f;
            for (int r = 0; r < n; ++r) {
                const float h = G.h2[r][tid];
                s3 += G.dl[r] * h;
                s2 += h > 0.f ? G.dl[r] * P.w3r[tid] : 0.f;
            }
            G.gw3[tid] += s3;
            G.gb2[tid] += s2;
        }
        if (tid == 0) {
            float s = 0.f;
            for (int r = 0; r < n; ++r) s += G.dl[r];
            G.gb3 += s;
        }
        __syncthreads();
        // gW2[u][k] += sum_r d2[r][u] h1[r][k]: A[u][r] = d2, B[r][k] = h1, K = 64 rows in two
        // steps of 32, for the products (d2 hi, h1 hi), (d2 hi, h1 lo), (d2 lo, h1 hi)
#pragma unroll
        for (int q = 0; q < kW2TilesPerWave; ++q) {
            const int tile = wave * kW2TilesPerWave + q, ut = tile >> 3, kt = tile & 7;
#pragma unroll
            for (int pr = 0; pr < 3; ++pr) {
                const int pd = pr == 2 ? 1 : 0, ph = pr == 1 ? 1 : 0;
#pragma unroll
                for (int ks = 0; ks < 2; ++ks) {
                    const int r0 = ks * 32 + 8 * g;
                    accW2[q] = mfma32(ld8_strided(&G.d2[pd][r0][ut * 16 + li], kHP),
                                      ld8_strided(&G.f.h1[ph][r0][kt * 16 + li], kHP), accW2[q]);
                }
            }
        }
        __syncthreads();
        // dh1[r][k] = sum_u d2[r][u] W2[u][k] (K = 128, hi then lo); dpre1 = relu'(pre1) dh1 -> G.h2
        for (int tile = wave; tile < 32; tile += kGradWaves) {
            const int rt = tile >> 3, kt = tile & 7;
            v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                const int pd = s >> 2, ub = (s & 3) * 32 + 8 * g;
                d = mfma32(ld8(&G.d2[pd][rt * 16 + li][ub]), ld8(P.W2tb + (kt * 16 + li) * kH + ub), d);
            }
            const int k = kt * 16 + li;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = rt * 16 + 4 * g + r;
                G.h2[row][k] = (row < n && G.f.h1[0][row][k] != 0) ? d[r] : 0.f;
            }
        }
        __syncthreads();
        if (tid < kH) {
            float s1 = 0.f;
            for (int r = 0; r < n; ++r) s1 += G.h2[r][tid];
            G.gb1[tid] += s1;
        }
        // gW1[u][k] += sum_r dpre1[r][u] z[r][k]: A[u][r] = dpre1 (hi, then lo), B[r][c] = the
        // z row (columns 0..7 hi, 8..15 lo); columns c and c + 8 are added at the end, so the
        // tile sums hi*hi + hi*lo + lo*hi + lo*lo (8 tiles of 16 hidden units)
        if (wave < 8) {
            const int ut = wave;
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const int part = s >> 1, r0 = (s & 1) * 32 + 8 * g;
                v4u a;
#pragma unroll
                for (int jj = 0; jj < 4; ++jj) {
                    uint16_t h0, l0, h1v, l1;
                    split_bf(G.h2[r0 + 2 * jj][ut * 16 + li], h0, l0);
                    split_bf(G.h2[r0 + 2 * jj + 1][ut * 16 + li], h1v, l1);
                    a[jj] = part ? ((uint32_t)l0 | ((uint32_t)l1 << 16)) : ((uint32_t)h0 | ((uint32_t)h1v << 16));
                }
                accW1 = mfma32(a, ld8_strided(&G.f.z[r0][li], 16), accW1);
            }
        }
        __syncthreads();
    }
    // partial gradient of this block
    float *out = part + (int64_t)blockIdx.x * (kNParam + 1);
#pragma unroll
    for (int q = 0; q < kW2TilesPerWave; ++q) {
        const int tile = wave * kW2TilesPerWave + q, ut = tile >> 3, kt = tile & 7;
#pragma unroll
        for (int r = 0; r < 4; ++r) out[kOffW2 + (ut * 16 + 4 * g + r) * kH + kt * 16 + li] = accW2[q][r];
    }
    if (wave < 8) {
        // column li + 8 holds the products with z_lo of column li
        float hi8[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) hi8[r] = __shfl(accW1[r], (lane & ~15) | ((li + 8) & 15), 64);
        if (li < kF)
#pragma unroll
            for (int r = 0; r < 4; ++r) out[kOffW1 + (wave * 16 + 4 * g + r) * kF + li] = accW1[r] + hi8[r];
    }
    if (tid < kH) {
        out[kOffB1 + tid] = G.gb1[tid];
        out[kOffB2 + tid] = G.gb2[tid];
        out[kOffW3 + tid] = G.gw3[tid];
    }
    if (tid == 0) {
        out[kOffB3] = G.gb3;
        out[kNParam] = (float)G.loss;
    }
}

// grad[p] = (sum over blocks, in block order) / count; loss likewise.
__global__ void k_grad_reduce(const float *__restrict__ part, int blocks, double inv, float *__restrict__ grad,
                              double *__restrict__ loss, float *__restrict__ loss_slot)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kNParam) return;
    double s = 0.0;
    for (int b = 0; b < blocks; ++b) s += part[(int64_t)b * (kNParam + 1) + p];
    if (p < kNParam) {
        grad[p] = (float)(s * inv);
    } else {
        if (loss) *loss = s * inv;
        if (loss_slot) *loss_slot = (float)(s * inv);
    }
}

// Adam (Kingma & Ba 2015) on the FP32 master weights.
__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kNParam) return;
    const float gp = g[p];
    const float mp = b1 * m[p] + (1.f - b1) * gp;
    const float vp = b2 * v[p] + (1.f - b2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    w[p] -= lr * (mp / c1) / (sqrtf(vp / c2) + eps);
}

static void refresh(MlpT *m, hipStream_t st)
{
    const int total = kH * kF + kH * kH + kH;
    hipLaunchKernelGGL(k_mlp_refresh, dim3((total + 255) / 256), dim3(256), 0, st, m->d_master, m->d_W1b,
                       m->d_W2b, m->d_W2tb, m->d_w3r);
}

static void free_mlp(MlpT *m)
{
    hipFree(m->d_master);
    hipFree(m->d_m);
    hipFree(m->d_v);
    hipFree(m->d_W1b);
    hipFree(m->d_W2b);
    hipFree(m->d_W2tb);
    hipFree(m->d_w3r);
    hipFree(m->d_norm);
    hipFree(m->d_normpart);
}

constexpr int kSamplesPerBlock = 8;

static bnos_status grad_impl(MlpT *m, const float *feats, const int32_t *pairs, int64_t count, int64_t first,
                             int64_t nsamples, int64_t stride, int64_t offset, int n, double eps, float *grad,
                             double *loss, float *loss_slot, float *part, hipStream_t st)
{
    const int blocks = (int)((nsamples + kSamplesPerBlock - 1) / kSamplesPerBlock);
    hipLaunchKernelGGL(k_mlp_grad, dim3(blocks), dim3(kGradWaves * 64), 0, st, mlp_view(m), feats, pairs, count, first, nsamples,
                       stride, offset, n, kSamplesPerBlock, eps, part);
    BNOS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_grad_reduce, dim3((kNParam + 1 + 255) / 256), dim3(256), 0, st, part, blocks,
                       1.0 / (double)nsamples, grad, loss, loss_slot);
    BNOS_HIP(hipGetLastError());
    return BNOS_OK;
}

}  // namespace bnos

using namespace bnos;

extern "C" bnos_status bnos_mlp_create(bnos_mlp *out)
{
    if (!out) { set_error("out is NULL"); return BNOS_E_INVALID; }
    MlpT *m = new (std::nothrow) MlpT();
    if (!m) { set_error("host allocation failed"); return BNOS_E_NOMEM; }
    hipError_t e;
    if ((e = hipGetDevice(&m->device)) != hipSuccess) { delete m; set_error(hipGetErrorString(e)); return BNOS_E_DEVICE; }
#define ALLOC(p, bytes) if ((e = hipMalloc((void **)&(p), (bytes))) != hipSuccess) { free_mlp(m); delete m; set_error(std::string("hipMalloc: ") + hipGetErrorString(e)); return e == hipErrorOutOfMemory ? BNOS_E_NOMEM : BNOS_E_DEVICE; }
    ALLOC(m->d_master, sizeof(float) * kNParam);
    ALLOC(m->d_m, sizeof(float) * kNParam);
    ALLOC(m->d_v, sizeof(float) * kNParam);
    ALLOC(m->d_W1b, sizeof(uint16_t) * kH * kF);
    ALLOC(m->d_W2b, sizeof(uint16_t) * kH * kH);
    ALLOC(m->d_W2tb, sizeof(uint16_t) * kH * kH);
    ALLOC(m->d_normpart, sizeof(double) * kNormBlocks * 2 * kF);
    ALLOC(m->d_w3r, sizeof(float) * kH);
    ALLOC(m->d_norm, sizeof(float) * 2 * kF);
#undef ALLOC
    std::vector<float> zero(kNParam, 0.f);
    float norm[2 * kF];
    for (int k = 0; k < kF; ++k) {
        m->h_mu[k] = 0.f;
        m->h_sd[k] = 1.f;
        norm[k] = 0.f;
        norm[kF + k] = 1.f;
    }
    bool ok = hipMemcpy(m->d_master, zero.data(), sizeof(float) * kNParam, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(m->d_m, zero.data(), sizeof(float) * kNParam, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(m->d_v, zero.data(), sizeof(float) * kNParam, hipMemcpyHostToDevice) == hipSuccess &&
              hipMemcpy(m->d_norm, norm, sizeof norm, hipMemcpyHostToDevice) == hipSuccess;
    if (!ok) { free_mlp(m); delete m; set_error("hipMemcpy failed"); return BNOS_E_DEVICE; }
    refresh(m, nullptr);
    if (hipDeviceSynchronize() != hipSuccess) { free_mlp(m); delete m; set_error("refresh failed"); return BNOS_E_DEVICE; }
    m->magic = kMlpMagic;
    {
        std::lock_guard<std::mutex> lk(g_mlp_mu);
        g_mlps.insert(m);
    }
    *out = reinterpret_cast<bnos_mlp>(m);
    return BNOS_OK;
}

extern "C" void bnos_mlp_free(bnos_mlp h)
{
    MlpT *m = reinterpret_cast<MlpT *>(h);
    if (!mlp_live(m)) return;
    {
        std::lock_guard<std::mutex> lk(g_mlp_mu);
        g_mlps.erase(m);
    }
    hipDeviceSynchronize();
    m->magic = 0;
    free_mlp(m);
    delete m;
}

extern "C" bnos_status bnos_mlp_set_params(bnos_mlp h, const float *params, const float *mu, const float *sd)
{
    MlpT *m = reinterpret_cast<MlpT *>(h);
    if (!mlp_live(m)) { set_error("invalid network handle"); return BNOS_E_STATE; }
    if (params)
        for (int p = 0; p < kNParam; ++p)
            if (!std::isfinite(params[p])) { set_error("non-finite parameter"); return BNOS_E_INVALID; }
    if ((mu && !sd) || (!mu && sd)) { set_error("mu and sd go together"); return BNOS_E_INVALID; }
    if (sd)
        for (int k = 0; k < kF; ++k)
            if (!(sd[k] > 0.f) || !std::isfinite(sd[k]) || !std::isfinite(mu[k])) { set_error("sd must be > 0, finite"); return BNOS_E_INVALID; }
    BNOS_HIP(hipSetDevice(m->device));
    if (params) {
        std::vector<float> zero(kNParam, 0.f);
        BNOS_HIP(hipMemcpy(m->d_master, params, sizeof(float) * kNParam, hipMemcpyHostToDevice));
        BNOS_HIP(hipMemcpy(m->d_m, zero.data(), sizeof(float) * kNParam, hipMemcpyHostToDevice));
        BNOS_HIP(hipMemcpy(m->d_v, zero.data(), sizeof(float) * kNParam, hipMemcpyHostToDevice));
        m->adam_t = 0;
        refresh(m, nullptr);
        BNOS_HIP(hipGetLastError());
    }
    if (mu) {
        float norm[2 * kF];
        for (int k = 0; k < kF; ++k) {
            m->h_mu[k] = mu[k];
            m->h_sd[k] = sd[k];
            norm[k] = mu[k];
            norm[kF + k] = 1.f / sd[k];
        }
        BNOS_HIP(hipMemcpy(m->d_norm, norm, sizeof norm, hipMemcpyHostToDevice));
    }
    BNOS_HIP(hipDeviceSynchronize());
    return BNOS_OK;
}

extern "C" bnos_status bnos_mlp_get_params(bnos_mlp h, float *params, float *mu, float *sd)
{
    MlpT *m = reinterpret_cast<MlpT *>(h);
    if (!mlp_live(m)) { set_error("invalid network handle"); return BNOS_E_STATE; }
    BNOS_HIP(hipSetDevice(m->device));
    BNOS_HIP(hipDeviceSynchronize());
    if (params) BNOS_HIP(hipMemcpy(params, m->d_master, sizeof(float) * kNParam, hipMemcpyDeviceToHost));
    if (mu || sd) {
        float norm[2 * kF];
        BNOS_HIP(hipMemcpy(norm, m->d_norm, sizeof norm, hipMemcpyDeviceToHost));
        for (int k = 0; k < kF; ++k) {
            if (mu) mu[k] = norm[k];
            if (sd) sd[k] = 1.f / norm[kF + k];
        }
    }
    return BNOS_OK;
}

extern "C" bnos_status bnos_mlp_fit_norm(bnos_mlp h, const float *feats, int64_t rows, void *stream)
{
    MlpT *m = reinterpret_cast<MlpT *>(h);
    if (!mlp_live(m)) { set_error("invalid network handle"); return BNOS_E_STATE; }
    if (!feats || rows < 1) { set_error("need at least one feature row"); return BNOS_E_INVALID; }
    if (reinterpret_cast<uintptr_t>(feats) % 16) { set_error("feats must be 16-byte aligned"); return BNOS_E_INVALID; }
    BNOS_HIP(hipSetDevice(m->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    int64_t want = (rows + kNormThreads - 1) / kNormThreads;
    const int blocks = (int)(want < kNormBlocks ? want : kNormBlocks);
    hipLaunchKernelGGL(k_feat_norm_part, dim3(blocks), dim3(kNormThreads), 0, st, feats, rows, m->d_normpart);
    BNOS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_feat_norm_final, dim3(1), dim3(64), 0, st, m->d_normpart, blocks, rows, m->d_norm);
    BNOS_HIP(hipGetLastError());
    return BNOS_OK;
}

extern "C" bnos_status bnos_mlp_forward(bnos_mlp h, const float *feats, int32_t R, int32_t n, float *logits,
                                        void *stream)
{
    MlpT *m = reinterpret_cast<MlpT *>(h);
    if (!mlp_live(m)) { set_error("invalid network handle"); return BNOS_E_STATE; }
    if (!feats || !logits) { set_error("NULL argument"); return BNOS_E_INVALID; }
    if (R < 1 || n < 2 || n > 64) { set_error("need R >= 1 and 2 <= n <= 64"); return BNOS_E_RANGE; }
    BNOS_HIP(hipSetDevice(m->device));
    hipLaunchKernelGGL(k_mlp_forward, dim3(R), dim3(1024), 0, reinterpret_cast<hipStream_t>(stream), mlp_view(m),
                       feats, n, logits);
    BNOS_HIP(hipGetLastError());
    return BNOS_OK;
}

extern "C" bnos_status bnos_mlp_grad(bnos_mlp h, const float *feats, const int32_t *pairs, int32_t R, int32_t n,
                                     float eps, float *grad, double *loss, void *stream)
{
    MlpT *m = reinterpret_cast<MlpT *>(h);
    if (!mlp_live(m)) { set_error("invalid network handle"); return BNOS_E_STATE; }
    if (!feats || !pairs || !grad) { set_error("NULL argument"); return BNOS_E_INVALID; }
    if (R < 1 || n < 2 || n > 64) { set_error("need R >= 1 and 2 <= n <= 64"); return BNOS_E_RANGE; }
    if (!(eps >= 0.f && eps <= 1.f)) { set_error("eps outside [0, 1]"); return BNOS_E_RANGE; }
    BNOS_HIP(hipSetDevice(m->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int blocks = (R + kSamplesPerBlock - 1) / kSamplesPerBlock;
    float *part = nullptr;
    BNOS_HIP(hipMalloc((void **)&part, sizeof(float) * (size_t)blocks * (kNParam + 1)));
    bnos_status s = grad_impl(m, feats, pairs, R, 0, R, 1, 0, n, eps, grad, loss, nullptr, part, st);
    hipError_t e = hipStreamSynchronize(st);
    hipFree(part);
    if (s != BNOS_OK) return s;
    if (e != hipSuccess) { set_error(hipGetErrorString(e)); return BNOS_E_DEVICE; }
    return BNOS_OK;
}

static uint64_t host_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int64_t gcd64(int64_t a, int64_t b)
{
    while (b) {
        int64_t t = a % b;
        a = b;
        b = t;
    }
    return a;
}

extern "C" bnos_status bnos_mlp_train(bnos_mlp h, const float *feats, const int32_t *pairs, int64_t count, int32_t n,
                                      float eps, int32_t epochs, int32_t batch, float lr, uint64_t seed,
                                      float *loss_trace, void *stream)
{
    MlpT *m = reinterpret_cast<MlpT *>(h);
    if (!mlp_live(m)) { set_error("invalid network handle"); return BNOS_E_STATE; }
    if (!feats || !pairs) { set_error("NULL argument"); return BNOS_E_INVALID; }
    if (count < 1 || n < 2 || n > 64 || epochs < 0 || batch < 1) { set_error("bad sizes"); return BNOS_E_RANGE; }
    if (!(eps >= 0.f && eps <= 1.f) || !(lr > 0.f)) { set_error("bad eps or lr"); return BNOS_E_RANGE; }
    BNOS_HIP(hipSetDevice(m->device));
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t bsz = batch < count ? batch : count;
    const int blocks = (int)((bsz + kSamplesPerBlock - 1) / kSamplesPerBlock);
    float *part = nullptr, *grad = nullptr;
    BNOS_HIP(hipMalloc((void **)&part, sizeof(float) * (size_t)blocks * (kNParam + 1) + sizeof(float) * kNParam + 64));
    grad = part + (size_t)blocks * (kNParam + 1);
    const int64_t steps_per_epoch = (count + bsz - 1) / bsz;
    int64_t step = 0;
    bnos_status s = BNOS_OK;
    for (int ep = 0; ep < epochs && s == BNOS_OK; ++ep) {
        // visiting order of this epoch: j -> (offset + j * stride) mod count, stride coprime to count
        uint64_t r = host_mix(seed ^ host_mix(0x5EEDull + (uint64_t)ep));
        int64_t stride = 1 + (int64_t)(r % (uint64_t)count);
        while (gcd64(stride, count) != 1) stride = stride % count + 1;
        const int64_t offset = (int64_t)(host_mix(r) % (uint64_t)count);
        for (int64_t b = 0; b < steps_per_epoch && s == BNOS_OK; ++b) {
            const int64_t first = b * bsz;
            const int64_t ns = (first + bsz <= count) ? bsz : count - first;
            s = grad_impl(m, feats, pairs, count, first, ns, stride, offset, n, eps, grad, nullptr,
                          loss_trace ? loss_trace + step : nullptr, part, st);
            if (s != BNOS_OK) break;
            ++m->adam_t;
            const float b1 = 0.9f, b2 = 0.999f;
            const float c1 = 1.f - powf(b1, (float)m->adam_t), c2 = 1.f - powf(b2, (float)m->adam_t);
            hipLaunchKernelGGL(k_adam, dim3((kNParam + 255) / 256), dim3(256), 0, st, m->d_master, m->d_m, m->d_v,
                               grad, lr, b1, b2, 1e-8f, c1, c2);
            refresh(m, st);
            if (hipGetLastError() != hipSuccess) { s = BNOS_E_DEVICE; set_error("training launch failed"); }
            ++step;
        }
    }
    hipError_t e = hipStreamSynchronize(st);
    hipFree(part);
    if (s != BNOS_OK) return s;
    if (e != hipSuccess) { set_error(hipGetErrorString(e)); return BNOS_E_DEVICE; }
    return BNOS_OK;
}
