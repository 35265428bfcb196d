// Local-score table build on the device: data ingest, parent-set
// enumeration, contingency counting in LDS and the BDeu + pairwise-prior
// score (Sec. II Eq. (3); Sec. III.A Eq. (4); Sec. IV Eq. (9)-(10)).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <set>
#include <string>
#include <vector>

#include "bnos_internal.h"

namespace bnos {

// ------------------------------------------------------------------ errors, handles

static thread_local std::string g_err;
static std::mutex g_handles_mu;
static std::set<const TableT *> g_handles;

void set_error(const std::string &msg) { g_err = msg; }

bool handle_live(const TableT *t)
{
    std::lock_guard<std::mutex> lk(g_handles_mu);
    return t && g_handles.count(t) && t->magic == kMagic;
}

void register_handle(TableT *t)
{
    std::lock_guard<std::mutex> lk(g_handles_mu);
    g_handles.insert(t);
}

void unregister_handle(TableT *t)
{
    std::lock_guard<std::mutex> lk(g_handles_mu);
    g_handles.erase(t);
}

int64_t TableT::device_bytes() const
{
    return (int64_t)n * S_pad * (int64_t)(sizeof(uint64_t) + sizeof(float)) + (int64_t)n * N_pad +
           (int64_t)n * (int64_t)(sizeof(int32_t) + n * sizeof(double) + 5 * sizeof(double)) + 64 * 8 * 8 +
           part_bytes + (int64_t)n * (S_pad / 256) * 8 + (int64_t)n * (S_pad / 64) * 8 +
           (int64_t)n * (S_pad / 4) * 8 + (int64_t)n * (S_pad / 256) * 4 + (int64_t)n * kBoundSlots * 12;
}

// ------------------------------------------------------------------ device helpers

// Orders LDS traffic of one wavefront between phases (zero / count / read).
__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Mask over the n-1 candidate slots -> mask over node ids: a zero bit is
// inserted at position `node` (slot s < node is node s, slot s >= node is s+1).
__device__ __forceinline__ uint64_t slot_to_node_mask(uint64_t m, int node)
{
    uint64_t lo = m & ((1ull << node) - 1ull);
    uint64_t hi = (node >= 63) ? 0ull : ((m >> node) << (node + 1));
    return hi | lo;
}

// The e-th mask, in ascending numeric order, among masks over `bits` bits with
// at most K set bits.  nsets[b*8 + k] = number of masks over b bits with <= k
// set bits; the masks whose top bit is clear come first.
__device__ __forceinline__ uint64_t unrank_ascending(int64_t e, int bits, int K,
                                                      const int64_t *__restrict__ nsets)
{
    uint64_t m = 0;
    int k = K;
    for (int b = bits - 1; b >= 0 && k > 0; --b) {
        int64_t c = nsets[b * 8 + k];
        if (e >= c) {
            m |= 1ull << b;
            e -= c;
            --k;
        }
    }
    return m;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Parent members of a node mask, ascending, with the cell weights of the
// counting layout: cell = x_child + r_child * sum_t x_{m_t} * prod_{t'>t} r_{m_t'}.
struct Members {
    int id[kMaxK];
    int w[kMaxK];
    int cnt;
    int q;
};

__device__ __forceinline__ Members decode_members(uint64_t mask, int r_child,
                                                  const int32_t *__restrict__ ar)
{
    Members M;
    M.cnt = 0;
    uint64_t m = mask;
#pragma unroll
    for (int t = 0; t < kMaxK; ++t) {
        M.id[t] = 0;
        M.w[t] = 0;
        if (m) {
            int b = __builtin_ctzll(m);
            m &= m - 1;
            M.id[t] = b;
            M.cnt = t + 1;
        }
    }
    int acc = r_child;
#pragma unroll
    for (int t = kMaxK - 1; t >= 0; --t) {
        if (t < M.cnt) {
            M.w[t] = acc;
            acc *= ar[M.id[t]];
        }
    }
    M.q = acc / r_child;
    return M;
}

// Histogram of the N samples into hist[0 .. q*r) (one wavefront; hist is this
// wavefront's private LDS region).  Each lane takes 4 consecutive samples per
// step from 32-bit loads of the column-major data.
__device__ __forceinline__ void wave_count(const uint8_t *__restrict__ data, int64_t N, int64_t N_pad,
                                           int child, const Members &M, int cells, uint32_t *hist,
                                           int lane)
{
    for (int c = lane; c < cells; c += 64) hist[c] = 0u;
    wave_lds_sync();
    const uint32_t *colc = reinterpret_cast<const uint32_t *>(data + (int64_t)child * N_pad);
    const uint32_t *colm[kMaxK];
#pragma unroll
    for (int t = 0; t < kMaxK; ++t)
        colm[t] = reinterpret_cast<const uint32_t *>(data + (int64_t)M.id[t] * N_pad);
    for (int64_t base = (int64_t)lane * 4; base < N; base += 256) {
        uint32_t xc = colc[base >> 2];
        uint32_t xm[kMaxK];
#pragma unroll
        for (int t = 0; t < kMaxK; ++t) xm[t] = (t < M.cnt) ? colm[t][base >> 2] : 0u;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            int cell = (int)((xc >> (8 * b)) & 0xffu);
#pragma unroll
            for (int t = 0; t < kMaxK; ++t) cell += M.w[t] * (int)((xm[t] >> (8 * b)) & 0xffu);
            if (base + b < N) atomicAdd(&hist[cell], 1u);
        }
    }
    wave_lds_sync();
}

// ------------------------------------------------------------------ kernels

// Row-major int8 [N][n] -> column-major uint8 [n][N_pad] (padding already zero).
__global__ void k_ingest(const int8_t *__restrict__ src, int64_t N, int n, int64_t N_pad,
                         uint8_t *__restrict__ dst)
{
    int64_t total = N * n;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        int64_t t = g / n;
        int v = (int)(g - t * n);
        dst[(int64_t)v * N_pad + t] = (uint8_t)src[g];
    }
}

// Device-resident input: counts the states outside [0, arity) (the host input
// is checked on the host instead).
__global__ void k_check_states(const int8_t *__restrict__ src, int64_t N, int n, const int32_t *__restrict__ ar,
                               unsigned *__restrict__ bad)
{
    const int64_t total = N * n;
    unsigned c = 0;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total;
         g += (int64_t)gridDim.x * blockDim.x) {
        const int x = src[g];
        const int v = (int)(g % n);
        c += (x < 0 || x >= ar[v]) ? 1u : 0u;
    }
    if (c) atomicAdd(bad, c);
}

// Prior term in nats per (child i, parent m): ln(10) * 100 * (R - 0.5)^3 (Eq. (10),
// a log10 quantity in Eq. (9)); R = (1 + w)/2 in mode 0, R given in mode 1.
__global__ void k_prior(const float *__restrict__ src, int n, int mode, double *__restrict__ dst)
{
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n * n) return;
    int i = g / n, m = g - (g / n) * n;
    double v = 0.0;
    if (src && i != m) {
        double x = (double)src[g];
        double R = (mode == 0) ? 0.5 * (1.0 + x) : x;
        double d = R - 0.5;
        v = 2.302585092994045684 * 100.0 * d * d * d;
    }
    dst[g] = v;
}

// lut[row][c] = lnG(c + a) - lnG(a), a = ess / den[row], c = 0..N (FP64 ocml lgamma).
__global__ void k_lut(const int32_t *__restrict__ den, int rows, int64_t N, double ess, double *__restrict__ lut)
{
    const int64_t total = (int64_t)rows * (N + 1);
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int row = (int)(g / (N + 1));
        const int64_t c = g - (int64_t)row * (N + 1);
        const double a = ess / (double)den[row];
        lut[g] = lgamma((double)c + a) - lgamma(a);
    }
}

// Rank of a mask among the masks over `bits` bits with at most K set bits, in
// ascending numeric order (the inverse of unrank_ascending).
__device__ __forceinline__ int64_t rank_ascending(uint64_t m, int bits, int K, const int64_t *__restrict__ nsets)
{
    int64_t r = 0;
    int k = K;
    for (int b = bits - 1; b >= 0; --b)
        if ((m >> b) & 1ull) {
            r += nsets[b * 8 + k];
            --k;
        }
    return r;
}

// A node subset U (|U| <= K+1) as the joint histogram sees it: members
// ascending, their arities, and the stride of each member's digit in the joint
// cell index (the last member fastest).
struct Subset {
    int u[kMaxK + 1], r[kMaxK + 1], stride[kMaxK + 1];
    uint32_t magic[kMaxK + 1];   // floor(2^32 / r) + 1: quotients by r of cell indices (<= 2^14) by multiply-high
    int j;        // members
    int cells;    // product of the members' arities
};

// q = x / r and x - q r for 0 <= x <= 2^14 and 1 <= r <= 255: with m = floor(2^32/r) + 1,
// x m / 2^32 exceeds x / r by less than x / 2^32 <= 2^-18, too little to carry a
// fraction of at most (r - 1) / r past the next integer.  q r <= x fits a 24-bit multiply.
__device__ __forceinline__ void divmod_small(int x, int r, uint32_t magic, int &q, int &rem)
{
    q = (r == 1) ? x : (int)__umulhi((uint32_t)x, magic);
    rem = x - (int)__umul24((uint32_t)q, (uint32_t)r);
}

__device__ __forceinline__ Subset decode_subset(uint64_t U, const int32_t *__restrict__ ar)
{
    Subset S;
    S.j = 0;
    uint64_t m = U;
#pragma unroll
    for (int t = 0; t <= kMaxK; ++t) {
        S.u[t] = 0;
        S.r[t] = 1;
        if (m) {
            S.u[t] = __builtin_ctzll(m);
            m &= m - 1;
            S.r[t] = ar[S.u[t]];
            S.j = t + 1;
        }
        S.magic[t] = S.r[t] > 1 ? (uint32_t)(0x100000000ull / (uint64_t)S.r[t]) + 1u : 0u;
    }
    int cells = 1;
#pragma unroll
    for (int t = kMaxK; t >= 0; --t) {
        S.stride[t] = cells;
        if (t < S.j) cells *= S.r[t];
    }
    S.cells = cells;
    return S;
}

// Joint histogram of U's variables over the N samples into hist[0 .. cells)
// (one wavefront, its private LDS region); each lane takes 4 consecutive
// samples per step from 32-bit loads of the column-major data.  A cell's byte
// offset is the sum of each member's state times its stride in bytes: states
// are below 256 and cells number at most 2^14, so every product and the sum
// fit 24-bit multiplies.  Whole 256-sample steps need no per-sample check;
// only the last, partial step tests each sample against N.
// (J = the number of members, a constant of the instance.)
template <int J>
__device__ __forceinline__ void joint_histogram_j(const uint8_t *__restrict__ data, int64_t N, int64_t N_pad,
                                                  const Subset &S, uint32_t *hist, int lane)
{
    const uint32_t *col[J];
    uint32_t st4[J];
#pragma unroll
    for (int t = 0; t < J; ++t) {
        col[t] = reinterpret_cast<const uint32_t *>(data + (int64_t)S.u[t] * N_pad);
        st4[t] = (uint32_t)S.stride[t] * 4u;
    }
    char *hb = reinterpret_cast<char *>(hist);
    auto offset_of = [&](const uint32_t (&x)[J], int b) -> uint32_t {
        uint32_t off = 0;
#pragma unroll
        for (int t = 0; t < J; ++t) off += __umul24((x[t] >> (8 * b)) & 0xffu, st4[t]);
        return off;
    };
    const int64_t whole = N & ~(int64_t)255;
    for (int64_t base = (int64_t)lane * 4; base < whole; base += 256) {
        uint32_t x[J];
#pragma unroll
        for (int t = 0; t < J; ++t) x[t] = col[t][base >> 2];
#pragma unroll
        for (int b = 0; b < 4; ++b) atomicAdd(reinterpret_cast<uint32_t *>(hb + offset_of(x, b)), 1u);
    }
    const int64_t base = whole + (int64_t)lane * 4;
    if (base < N) {
        uint32_t x[J];
#pragma unroll
        for (int t = 0; t < J; ++t) x[t] = col[t][base >> 2];
#pragma unroll
        for (int b = 0; b < 4; ++b)
            if (base + b < N) atomicAdd(reinterpret_cast<uint32_t *>(hb + offset_of(x, b)), 1u);
    }
}

__device__ __forceinline__ void joint_histogram(const uint8_t *__restrict__ data, int64_t N, int64_t N_pad,
                                                const Subset &S, uint32_t *hist, int lane)
{
    for (int c = lane; c < S.cells; c += 64) hist[c] = 0u;
    wave_lds_sync();
    switch (S.j) {                 // uniform: one subset per wavefront
    case 1: joint_histogram_j<1>(data, N, N_pad, S, hist, lane); break;
    case 2: joint_histogram_j<2>(data, N, N_pad, S, hist, lane); break;
    case 3: joint_histogram_j<3>(data, N, N_pad, S, hist, lane); break;
    case 4: joint_histogram_j<4>(data, N, N_pad, S, hist, lane); break;
    case 5: joint_histogram_j<5>(data, N, N_pad, S, hist, lane); break;
    case 6: joint_histogram_j<6>(data, N, N_pad, S, hist, lane); break;
    default: joint_histogram_j<kMaxK + 1>(data, N, N_pad, S, hist, lane); break;
    }
    wave_lds_sync();
}

// Member c of U as the child of the family (u_c, U \ {u_c}): its id, arity,
// digit stride and the family's number of parent configurations (the cells
// divided by the arity), selected without indexing the arrays by c.
__device__ __forceinline__ void subset_member(const Subset &S, int c, int &node, int &ri, int &sci, int &q)
{
    node = 0;
    ri = 1;
    sci = 1;
    uint32_t mag = 0;
#pragma unroll
    for (int t = 0; t <= kMaxK; ++t)
        if (t == c) {
            node = S.u[t];
            ri = S.r[t];
            sci = S.stride[t];
            mag = S.magic[t];
        }
    int rem;
    divmod_small(S.cells, ri, mag, q, rem);
}

// Joint cell of parent configuration k of the family whose child is member c,
// with the child's state 0: k's digits run over the parents ascending, the
// last one fastest (the lowest id most significant, as in the per-family
// count layout); the child's state x adds x * (c's stride).
__device__ __forceinline__ int family_base(const Subset &S, int c, int k)
{
    int rest = k, J = 0;
#pragma unroll
    for (int t = kMaxK; t >= 0; --t) {
        if (t < S.j && t != c) {
            int q, d;
            divmod_small(rest, S.r[t], S.magic[t], q, d);
            J += (int)__umul24((uint32_t)d, (uint32_t)S.stride[t]);
            rest = q;
        }
    }
    return J;
}

// One wavefront per node subset U, |U| = 1 .. K+1 (U's rank + 1 among the
// masks over n bits with at most K+1 bits): the joint histogram of U's
// variables over the N samples, then for every member i of U the local score
// of the family (i, U \ {i}) from it -- that family's N_ijk are the joint
// counts with i's state as the child state -- stored at U \ {i}'s entry of i's
// row.  Counting once per U instead of once per family cuts the sample visits
// by the mean family size (about 5x at K = 4).  The BDeu terms are summed in
// the same order as in k_build (parent configurations k by lane, the lowest id
// most significant; child states in order; the same butterfly), so the stored
// scores are the same, bit for bit.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_build_joint(
    const uint8_t *__restrict__ data, int64_t N, int64_t N_pad, const int32_t *__restrict__ ar,
    const double *__restrict__ prior, const int64_t *__restrict__ nsets, int n, int K, double ess,
    double log_gamma, int64_t n_subsets, int64_t S_pad, int cells_cap, const int32_t *__restrict__ lut_row,
    const double *__restrict__ lut, uint64_t *__restrict__ masks, float *__restrict__ scores)
{
    extern __shared__ uint32_t lds_hist[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: the subset's decode stays scalar
    const int lane = threadIdx.x & 63;
    uint32_t *hist = lds_hist + wave * cells_cap;
    for (int64_t g = (int64_t)blockIdx.x * WAVES + wave; g < n_subsets; g += (int64_t)gridDim.x * WAVES) {
        const uint64_t U = unrank_ascending(g + 1, n, K + 1, nsets);
        const Subset Sb = decode_subset(U, ar);
        const int j = Sb.j, cells = Sb.cells;
        joint_histogram(data, N, N_pad, Sb, hist, lane);
        // one family per member
        for (int c = 0; c < j; ++c) {
            int node, ri, sci, q;
            subset_member(Sb, c, node, ri, sci, q);
            const double *L_ijk = lut + (int64_t)lut_row[cells] * (N + 1);
            const double *L_ik = lut + (int64_t)lut_row[q] * (N + 1);
            double acc = 0.0;
            for (int k = lane; k < q; k += 64) {
                const int J = family_base(Sb, c, k);
                uint32_t nik = 0;
                double part = 0.0;
                for (int x = 0; x < ri; ++x) {
                    const uint32_t cnt = hist[J + (int)__umul24((uint32_t)x, (uint32_t)sci)];
                    nik += cnt;
                    if (cnt) part += L_ijk[cnt];
                }
                if (nik) part += -L_ik[nik];
                acc += part;
            }
            acc = wave_sum_f64(acc);
            if (lane == 0) {
                const uint64_t pm = U & ~(1ull << node);
                double sc = acc + (double)(j - 1) * log_gamma;
#pragma unroll
                for (int t = 0; t <= kMaxK; ++t)
                    if (t < j && t != c) sc += prior[(int64_t)node * n + Sb.u[t]];
                const uint64_t slot = (pm & ((1ull << node) - 1ull)) | (node >= 63 ? 0ull : ((pm >> (node + 1)) << node));
                const int64_t e = (int64_t)node * S_pad + rank_ascending(slot, n - 1, K, nsets);
                masks[e] = pm;
                scores[e] = (float)sc;   // round to nearest even
            }
        }
        wave_lds_sync();   // every lane has read hist before the next subset clears it
    }
}

// Padding entries e in [S, S_pad) of every row: (~0, -inf), which no
// predecessor set can contain.
__global__ void k_pad_rows(int n, int64_t S, int64_t S_pad, uint64_t *__restrict__ masks, float *__restrict__ scores)
{
    const int64_t per = S_pad - S;
    const int64_t total = (int64_t)n * per;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < total; g += (int64_t)gridDim.x * blockDim.x) {
        const int64_t node = g / per;
        const int64_t e = node * S_pad + S + (g - node * per);
        masks[e] = ~0ull;
        scores[e] = -INFINITY;
    }
}

// One wavefront per (node, entry): enumerate the entry's parent set, count
// N_ijk in LDS, reduce the BDeu terms in FP64, add the structure penalty and
// the prior terms, store (mask, FP32 score).  Padding entries get (~0, -inf),
// which no predecessor set can contain.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_build(
    const uint8_t *__restrict__ data, int64_t N, int64_t N_pad, const int32_t *__restrict__ ar,
    const double *__restrict__ prior, const int64_t *__restrict__ nsets, int n, int K, double ess,
    double log_gamma, int64_t S, int64_t S_pad, int cells_cap, const int32_t *__restrict__ lut_row,
    const double *__restrict__ lut, uint64_t *__restrict__ masks, float *__restrict__ scores)
{
    extern __shared__ uint32_t lds_hist[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint32_t *hist = lds_hist + wave * cells_cap;
    const int64_t total = (int64_t)n * S_pad;
    for (int64_t g = (int64_t)blockIdx.x * WAVES + wave; g < total; g += (int64_t)gridDim.x * WAVES) {
        const int node = (int)(g / S_pad);
        const int64_t e = g - (int64_t)node * S_pad;
        if (e >= S) {
            if (lane == 0) {
                masks[g] = ~0ull;
                scores[g] = -INFINITY;
            }
            continue;
        }
        const uint64_t mask = slot_to_node_mask(unrank_ascending(e, n - 1, K, nsets), node);
        const int r = ar[node];
        Members M = decode_members(mask, r, ar);
        const int cells = M.q * r;
        wave_count(data, N, N_pad, node, M, cells, hist, lane);

        const double a_ijk = ess / (double)cells;
        const double a_ik = ess / (double)M.q;
        double acc = 0.0;
        if (lut) {
            // lnG(c + a) - lnG(a) looked up per count (same FP64 values as computed below)
            const double *L_ijk = lut + (int64_t)lut_row[cells] * (N + 1);
            const double *L_ik = lut + (int64_t)lut_row[M.q] * (N + 1);
            for (int k = lane; k < M.q; k += 64) {
                uint32_t nik = 0;
                double part = 0.0;
                for (int j = 0; j < r; ++j) {
                    const uint32_t c = hist[k * r + j];
                    nik += c;
                    if (c) part += L_ijk[c];
                }
                if (nik) part += -L_ik[nik];
                acc += part;
            }
        } else {
            const double lg_ijk = lgamma(a_ijk);
            const double lg_ik = lgamma(a_ik);
            for (int k = lane; k < M.q; k += 64) {
                uint32_t nik = 0;
                double part = 0.0;
                for (int j = 0; j < r; ++j) {
                    const uint32_t c = hist[k * r + j];
                    nik += c;
                    if (c) part += lgamma((double)c + a_ijk) - lg_ijk;
                }
                if (nik) part += -(lgamma(a_ik + (double)nik) - lg_ik);
                acc += part;
            }
        }
        acc = wave_sum_f64(acc);
        wave_lds_sync();   // every lane has read hist before the next entry clears it
        if (lane == 0) {
            double s = acc + (double)M.cnt * log_gamma;
#pragma unroll
            for (int t = 0; t < kMaxK; ++t)
                if (t < M.cnt) s += prior[(int64_t)node * n + M.id[t]];
            masks[g] = mask;
            scores[g] = (float)s;   // round to nearest even
        }
    }
}

// Per-node static features of the learned proposal: prior terms summed as
// child (row) and as parent (column), and max, mean and population standard
// deviation of the node's stored FP32 scores (FP64 sums, fixed tree).
__global__ __launch_bounds__(1024) void k_node_stats(const float *__restrict__ scores, int64_t S, int64_t S_pad,
                                                     const double *__restrict__ prior, int n,
                                                     double *__restrict__ out)
{
    __shared__ double s_a[1024], s_b[1024];
    const int node = blockIdx.x;
    const int tid = threadIdx.x;
    const float *row = scores + (int64_t)node * S_pad;
    double mx = -INFINITY, sum = 0.0;
    for (int64_t e = tid; e < S; e += 1024) {
        const double v = row[e];
        mx = v > mx ? v : mx;
        sum += v;
    }
    s_a[tid] = mx;
    s_b[tid] = sum;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (tid < w) {
            s_a[tid] = s_a[tid + w] > s_a[tid] ? s_a[tid + w] : s_a[tid];
            s_b[tid] += s_b[tid + w];
        }
        __syncthreads();
    }
    const double gmax = s_a[0];
    const double mean = s_b[0] / (double)S;
    __syncthreads();
    double sq = 0.0;
    for (int64_t e = tid; e < S; e += 1024) {
        const double d = (double)row[e] - mean;
        sq += d * d;
    }
    s_b[tid] = sq;
    __syncthreads();
    for (int w = 512; w >= 1; w >>= 1) {
        if (tid < w) s_b[tid] += s_b[tid + w];
        __syncthreads();
    }
    if (tid == 0) {
        double rs = 0.0, cs = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == node) continue;
            rs += prior[(int64_t)node * n + m];
            cs += prior[(int64_t)m * n + node];
        }
        double *o = out + (int64_t)node * 5;
        o[0] = rs;
        o[1] = cs;
        o[2] = gmax;
        o[3] = mean;
        o[4] = sqrt(s_b[0] / (double)S);
    }
}

// AND of the masks of every 256-entry tile and of its four 64-entry sub-tiles,
// and the tile's largest score (one wavefront per tile), stored at the tile's
// summary place (summary_pos: row_tiles tiles per row, in sum_chunks chunks of
// sum_steps steps).
__global__ __launch_bounds__(256) void k_tile_and(const uint64_t *__restrict__ masks,
                                                  const float *__restrict__ scores, int64_t tiles,
                                                  int64_t row_tiles, int64_t sum_chunks, int sum_steps,
                                                  uint64_t *__restrict__ tand, uint64_t *__restrict__ tsub,
                                                  float *__restrict__ tmax)
{
    const int64_t tile = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (tile >= tiles) return;                       // uniform per wavefront
    const int64_t row = tile / row_tiles, r = tile - row * row_tiles;
    const int64_t at = row * row_tiles + summary_pos(r >> 2, (int)(r & 3), sum_chunks, sum_steps);
    const uint64_t *p = masks + tile * 256 + lane * 4;
    const float *q = scores + tile * 256 + lane * 4;
    uint64_t v = p[0] & p[1] & p[2] & p[3];
    float x = fmaxf(fmaxf(q[0], q[1]), fmaxf(q[2], q[3]));
    // lanes 16s .. 16s+15 hold sub-tile s (entries 64s .. 64s+63)
#pragma unroll
    for (int off = 1; off <= 8; off <<= 1) v &= (uint64_t)__shfl_xor((unsigned long long)v, off, 64);
    if ((lane & 15) == 0) tsub[at * 4 + (lane >> 4)] = v;
#pragma unroll
    for (int off = 16; off <= 32; off <<= 1) v &= (uint64_t)__shfl_xor((unsigned long long)v, off, 64);
#pragma unroll
    for (int off = 1; off <= 32; off <<= 1) x = fmaxf(x, __shfl_xor(x, off, 64));
    if (lane == 0) {
        tand[at] = v;
        tmax[at] = x;
    }
}

// Index in a row of the singleton {slot s}: every mask below 1 << s, i.e.
// every set of at most K slots below s, comes first.
__device__ __forceinline__ int64_t singleton_index(int s, int K)
{
    int64_t c = 1, tot = 1;
    for (int k = 1; k <= K; ++k) {
        c = c * (s - k + 1) / k;
        tot += c;
    }
    return tot;
}

// The score bound's candidates of each row (one block per node), in
// kBoundSlots slots: slot s < n - 1 the singleton of slot s (K >= 1), slot 63
// the empty set, then the listed top entries: with M the row's largest score
// among the sets of two or more members, the entries of those sets within b
// quarter-nats of M, for the largest b that keeps them to at most
// kBoundCands.  Unused slots hold (~0, -inf), which no order can use.  The
// list's order is that of the appends and does not matter: only the entries'
// values are used.
constexpr int kBoundBins = 1024;
__global__ __launch_bounds__(1024) void k_bound_cands(const uint64_t *__restrict__ masks,
                                                      const float *__restrict__ scores, int n, int K, int64_t S,
                                                      int64_t S_pad, uint64_t *__restrict__ cmask,
                                                      float *__restrict__ cscore)
{
    __shared__ float s_max[1024 / 64];
    __shared__ unsigned s_hist[kBoundBins];
    __shared__ unsigned s_cut, s_cnt;
    const int node = blockIdx.x;
    const int tid = threadIdx.x;
    const uint64_t *mr = masks + (int64_t)node * S_pad;
    const float *sr = scores + (int64_t)node * S_pad;
    float mx = -INFINITY;
    for (int64_t e = tid; e < S; e += 1024)
        if (__popcll(mr[e]) >= 2) mx = fmaxf(mx, sr[e]);
#pragma unroll
    for (int off = 1; off <= 32; off <<= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    if ((tid & 63) == 0) s_max[tid >> 6] = mx;
    for (int i = tid; i < kBoundBins; i += 1024) s_hist[i] = 0u;
    __syncthreads();
    float M = s_max[0];
    for (int w = 1; w < 1024 / 64; ++w) M = fmaxf(M, s_max[w]);
    for (int64_t e = tid; e < S; e += 1024) {
        if (__popcll(mr[e]) < 2) continue;
        const float d = (M - sr[e]) * 4.0f;
        if (d < (float)kBoundBins) atomicAdd(&s_hist[(int)d], 1u);
    }
    __syncthreads();
    if (tid == 0) {
        unsigned acc = 0u;
        int b = 0;
        while (b < kBoundBins && acc + s_hist[b] <= (unsigned)kBoundCands) acc += s_hist[b++];
        s_cut = (unsigned)b;
        s_cnt = 0u;
    }
    __syncthreads();
    const float cut = (float)s_cut;
    if (tid < 64) {
        uint64_t fm = ~0ull;
        float fx = -INFINITY;
        if (tid == 63) {
            fm = 0ull;
            fx = sr[0];
        } else if (tid < n - 1 && K >= 1) {
            fm = 1ull << (tid < node ? tid : tid + 1);
            fx = sr[singleton_index(tid, K)];
        }
        cmask[(int64_t)node * kBoundSlots + tid] = fm;
        cscore[(int64_t)node * kBoundSlots + tid] = fx;
    }
    uint64_t *cm = cmask + (int64_t)node * kBoundSlots + 64;
    float *cs = cscore + (int64_t)node * kBoundSlots + 64;
    for (int64_t e = tid; e < S; e += 1024) {
        const uint64_t m = mr[e];
        if (__popcll(m) < 2) continue;
        const float x = sr[e];
        if ((M - x) * 4.0f < cut) {
            const unsigned k = atomicAdd(&s_cnt, 1u);
            cm[k] = m;
            cs[k] = x;
        }
    }
    __syncthreads();
    for (int k = (int)s_cnt + tid; k < kBoundCands; k += 1024) {
        cm[k] = ~0ull;
        cs[k] = -INFINITY;
    }
}

// The slot-space mask (the node's own bit removed: slot s is node s below the
// node, node s + 1 above it) of the first entry of every 4-entry group of each
// row, for the scoring pass that computes the other masks; for padding, the
// mask of slot n - 1, which no row holds and no step from it leaves.
__global__ __launch_bounds__(256) void k_anchor(const uint64_t *__restrict__ masks, int n, int64_t S_pad,
                                                uint64_t *__restrict__ anchor)
{
    const int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t per_row = S_pad / 4;
    if (g >= (int64_t)n * per_row) return;
    const int node = (int)(g / per_row);
    const uint64_t m = masks[g * 4];
    const uint64_t low = (1ull << node) - 1ull;
    anchor[g] = (m == ~0ull) ? (1ull << (n - 1)) : ((m & low) | ((m >> 1) & ~low));
}

// Counts for explicit (node, parent mask) queries, with the build's counting code.
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_counts(
    const uint8_t *__restrict__ data, int64_t N, int64_t N_pad, const int32_t *__restrict__ ar,
    int Q, const int32_t *__restrict__ qnode, const uint64_t *__restrict__ qmask,
    const int64_t *__restrict__ qoff, int cells_cap, uint32_t *__restrict__ out)
{
    extern __shared__ uint32_t lds_hist[];
    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    uint32_t *hist = lds_hist + wave * cells_cap;
    for (int qi = blockIdx.x * WAVES + wave; qi < Q; qi += gridDim.x * WAVES) {
        const int node = qnode[qi];
        const int r = ar[node];
        Members M = decode_members(qmask[qi], r, ar);
        const int cells = M.q * r;
        wave_count(data, N, N_pad, node, M, cells, hist, lane);
        for (int c = lane; c < cells; c += 64) out[qoff[qi] + c] = hist[c];
        wave_lds_sync();
    }
}

// The same queries answered by the joint-histogram path of the default build
// (k_build_joint): the histogram of U = parents + node, read out as the
// family's cells (parent configuration k, the lowest id most significant, then
// the child state).
template <int WAVES>
__global__ __launch_bounds__(WAVES * 64) void k_counts_joint(
    const uint8_t *__restrict__ data, int64_t N, int64_t N_pad, const int32_t *__restrict__ ar,
    int Q, const int32_t *__restrict__ qnode, const uint64_t *__restrict__ qmask,
    const int64_t *__restrict__ qoff, int cells_cap, uint32_t *__restrict__ out)
{
    extern __shared__ uint32_t lds_hist[];
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: the subset's decode stays scalar
    const int lane = threadIdx.x & 63;
    uint32_t *hist = lds_hist + wave * cells_cap;
    for (int qi = blockIdx.x * WAVES + wave; qi < Q; qi += gridDim.x * WAVES) {
        const int child = qnode[qi];
        const uint64_t U = qmask[qi] | (1ull << child);
        const Subset Sb = decode_subset(U, ar);
        joint_histogram(data, N, N_pad, Sb, hist, lane);
        const int c = __popcll(U & ((1ull << child) - 1ull));       // the child's place among U's members
        int node, ri, sci, q;
        subset_member(Sb, c, node, ri, sci, q);
        for (int k = lane; k < q; k += 64) {
            const int J = family_base(Sb, c, k);
            for (int x = 0; x < ri; ++x)
                out[qoff[qi] + (int64_t)k * ri + x] = hist[J + (int)__umul24((uint32_t)x, (uint32_t)sci)];
        }
        wave_lds_sync();
    }
}

// ------------------------------------------------------------------ host side

static int64_t binom_host(int a, int b)
{
    if (b < 0 || a < 0 || b > a) return 0;
    int64_t r = 1;
    for (int t = 1; t <= b; ++t) r = r * (a - b + t) / t;
    return r;
}

static int64_t sets_upto(int m, int K)
{
    int64_t s = 0;
    for (int j = 0; j <= K && j <= m; ++j) s += binom_host(m, j);
    return s;
}

static int waves_for_cells(int cells_cap) { return cells_cap <= 4096 ? 4 : 1; }

template <int W>
static hipError_t launch_build(TableT *t, hipStream_t st, int cells_cap, const int32_t *lut_row, const double *lut)
{
    int64_t total = (int64_t)t->n * t->S_pad;
    int64_t blocks = (total + W - 1) / W;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    size_t lds = (size_t)W * cells_cap * sizeof(uint32_t);
    hipLaunchKernelGGL(k_build<W>, dim3((unsigned)blocks), dim3(W * 64), lds, st, t->d_data, t->N,
                       t->N_pad, t->d_ar, t->d_prior, t->d_nsets, t->n, t->K, t->ess, t->log_gamma,
                       t->S, t->S_pad, cells_cap, lut_row, lut, t->d_masks, t->d_scores);
    return hipGetLastError();
}

template <int W>
static hipError_t launch_build_joint(TableT *t, hipStream_t st, int cells_cap, const int32_t *lut_row,
                                     const double *lut)
{
    const int64_t subsets = sets_upto(t->n, t->K + 1) - 1;
    int64_t blocks = (subsets + W - 1) / W;
    if (blocks > (1 << 22)) blocks = 1 << 22;
    size_t lds = (size_t)W * cells_cap * sizeof(uint32_t);
    hipLaunchKernelGGL(k_build_joint<W>, dim3((unsigned)blocks), dim3(W * 64), lds, st, t->d_data, t->N,
                       t->N_pad, t->d_ar, t->d_prior, t->d_nsets, t->n, t->K, t->ess, t->log_gamma, subsets,
                       t->S_pad, cells_cap, lut_row, lut, t->d_masks, t->d_scores);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || t->S_pad == t->S) return e;
    const int64_t pad = (int64_t)t->n * (t->S_pad - t->S);
    hipLaunchKernelGGL(k_pad_rows, dim3((unsigned)std::min<int64_t>((pad + 255) / 256, 1 << 16)), dim3(256), 0, st,
                       t->n, t->S, t->S_pad, t->d_masks, t->d_scores);
    return hipGetLastError();
}

static int cells_cap_for(int max_cells)
{
    int c = 64;
    while (c < max_cells) c <<= 1;
    return c;
}

static void free_device(TableT *t)
{
    hipFree(t->d_data);
    hipFree(t->d_ar);
    hipFree(t->d_prior);
    hipFree(t->d_nsets);
    hipFree(t->d_masks);
    hipFree(t->d_scores);
    hipFree(t->d_nstat);
    hipFree(t->d_tand);
    hipFree(t->d_tsub);
    hipFree(t->d_anchor);
    hipFree(t->d_tmax);
    hipFree(t->d_cmask);
    hipFree(t->d_cscore);
    hipFree(t->d_part);
    for (auto e : t->ev_start) hipEventDestroy(e);
    for (auto e : t->ev_stop) hipEventDestroy(e);
}

}  // namespace bnos

using namespace bnos;

extern "C" const char *bnos_last_error(void) { return g_err.c_str(); }

extern "C" int32_t bnos_version(void) { return 100; }

extern "C" bnos_status bnos_build_score_table(const int8_t *data, int64_t N, int32_t n,
                                              const int32_t *arities, int32_t K, double ess,
                                              const float *prior, const bnos_build_opts *opts,
                                              void *stream, bnos_table *out)
{
    if (!out) { set_error("out is NULL"); return BNOS_E_INVALID; }
    if (!arities) { set_error("arities is NULL"); return BNOS_E_INVALID; }
    if (N < 0 || N > 2147483647LL) { set_error("N outside [0, 2^31-1]"); return BNOS_E_RANGE; }
    if (N > 0 && !data) { set_error("data is NULL"); return BNOS_E_INVALID; }
    if (n < 1 || n > 64) { set_error("n outside [1, 64]"); return BNOS_E_RANGE; }
    if (K < 0 || K > n - 1 || K > kMaxK) { set_error("K outside [0, min(n-1, 6)]"); return BNOS_E_RANGE; }
    if (!(ess > 0.0) || !std::isfinite(ess)) { set_error("ess must be finite and > 0"); return BNOS_E_INVALID; }
    bnos_build_opts o;
    std::memset(&o, 0, sizeof(o));
    if (opts) o = *opts;
    for (int r = 0; r < 4; ++r)
        if (o.reserved[r] != 0) { set_error("opts.reserved must be zero"); return BNOS_E_INVALID; }
    if (o.data_on_device != 0 && o.data_on_device != 1) { set_error("data_on_device must be 0 or 1"); return BNOS_E_INVALID; }
    const bool dev_data = o.data_on_device == 1;
    if (o.prior_mode != 0 && o.prior_mode != 1) { set_error("prior_mode must be 0 or 1"); return BNOS_E_INVALID; }
    if (o.count_mode != 0 && o.count_mode != 1) { set_error("count_mode must be 0 or 1"); return BNOS_E_INVALID; }
    if (!std::isfinite(o.log_gamma)) { set_error("log_gamma must be finite"); return BNOS_E_INVALID; }
    for (int v = 0; v < n; ++v)
        if (arities[v] < 1 || arities[v] > 255) { set_error("arity outside [1, 255]"); return BNOS_E_RANGE; }
    for (int64_t t = 0; t < (dev_data ? 0 : N); ++t)        // device data: checked on the device
        for (int v = 0; v < n; ++v) {
            int x = data[t * n + v];
            if (x < 0 || x >= arities[v]) {
                char buf[128];
                std::snprintf(buf, sizeof buf, "state %d of node %d in sample %lld is outside [0, %d)", x, v,
                              (long long)t, arities[v]);
                set_error(buf);
                return BNOS_E_INVALID;
            }
        }
    if (prior) {
        for (int i = 0; i < n; ++i)
            for (int m = 0; m < n; ++m) {
                if (i == m) continue;
                float x = prior[i * n + m];
                bool ok = std::isfinite(x) && (o.prior_mode == 0 ? (x >= -1.f && x <= 1.f) : (x >= 0.f && x <= 1.f));
                if (!ok) { set_error("prior entry NaN or out of range"); return BNOS_E_INVALID; }
            }
    }
    // Largest contingency table: r_i times the K largest arities among the other nodes.
    int max_cells = 1;
    for (int i = 0; i < n; ++i) {
        std::vector<int> o2;
        for (int m = 0; m < n; ++m) if (m != i) o2.push_back(arities[m]);
        std::sort(o2.rbegin(), o2.rend());
        int64_t c = arities[i];
        for (int j = 0; j < K && j < (int)o2.size(); ++j) c *= o2[j];
        if (c > kMaxCells) { set_error("q_i * r_i above 16384"); return BNOS_E_RANGE; }
        if (c > max_cells) max_cells = (int)c;
    }

    TableT *t = new (std::nothrow) TableT();
    if (!t) { set_error("host allocation failed"); return BNOS_E_NOMEM; }
    t->n = n;
    t->K = K;
    t->N = N;
    t->N_pad = ((N + 255) / 256) * 256;
    if (t->N_pad == 0) t->N_pad = 256;
    t->S = sets_upto(n - 1, K);
    {
        // Rows are padded to a multiple of P * 1024 entries, P the smallest power
        // of two >= the row's 1024-entry steps (and >= a requested chunk
        // length), at most 16; chunk lengths are the powers of two dividing P.
        const int64_t node_steps = (t->S + kEntriesPerStep - 1) / kEntriesPerStep;
        int st = o.chunk_steps;
        if (st != 0 && (st < 1 || st > kMaxStepsPerChunk || (st & (st - 1)) != 0)) {
            set_error("chunk_steps must be 0 or a power of two <= 16");
            delete t;
            return BNOS_E_RANGE;
        }
        int P = 1;
        while (P < kMaxStepsPerChunk && (P < node_steps || P < st)) P <<= 1;
        t->pad_steps = P;
        t->S_pad = ((node_steps + P - 1) / P) * P * kEntriesPerStep;
        if (const char *cap_s = std::getenv("BNOS_MAX_DEVICE_BYTES")) {
            const long long cap = std::atoll(cap_s);
            if (cap > 0 && t->device_bytes() > cap) {
                char buf[160];
                std::snprintf(buf, sizeof buf, "table needs %lld device bytes, above BNOS_MAX_DEVICE_BYTES = %lld",
                              (long long)t->device_bytes(), cap);
                set_error(buf);
                delete t;
                return BNOS_E_NOMEM;
            }
        }
        if (st == 0) {
            // automatic: the length that best fills whole rounds of resident blocks
            // (8 blocks of 256 threads per compute unit) for a single-order pass
            int cus = 256;
            int dev = 0;
            if (hipGetDevice(&dev) == hipSuccess) {
                int v = 0;
                if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
                    cus = v;
            }
            const int64_t slots = (int64_t)cus * 8;
            const int64_t steps_pad = t->S_pad / kEntriesPerStep;
            double best_eff = -1.0;
            st = 1;
            for (int c = 1; c <= P; c <<= 1) {
                const int64_t blocks = (int64_t)n * (steps_pad / c);
                const int64_t rounds = (blocks + slots - 1) / slots;
                const double eff = (double)(n * node_steps) / (double)(rounds * slots * c);
                if (eff >= best_eff - 1e-12) {
                    best_eff = eff;
                    st = c;
                }
            }
        }
        t->chunk_entries = st * kEntriesPerStep;
        t->chunks = (int)(t->S_pad / t->chunk_entries);
    }
    t->max_cells = max_cells;
    t->ess = ess;
    t->log_gamma = o.log_gamma;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);

    auto fail = [&](bnos_status s) {
        free_device(t);
        delete t;
        return s;
    };
    hipError_t e;
    if ((e = hipGetDevice(&t->device)) != hipSuccess) { set_error(std::string("hipGetDevice: ") + hipGetErrorString(e)); return fail(BNOS_E_DEVICE); }
#define ALLOC(ptr, bytes)                                                               \
    if ((e = hipMalloc((void **)&(ptr), (bytes))) != hipSuccess) {                      \
        set_error(std::string("hipMalloc " #ptr ": ") + hipGetErrorString(e));          \
        return fail(e == hipErrorOutOfMemory ? BNOS_E_NOMEM : BNOS_E_DEVICE);           \
    }
    ALLOC(t->d_data, (size_t)n * t->N_pad);
    ALLOC(t->d_ar, sizeof(int32_t) * n);
    ALLOC(t->d_prior, sizeof(double) * n * n);
    ALLOC(t->d_nsets, sizeof(int64_t) * 64 * 8);
    ALLOC(t->d_masks, sizeof(uint64_t) * (size_t)n * t->S_pad);
    ALLOC(t->d_scores, sizeof(float) * (size_t)n * t->S_pad);
    ALLOC(t->d_nstat, sizeof(double) * (size_t)n * 5);
    ALLOC(t->d_tand, sizeof(uint64_t) * (size_t)n * (t->S_pad / 256));
    ALLOC(t->d_tsub, sizeof(uint64_t) * (size_t)n * (t->S_pad / 64));
    ALLOC(t->d_anchor, sizeof(uint64_t) * (size_t)n * (t->S_pad / 4));
    ALLOC(t->d_tmax, sizeof(float) * (size_t)n * (t->S_pad / 256));
    ALLOC(t->d_cmask, sizeof(uint64_t) * (size_t)n * kBoundSlots);
    ALLOC(t->d_cscore, sizeof(float) * (size_t)n * kBoundSlots);
#undef ALLOC
    int8_t *d_rows = nullptr;
    float *d_prior_in = nullptr;
    int32_t *d_lut_row = nullptr, *d_den = nullptr;
    double *d_lut = nullptr;
    std::vector<int64_t> nsets(64 * 8, 0);
    for (int b = 0; b < 64; ++b)
        for (int k = 0; k < 8; ++k) nsets[b * 8 + k] = sets_upto(b, k);
#define CK(call)                                                                         \
    if ((e = (call)) != hipSuccess) {                                                     \
        set_error(std::string(#call) + ": " + hipGetErrorString(e));                      \
        hipFree(d_rows); hipFree(d_prior_in);                                             \
        hipFree(d_lut_row); hipFree(d_den); hipFree(d_lut);                               \
        return fail(BNOS_E_DEVICE);                                                       \
    }
    if (N > 0 && !dev_data) CK(hipMalloc((void **)&d_rows, (size_t)N * n));
    if (prior) CK(hipMalloc((void **)&d_prior_in, sizeof(float) * n * n));
    CK(hipMemsetAsync(t->d_data, 0, (size_t)n * t->N_pad, st));
    if (N > 0 && !dev_data) CK(hipMemcpyAsync(d_rows, data, (size_t)N * n, hipMemcpyHostToDevice, st));
    if (prior) CK(hipMemcpyAsync(d_prior_in, prior, sizeof(float) * n * n, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(t->d_ar, arities, sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(t->d_nsets, nsets.data(), sizeof(int64_t) * 64 * 8, hipMemcpyHostToDevice, st));
    if (N > 0) {
        int64_t tot = N * n;
        int blocks = (int)std::min<int64_t>((tot + 255) / 256, 1 << 16);
        if (dev_data) {                          // the caller's device rows: check their states first
            unsigned *d_bad = nullptr;
            unsigned bad = 0;
            CK(hipMalloc((void **)&d_bad, sizeof(unsigned)));
            hipError_t e2 = hipMemsetAsync(d_bad, 0, sizeof(unsigned), st);
            if (e2 == hipSuccess) {
                hipLaunchKernelGGL(k_check_states, dim3(blocks), dim3(256), 0, st, data, N, n, t->d_ar, d_bad);
                e2 = hipGetLastError();
            }
            if (e2 == hipSuccess) e2 = hipMemcpyAsync(&bad, d_bad, sizeof(unsigned), hipMemcpyDeviceToHost, st);
            if (e2 == hipSuccess) e2 = hipStreamSynchronize(st);
            hipFree(d_bad);
            CK(e2);
            if (bad) {
                char buf[128];
                std::snprintf(buf, sizeof buf, "%u states of the device data are outside their node's arity", bad);
                set_error(buf);
                hipFree(d_prior_in);
                return fail(BNOS_E_INVALID);
            }
        }
        hipLaunchKernelGGL(k_ingest, dim3(blocks), dim3(256), 0, st, dev_data ? data : d_rows, N, n, t->N_pad,
                           t->d_data);
        CK(hipGetLastError());
    }
    hipLaunchKernelGGL(k_prior, dim3((n * n + 255) / 256), dim3(256), 0, st, d_prior_in, n, o.prior_mode,
                       t->d_prior);
    CK(hipGetLastError());
    // lnGamma lookup: the BDeu terms only take alpha = ess / d for d = q (a
    // product of at most K parent arities) and d = q * r_i; every such d up to
    // the largest q * r_i gets a row of lnG(c + alpha) - lnG(alpha), c = 0..N,
    // unless that would take more than kLutBytes (then lgamma is called inline).
    {
        std::vector<char> isq(max_cells + 1, 0), isd(max_cells + 1, 0);
        std::vector<int> ar_set;
        for (int v = 0; v < n; ++v)
            if (std::find(ar_set.begin(), ar_set.end(), arities[v]) == ar_set.end()) ar_set.push_back(arities[v]);
        std::vector<int> qs = {1};
        isq[1] = 1;
        for (int depth = 0; depth < K; ++depth) {
            const size_t m = qs.size();
            for (size_t i = 0; i < m; ++i)
                for (int a : ar_set) {
                    const int64_t q = (int64_t)qs[i] * a;
                    if (q <= max_cells && !isq[q]) { isq[q] = 1; qs.push_back((int)q); }
                }
        }
        std::vector<int32_t> den, row(max_cells + 1, 0);
        for (int q : qs) {
            isd[q] = 1;
            for (int a : ar_set)
                if ((int64_t)q * a <= max_cells) isd[(int64_t)q * a] = 1;
        }
        for (int d = 1; d <= max_cells; ++d)
            if (isd[d]) { row[d] = (int32_t)den.size(); den.push_back(d); }
        constexpr int64_t kLutBytes = 256ll << 20;
        if ((int64_t)den.size() * (N + 1) * 8 <= kLutBytes) {
            CK(hipMalloc((void **)&d_den, sizeof(int32_t) * den.size()));
            CK(hipMalloc((void **)&d_lut_row, sizeof(int32_t) * row.size()));
            CK(hipMalloc((void **)&d_lut, sizeof(double) * den.size() * (size_t)(N + 1)));
            CK(hipMemcpyAsync(d_den, den.data(), sizeof(int32_t) * den.size(), hipMemcpyHostToDevice, st));
            CK(hipMemcpyAsync(d_lut_row, row.data(), sizeof(int32_t) * row.size(), hipMemcpyHostToDevice, st));
            const int64_t tot = (int64_t)den.size() * (N + 1);
            hipLaunchKernelGGL(k_lut, dim3((unsigned)std::min<int64_t>((tot + 255) / 256, 1 << 16)), dim3(256), 0, st,
                               d_den, (int)den.size(), N, ess, d_lut);
            CK(hipGetLastError());
        }
    }
    int cap = cells_cap_for(max_cells);
    t->count_mode = (d_lut && o.count_mode == 0) ? 0 : 1;
    if (t->count_mode == 0) {                    // one joint histogram per node subset
        if (waves_for_cells(cap) == 4) { CK(launch_build_joint<4>(t, st, cap, d_lut_row, d_lut)); }
        else { CK(launch_build_joint<1>(t, st, cap, d_lut_row, d_lut)); }
    } else {                                     // one histogram per family
        if (waves_for_cells(cap) == 4) { CK(launch_build<4>(t, st, cap, d_lut_row, d_lut)); }
        else { CK(launch_build<1>(t, st, cap, d_lut_row, d_lut)); }
    }
    hipLaunchKernelGGL(k_node_stats, dim3(n), dim3(1024), 0, st, t->d_scores, t->S, t->S_pad, t->d_prior, n,
                       t->d_nstat);
    CK(hipGetLastError());
    {
        const int64_t tiles = (int64_t)n * (t->S_pad / 256);
        const int64_t row_tiles = t->S_pad / 256;
        hipLaunchKernelGGL(k_tile_and, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, st, t->d_masks,
                           t->d_scores, tiles, row_tiles, row_tiles / (4 * (int64_t)t->pad_steps), t->pad_steps,
                           t->d_tand, t->d_tsub, t->d_tmax);
        CK(hipGetLastError());
        hipLaunchKernelGGL(k_bound_cands, dim3(n), dim3(1024), 0, st, t->d_masks, t->d_scores, n, K, t->S,
                           t->S_pad, t->d_cmask, t->d_cscore);
        CK(hipGetLastError());
        const int64_t groups = (int64_t)n * (t->S_pad / 4);
        hipLaunchKernelGGL(k_anchor, dim3((unsigned)((groups + 255) / 256)), dim3(256), 0, st, t->d_masks, n,
                           t->S_pad, t->d_anchor);
        CK(hipGetLastError());
    }
    CK(hipStreamSynchronize(st));
    hipFree(d_rows);
    hipFree(d_prior_in);
    hipFree(d_lut_row);
    hipFree(d_den);
    hipFree(d_lut);
#undef CK
    t->magic = kMagic;
    register_handle(t);
    *out = reinterpret_cast<bnos_table>(t);
    return BNOS_OK;
}

extern "C" void bnos_table_free(bnos_table h)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!t || !handle_live(t)) return;
    unregister_handle(t);
    hipDeviceSynchronize();
    t->magic = 0;
    free_device(t);
    delete t;
}

extern "C" bnos_status bnos_table_info(bnos_table h, int32_t *n, int32_t *K, int64_t *S, int64_t *bytes)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (n) *n = t->n;
    if (K) *K = t->K;
    if (S) *S = t->S;
    if (bytes) *bytes = t->device_bytes();
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_export(bnos_table h, int32_t node, uint64_t *masks, float *scores, int64_t cap)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (!masks || !scores) { set_error("output is NULL"); return BNOS_E_INVALID; }
    if (node < 0 || node >= t->n) { set_error("node out of range"); return BNOS_E_RANGE; }
    if (cap < t->S) { set_error("cap below entries per node"); return BNOS_E_RANGE; }
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipMemcpy(masks, t->d_masks + (int64_t)node * t->S_pad, sizeof(uint64_t) * t->S, hipMemcpyDeviceToHost));
    BNOS_HIP(hipMemcpy(scores, t->d_scores + (int64_t)node * t->S_pad, sizeof(float) * t->S, hipMemcpyDeviceToHost));
    return BNOS_OK;
}

extern "C" bnos_status bnos_counts(bnos_table h, int32_t Q, const int32_t *nodes, const uint64_t *masks,
                                   uint32_t *counts, int64_t cap)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (Q < 0) { set_error("Q < 0"); return BNOS_E_RANGE; }
    if (Q == 0) return BNOS_OK;
    if (!nodes || !masks || !counts) { set_error("NULL argument"); return BNOS_E_INVALID; }
    std::vector<int32_t> ar(t->n);
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipMemcpy(ar.data(), t->d_ar, sizeof(int32_t) * t->n, hipMemcpyDeviceToHost));
    std::vector<int64_t> off(Q);
    int64_t tot = 0;
    int maxc = 1;
    for (int q = 0; q < Q; ++q) {
        int v = nodes[q];
        if (v < 0 || v >= t->n) { set_error("query node out of range"); return BNOS_E_RANGE; }
        uint64_t m = masks[q];
        if (t->n < 64 && (m >> t->n)) { set_error("query mask names a node >= n"); return BNOS_E_INVALID; }
        if ((m >> v) & 1ull) { set_error("query mask contains its own node"); return BNOS_E_INVALID; }
        if (__builtin_popcountll(m) > t->K) { set_error("query mask has more than K members"); return BNOS_E_RANGE; }
        int64_t c = ar[v];
        for (int b = 0; b < t->n; ++b) if ((m >> b) & 1ull) c *= ar[b];
        off[q] = tot;
        tot += c;
        if (c > maxc) maxc = (int)c;
    }
    if (tot > cap) { set_error("cap below total cells"); return BNOS_E_RANGE; }
    int32_t *d_nodes = nullptr;
    uint64_t *d_masks = nullptr;
    int64_t *d_off = nullptr;
    uint32_t *d_out = nullptr;
    hipError_t e = hipSuccess;
    auto cleanup = [&]() { hipFree(d_nodes); hipFree(d_masks); hipFree(d_off); hipFree(d_out); };
#define CK(call) if ((e = (call)) != hipSuccess) { set_error(std::string(#call) + ": " + hipGetErrorString(e)); cleanup(); return BNOS_E_DEVICE; }
    CK(hipMalloc((void **)&d_nodes, sizeof(int32_t) * Q));
    CK(hipMalloc((void **)&d_masks, sizeof(uint64_t) * Q));
    CK(hipMalloc((void **)&d_off, sizeof(int64_t) * Q));
    CK(hipMalloc((void **)&d_out, sizeof(uint32_t) * tot));
    CK(hipMemcpy(d_nodes, nodes, sizeof(int32_t) * Q, hipMemcpyHostToDevice));
    CK(hipMemcpy(d_masks, masks, sizeof(uint64_t) * Q, hipMemcpyHostToDevice));
    CK(hipMemcpy(d_off, off.data(), sizeof(int64_t) * Q, hipMemcpyHostToDevice));
    int cap_cells = cells_cap_for(maxc);
    int blocks = (int)std::min<int64_t>((Q + 3) / 4, 1 << 16);
    // the counting code of the table's own build: joint histograms (count_mode 0) or per family
    const bool four = waves_for_cells(cap_cells) == 4;
    const dim3 grid((unsigned)(four ? blocks : blocks * 4)), block(four ? 256 : 64);
    const size_t lds = (four ? 4 : 1) * cap_cells * sizeof(uint32_t);
    if (t->count_mode == 0) {
        if (four) hipLaunchKernelGGL(k_counts_joint<4>, grid, block, lds, 0, t->d_data, t->N, t->N_pad, t->d_ar, Q,
                                     d_nodes, d_masks, d_off, cap_cells, d_out);
        else hipLaunchKernelGGL(k_counts_joint<1>, grid, block, lds, 0, t->d_data, t->N, t->N_pad, t->d_ar, Q,
                                d_nodes, d_masks, d_off, cap_cells, d_out);
    } else {
        if (four) hipLaunchKernelGGL(k_counts<4>, grid, block, lds, 0, t->d_data, t->N, t->N_pad, t->d_ar, Q,
                                     d_nodes, d_masks, d_off, cap_cells, d_out);
        else hipLaunchKernelGGL(k_counts<1>, grid, block, lds, 0, t->d_data, t->N, t->N_pad, t->d_ar, Q, d_nodes,
                                d_masks, d_off, cap_cells, d_out);
    }
    CK(hipGetLastError());
    CK(hipMemcpy(counts, d_out, sizeof(uint32_t) * tot, hipMemcpyDeviceToHost));
#undef CK
    cleanup();
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_node_features(bnos_table h, double *out)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (!out) { set_error("out is NULL"); return BNOS_E_INVALID; }
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipMemcpy(out, t->d_nstat, sizeof(double) * 5 * t->n, hipMemcpyDeviceToHost));
    return BNOS_OK;
}
