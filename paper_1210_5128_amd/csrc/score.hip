// Order scoring: for every node, stream its (mask, score) entries, keep those
// whose parent set lies inside the node's predecessor set, and reduce them by
// log-sum-exp and by argmax (Sec. III.B, Alg. 1 and Eq. (6)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "bnos_internal.h"

namespace bnos {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ device helpers

struct Acc {
    float m, s;       // log-sum-exp state: max and sum of exp(x - m)
    float best, sec;  // top-1 score and best score among the other entries
    uint64_t bm;      // mask of the top-1 entry
};

__device__ __forceinline__ void acc_init(Acc &a)
{
    a.m = -INFINITY;
    a.s = 0.f;
    a.best = -INFINITY;
    a.sec = -INFINITY;
    a.bm = ~0ull;
}

// Fold one consistent entry (x, mask) into the state.  Argmax tie rule: the
// larger score wins; on equal scores the smaller mask wins.  Called under a
// divergent branch on consistency, so a wavefront whose lanes hold no
// consistent entry skips it entirely.
__device__ __forceinline__ void acc_push(Acc &a, float x, uint64_t mk)
{
    float d = x - a.m;
    float e = __expf(-fabsf(d));
    a.s = (d > 0.f) ? fmaf(a.s, e, 1.f) : a.s + e;
    a.m = fmaxf(a.m, x);
    if (x >= a.sec) {
        bool better = x > a.best || (x == a.best && mk < a.bm);
        a.sec = better ? a.best : fmaxf(a.sec, x);
        a.best = better ? x : a.best;
        a.bm = better ? mk : a.bm;
    }
}

// Combine two states (order-independent up to FP32 rounding; the callers fix the order).
__device__ __forceinline__ void acc_merge(Acc &a, const Acc &b)
{
    float M = fmaxf(a.m, b.m);
    float sa = (a.m == -INFINITY) ? 0.f : a.s * __expf(a.m - M);
    float sb = (b.m == -INFINITY) ? 0.f : b.s * __expf(b.m - M);
    a.m = M;
    a.s = sa + sb;
    bool take = b.best > a.best || (b.best == a.best && b.bm < a.bm);
    float sec = take ? fmaxf(a.best, b.sec) : fmaxf(a.sec, b.best);
    a.best = take ? b.best : a.best;
    a.bm = take ? b.bm : a.bm;
    a.sec = sec;
}

__device__ __forceinline__ Acc acc_shfl_xor(const Acc &a, int off)
{
    Acc b;
    b.m = __shfl_xor(a.m, off, 64);
    b.s = __shfl_xor(a.s, off, 64);
    b.best = __shfl_xor(a.best, off, 64);
    b.sec = __shfl_xor(a.sec, off, 64);
    b.bm = (uint64_t)__shfl_xor((unsigned long long)a.bm, off, 64);
    return b;
}

// Butterfly merge over the 64 lanes.  In every pair the lower lane's state is
// the left operand, so both lanes compute the same value and the result does
// not depend on scheduling.
__device__ __forceinline__ void acc_wave_reduce(Acc &a, int lane)
{
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        Acc o = acc_shfl_xor(a, off);
        const bool upper = (lane & off) != 0;
        Acc lo, hi;
        lo.m = upper ? o.m : a.m;
        hi.m = upper ? a.m : o.m;
        lo.s = upper ? o.s : a.s;
        hi.s = upper ? a.s : o.s;
        lo.best = upper ? o.best : a.best;
        hi.best = upper ? a.best : o.best;
        lo.sec = upper ? o.sec : a.sec;
        hi.sec = upper ? a.sec : o.sec;
        lo.bm = upper ? o.bm : a.bm;
        hi.bm = upper ? a.bm : o.bm;
        acc_merge(lo, hi);
        a = lo;
    }
}

__device__ __forceinline__ double wave_sum_f64(double v, int lane)
{
    // fixed butterfly: the lower lane's value is the left operand
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        double o = __shfl_xor(v, off, 64);
        v = (lane & off) ? (o + v) : (v + o);
    }
    return v;
}

// Predecessor mask of `node` in an order, computed by one wavefront (lane p
// reads position p).  valid = the order is a permutation of 0..n-1.
__device__ __forceinline__ uint64_t wave_pred(const int32_t *__restrict__ ord, int n, int node,
                                              int lane, bool &valid)
{
    int v = (lane < n) ? ord[lane] : -1;
    bool inr = (v >= 0 && v < n);
    uint64_t bit = inr ? (1ull << v) : 0ull;
    uint64_t here = __ballot(lane < n && v == node);
    int pos = here ? __builtin_ctzll(here) : 0;
    uint64_t before = (lane < pos) ? bit : 0ull;
    uint64_t all = bit;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        before |= (uint64_t)__shfl_xor((unsigned long long)before, off, 64);
        all |= (uint64_t)__shfl_xor((unsigned long long)all, off, 64);
    }
    uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    valid = (all == full) && (__ballot(lane < n && !inr) == 0ull);
    return valid ? before : 0ull;
}

__device__ __forceinline__ uint64_t uniform_u64(uint64_t v)
{
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------------------------ kernel

struct ScoreArgs {
    const uint64_t *masks;
    const float *scores;
    int64_t S_pad;
    int chunks, chunk_entries;
    const int32_t *orders;
    int B, n;
    Partial *part;          // [B][n][chunks]
    double *lse, *maxs;
    uint64_t *best;
    double *node_lse;
    float *node_second;
};

// Grid: x = node * chunks + chunk, y = group of BT orders.  Every block
// streams one chunk of one node's entries once, folds each entry into BT order
// states and writes one Partial per order.
template <int BT>
__global__ __launch_bounds__(kScoreThreads) void k_score(ScoreArgs A)
{
    __shared__ uint64_t s_npred[BT];
    __shared__ Acc s_red[kScoreThreads / 64][BT];
    const int node = blockIdx.x / A.chunks;
    const int chunk = blockIdx.x - node * A.chunks;
    const int b0 = blockIdx.y * BT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = A.n;

    for (int j = wave; j < BT; j += kScoreThreads / 64) {
        uint64_t np = ~0ull;   // no order in this slot: nothing is consistent
        if (b0 + j < A.B) {
            bool valid;
            uint64_t pred = wave_pred(A.orders + (int64_t)(b0 + j) * n, n, node, lane, valid);
            np = ~pred;        // invalid order: only the empty set is consistent
        }
        if (lane == 0) s_npred[j] = np;
    }
    __syncthreads();
    uint64_t npred[BT];
    Acc a[BT];
#pragma unroll
    for (int j = 0; j < BT; ++j) {
        npred[j] = uniform_u64(s_npred[j]);
        acc_init(a[j]);
    }

    const int64_t row = (int64_t)node * A.S_pad + (int64_t)chunk * A.chunk_entries;
    const u64x2 *mp = reinterpret_cast<const u64x2 *>(A.masks + row);
    const f32x4 *sp = reinterpret_cast<const f32x4 *>(A.scores + row);
    const int steps = A.chunk_entries / kEntriesPerStep;
    // Software pipeline: the loads of step it+1 are in flight while step it is folded.
    int q = threadIdx.x;                                     // this lane's 4-entry group
    u64x2 n01 = __builtin_nontemporal_load(&mp[2 * q]);
    u64x2 n23 = __builtin_nontemporal_load(&mp[2 * q + 1]);
    f32x4 nsc = __builtin_nontemporal_load(&sp[q]);
    for (int it = 0; it < steps; ++it) {
        const u64x2 m01 = n01, m23 = n23;
        const f32x4 sc = nsc;
        if (it + 1 < steps) {
            q += kScoreThreads;
            n01 = __builtin_nontemporal_load(&mp[2 * q]);
            n23 = __builtin_nontemporal_load(&mp[2 * q + 1]);
            nsc = __builtin_nontemporal_load(&sp[q]);
        }
        const uint64_t mk[4] = {m01.x, m01.y, m23.x, m23.y};
        const float x[4] = {sc.x, sc.y, sc.z, sc.w};
#pragma unroll
        for (int j = 0; j < BT; ++j) {
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                if ((mk[k] & npred[j]) == 0ull) acc_push(a[j], x[k], mk[k]);
            }
        }
    }

#pragma unroll
    for (int j = 0; j < BT; ++j) {
        acc_wave_reduce(a[j], lane);
        if (lane == 0) s_red[wave][j] = a[j];
    }
    __syncthreads();
    if (threadIdx.x < BT) {
        const int j = threadIdx.x;
        if (b0 + j < A.B) {
            Acc r;
            r.m = s_red[0][j].m;
            r.s = s_red[0][j].s;
            r.best = s_red[0][j].best;
            r.sec = s_red[0][j].sec;
            r.bm = s_red[0][j].bm;
#pragma unroll
            for (int w = 1; w < kScoreThreads / 64; ++w) {
                Acc o;
                o.m = s_red[w][j].m;
                o.s = s_red[w][j].s;
                o.best = s_red[w][j].best;
                o.sec = s_red[w][j].sec;
                o.bm = s_red[w][j].bm;
                acc_merge(r, o);
            }
            Partial p;
            p.m = r.m;
            p.s = r.s;
            p.best = r.best;
            p.second = r.sec;
            p.bmask = r.bm;
            A.part[((int64_t)(b0 + j) * n + node) * A.chunks + chunk] = p;
        }
    }
}

constexpr int kMergeWaves = 16;
constexpr int kMergeNodesPerWave = 4;   // 16 waves x 4 nodes covers n <= 64

__device__ __forceinline__ Acc load_partial(const Partial *p)
{
    Acc a;
    a.m = p->m;
    a.s = p->s;
    a.best = p->best;
    a.sec = p->second;
    a.bm = p->bmask;
    return a;
}

// One block per order.  Wave w merges the chunk partials of nodes w, w+16,
// w+32, w+48 (lanes over chunks, then a fixed butterfly); the first partial
// of every node is loaded before any merging so the loads overlap.  Wave 0
// then sums the per-node terms in FP64 with a fixed butterfly.
__global__ __launch_bounds__(kMergeWaves * 64) void k_merge(ScoreArgs A)
{
    __shared__ double s_l[64], s_b[64];
    const int b = blockIdx.x;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = A.n;
    const int chunks = A.chunks;
    bool valid;
    (void)wave_pred(A.orders + (int64_t)b * n, n, 0, lane, valid);

    Acc r[kMergeNodesPerWave];
#pragma unroll
    for (int k = 0; k < kMergeNodesPerWave; ++k) {
        const int i = wave + kMergeWaves * k;
        acc_init(r[k]);
        if (i < n && lane < chunks) r[k] = load_partial(A.part + ((int64_t)b * n + i) * chunks + lane);
    }
#pragma unroll
    for (int k = 0; k < kMergeNodesPerWave; ++k) {
        const int i = wave + kMergeWaves * k;
        if (i >= n) break;
        const Partial *pp = A.part + ((int64_t)b * n + i) * chunks;
        for (int c = lane + 64; c < chunks; c += 64) acc_merge(r[k], load_partial(pp + c));
        acc_wave_reduce(r[k], lane);
        if (lane == 0) {
            const double li = (double)r[k].m + log((double)r[k].s);
            const int64_t o = (int64_t)b * n + i;
            s_l[i] = li;
            s_b[i] = (double)r[k].best;
            A.best[o] = valid ? r[k].bm : 0ull;
            if (A.node_lse) A.node_lse[o] = valid ? li : NAN;
            if (A.node_second) A.node_second[o] = valid ? r[k].sec : NAN;
        }
    }
    __syncthreads();
    if (wave == 0) {
        double l = (lane < n) ? s_l[lane] : 0.0;
        double m = (lane < n) ? s_b[lane] : 0.0;
        l = wave_sum_f64(l, lane);
        m = wave_sum_f64(m, lane);
        if (lane == 0) {
            A.lse[b] = valid ? l : NAN;
            A.maxs[b] = valid ? m : NAN;
        }
    }
}

// ------------------------------------------------------------------ host side

// Orders per block: a block folds every streamed entry into this many order states.
static int pick_bt(int B) { return B >= 8 ? 8 : (B >= 4 ? 4 : (B >= 2 ? 2 : 1)); }

template <int BT>
static void launch_score(const ScoreArgs &A, int nblocks_x, hipStream_t st)
{
    dim3 grid((unsigned)nblocks_x, (unsigned)((A.B + BT - 1) / BT));
    hipLaunchKernelGGL(k_score<BT>, grid, dim3(kScoreThreads), 0, st, A);
}

// Scoring workspace for up to `B` orders: the chunk partials.
static bnos_status ensure_workspace(TableT *t, int B)
{
    if (t->part_orders >= B) return BNOS_OK;
    // A launch still in flight may use the old buffer.
    BNOS_HIP(hipDeviceSynchronize());
    BNOS_HIP(hipFree(t->d_part));
    t->d_part = nullptr;
    t->part_orders = 0;
    int64_t want = B < 64 ? 64 : B;
    hipError_t e = hipMalloc(&t->d_part, (size_t)want * t->workspace_bytes_per_order());
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc scoring workspace: ") + hipGetErrorString(e));
        t->d_part = nullptr;
        return e == hipErrorOutOfMemory ? BNOS_E_NOMEM : BNOS_E_DEVICE;
    }
    t->part_orders = want;
    return BNOS_OK;
}

static bnos_status record_event(TableT *t, bool start, hipStream_t st)
{
    std::vector<hipEvent_t> &pool = start ? t->ev_start : t->ev_stop;
    if (pool.size() <= t->ev_used) {
        hipEvent_t e;
        BNOS_HIP(hipEventCreate(&e));
        pool.push_back(e);
    }
    BNOS_HIP(hipEventRecord(pool[t->ev_used], st));
    return BNOS_OK;
}

static bnos_status score_impl(TableT *t, const int32_t *orders, int B, double *lse, double *maxs,
                              uint64_t *best, double *node_lse, float *node_second, hipStream_t st)
{
    bnos_status s = ensure_workspace(t, B);
    if (s != BNOS_OK) return s;
    ScoreArgs A;
    A.masks = t->d_masks;
    A.scores = t->d_scores;
    A.S_pad = t->S_pad;
    A.chunks = t->chunks;
    A.chunk_entries = t->chunk_entries;
    A.orders = orders;
    A.B = B;
    A.n = t->n;
    A.part = reinterpret_cast<Partial *>(t->d_part);
    A.lse = lse;
    A.maxs = maxs;
    A.best = best;
    A.node_lse = node_lse;
    A.node_second = node_second;
    if (t->timing) {
        if ((s = record_event(t, true, st)) != BNOS_OK) return s;
    }
    const int bt = pick_bt(B);
    const int nbx = t->n * t->chunks;
    if (bt == 8) launch_score<8>(A, nbx, st);
    else if (bt == 4) launch_score<4>(A, nbx, st);
    else if (bt == 2) launch_score<2>(A, nbx, st);
    else launch_score<1>(A, nbx, st);
    BNOS_HIP(hipGetLastError());
    if (t->timing) {
        if ((s = record_event(t, false, st)) != BNOS_OK) return s;
        if (t->ev_passes.size() <= t->ev_used) t->ev_passes.resize(t->ev_used + 1);
        t->ev_passes[t->ev_used] = (B + bt - 1) / bt;
        t->ev_used++;
    }
    hipLaunchKernelGGL(k_merge, dim3(B), dim3(kMergeWaves * 64), 0, st, A);
    BNOS_HIP(hipGetLastError());
    return BNOS_OK;
}

}  // namespace bnos

using namespace bnos;

extern "C" bnos_status bnos_score_orders(bnos_table h, const int32_t *orders, int32_t B, double *lse,
                                         double *maxs, uint64_t *best, double *node_lse, float *node_second,
                                         void *stream)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (B < 1 || B > (1 << 20)) { set_error("B outside [1, 2^20]"); return BNOS_E_RANGE; }
    if (!orders || !lse || !maxs || !best) { set_error("NULL argument"); return BNOS_E_INVALID; }
    BNOS_HIP(hipSetDevice(t->device));
    return score_impl(t, orders, B, lse, maxs, best, node_lse, node_second, reinterpret_cast<hipStream_t>(stream));
}

extern "C" bnos_status bnos_score_order(bnos_table h, const int32_t *order, double *lse, double *maxs,
                                        uint64_t *best_parents)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (!order || !lse || !maxs) { set_error("NULL argument"); return BNOS_E_INVALID; }
    const int n = t->n;
    uint64_t seen = 0;
    for (int p = 0; p < n; ++p) {
        if (order[p] < 0 || order[p] >= n || ((seen >> order[p]) & 1ull)) {
            set_error("order is not a permutation of 0..n-1");
            return BNOS_E_INVALID;
        }
        seen |= 1ull << order[p];
    }
    BNOS_HIP(hipSetDevice(t->device));
    int32_t *d_ord = nullptr;
    double *d_out = nullptr;
    uint64_t *d_best = nullptr;
    hipError_t e;
    auto cleanup = [&]() { hipFree(d_ord); hipFree(d_out); hipFree(d_best); };
#define CK(call) if ((e = (call)) != hipSuccess) { set_error(std::string(#call) + ": " + hipGetErrorString(e)); cleanup(); return BNOS_E_DEVICE; }
    CK(hipMalloc((void **)&d_ord, sizeof(int32_t) * n));
    CK(hipMalloc((void **)&d_out, sizeof(double) * 2));
    CK(hipMalloc((void **)&d_best, sizeof(uint64_t) * n));
    CK(hipMemcpy(d_ord, order, sizeof(int32_t) * n, hipMemcpyHostToDevice));
    bnos_status s = score_impl(t, d_ord, 1, d_out, d_out + 1, d_best, nullptr, nullptr, nullptr);
    if (s != BNOS_OK) { cleanup(); return s; }
    double host[2];
    CK(hipMemcpy(host, d_out, sizeof(double) * 2, hipMemcpyDeviceToHost));
    if (best_parents) CK(hipMemcpy(best_parents, d_best, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
#undef CK
    cleanup();
    *lse = host[0];
    *maxs = host[1];
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_timing(bnos_table h, int32_t enable)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    t->timing = enable != 0;
    t->ev_used = 0;
    t->timed_ms = 0.0;
    t->timed_launches = 0;
    t->timed_passes = 0;
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_timing_read(bnos_table h, double *total_ms, int64_t *launches,
                                              int64_t *table_passes)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    for (size_t k = 0; k < t->ev_used; ++k) {
        BNOS_HIP(hipEventSynchronize(t->ev_stop[k]));
        float ms = 0.f;
        BNOS_HIP(hipEventElapsedTime(&ms, t->ev_start[k], t->ev_stop[k]));
        t->timed_ms += ms;
        t->timed_launches += 1;
        t->timed_passes += t->ev_passes[k];
    }
    t->ev_used = 0;
    if (total_ms) *total_ms = t->timed_ms;
    if (launches) *launches = t->timed_launches;
    if (table_passes) *table_passes = t->timed_passes;
    return BNOS_OK;
}
