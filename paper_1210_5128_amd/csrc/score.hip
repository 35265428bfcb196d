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
// larger score wins; on equal scores the smaller mask wins.
__device__ __forceinline__ void acc_push(Acc &a, float x, uint64_t mk, bool ok)
{
    float d = x - a.m;
    float e = __expf(-fabsf(d));
    bool up = d > 0.f;
    float s_new = up ? fmaf(a.s, e, 1.f) : a.s + e;
    float m_new = up ? x : a.m;
    a.s = ok ? s_new : a.s;
    a.m = ok ? m_new : a.m;
    bool better = ok && (x > a.best || (x == a.best && mk < a.bm));
    bool sec_up = ok && !better && x > a.sec;
    a.sec = better ? a.best : (sec_up ? x : a.sec);
    a.best = better ? x : a.best;
    a.bm = better ? mk : a.bm;
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

// Predecessor mask of `node` in order b, computed by one wavefront (lane p
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

// ------------------------------------------------------------------ kernels

// Grid: x = node * chunks + chunk, y = group of BT orders.  Each block streams
// one chunk of one node's entries once and folds every entry into BT order
// states; it writes one Partial per (order, node, chunk).
template <int BT>
__global__ __launch_bounds__(kScoreThreads) void k_score_stream(
    const uint64_t *__restrict__ masks, const float *__restrict__ scores, int64_t S_pad, int chunks,
    int chunk_entries, const int32_t *__restrict__ orders, int B, int n, Partial *__restrict__ part)
{
    __shared__ uint64_t s_npred[BT];
    __shared__ Acc s_red[kScoreThreads / 64][BT];
    const int node = blockIdx.x / chunks;
    const int chunk = blockIdx.x - node * chunks;
    const int b0 = blockIdx.y * BT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;

    for (int j = wave; j < BT; j += kScoreThreads / 64) {
        uint64_t np = ~0ull;   // no order: nothing is consistent
        if (b0 + j < B) {
            bool valid;
            uint64_t pred = wave_pred(orders + (int64_t)(b0 + j) * n, n, node, lane, valid);
            np = ~pred;        // invalid order: only the empty set is consistent
        }
        if (lane == 0) s_npred[j] = np;
    }
    __syncthreads();
    uint64_t npred[BT];
    Acc a[BT];
#pragma unroll
    for (int j = 0; j < BT; ++j) {
        npred[j] = s_npred[j];
        acc_init(a[j]);
    }

    const int64_t row = (int64_t)node * S_pad + (int64_t)chunk * chunk_entries;
    const u64x2 *mp = reinterpret_cast<const u64x2 *>(masks + row);
    const f32x4 *sp = reinterpret_cast<const f32x4 *>(scores + row);
    const int steps = chunk_entries / kEntriesPerStep;
    for (int it = 0; it < steps; ++it) {
        const int q = it * kScoreThreads + threadIdx.x;      // index of this lane's 4-entry group
        u64x2 m01 = __builtin_nontemporal_load(&mp[2 * q]);
        u64x2 m23 = __builtin_nontemporal_load(&mp[2 * q + 1]);
        f32x4 sc = __builtin_nontemporal_load(&sp[q]);
        const uint64_t mk[4] = {m01.x, m01.y, m23.x, m23.y};
        const float x[4] = {sc.x, sc.y, sc.z, sc.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
#pragma unroll
            for (int j = 0; j < BT; ++j) acc_push(a[j], x[k], mk[k], (mk[k] & npred[j]) == 0ull);
        }
    }

#pragma unroll
    for (int j = 0; j < BT; ++j) {
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            Acc o = acc_shfl_xor(a[j], off);
            // fixed pairing: the lower lane's state is always the left operand,
            // so both lanes of a pair compute the same result
            const bool upper = (lane & off) != 0;
            Acc lo, hi;
            lo.m = upper ? o.m : a[j].m;       hi.m = upper ? a[j].m : o.m;
            lo.s = upper ? o.s : a[j].s;       hi.s = upper ? a[j].s : o.s;
            lo.best = upper ? o.best : a[j].best; hi.best = upper ? a[j].best : o.best;
            lo.sec = upper ? o.sec : a[j].sec; hi.sec = upper ? a[j].sec : o.sec;
            lo.bm = upper ? o.bm : a[j].bm;    hi.bm = upper ? a[j].bm : o.bm;
            acc_merge(lo, hi);
            a[j] = lo;
        }
        if (lane == 0) s_red[wave][j] = a[j];
    }
    __syncthreads();
    if (threadIdx.x < BT) {
        const int j = threadIdx.x;
        if (b0 + j < B) {
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
            part[((int64_t)(b0 + j) * n + node) * chunks + chunk] = p;
        }
    }
}

// One wavefront per order: lane i merges node i's chunk partials in chunk
// order, then the per-node terms are summed in FP64 in node-id order.
__global__ __launch_bounds__(64) void k_score_merge(const Partial *__restrict__ part, int chunks,
                                                    const int32_t *__restrict__ orders, int B, int n,
                                                    double *__restrict__ lse, double *__restrict__ maxs,
                                                    uint64_t *__restrict__ best, double *__restrict__ node_lse,
                                                    float *__restrict__ node_second)
{
    __shared__ double s_l[64], s_b[64];
    const int b = blockIdx.x;
    const int lane = threadIdx.x;
    bool valid;
    (void)wave_pred(orders + (int64_t)b * n, n, 0, lane, valid);
    double li = 0.0, bi = 0.0;
    if (lane < n) {
        const Partial *p = part + ((int64_t)b * n + lane) * chunks;
        Acc a;
        a.m = p[0].m;
        a.s = p[0].s;
        a.best = p[0].best;
        a.sec = p[0].second;
        a.bm = p[0].bmask;
        for (int c = 1; c < chunks; ++c) {
            Acc o;
            o.m = p[c].m;
            o.s = p[c].s;
            o.best = p[c].best;
            o.sec = p[c].second;
            o.bm = p[c].bmask;
            acc_merge(a, o);
        }
        li = (double)a.m + log((double)a.s);
        bi = (double)a.best;
        if (best) best[(int64_t)b * n + lane] = valid ? a.bm : 0ull;
        if (node_lse) node_lse[(int64_t)b * n + lane] = valid ? li : NAN;
        if (node_second) node_second[(int64_t)b * n + lane] = valid ? a.sec : NAN;
    }
    s_l[lane] = li;
    s_b[lane] = bi;
    __syncthreads();
    if (lane == 0) {
        double tl = 0.0, tb = 0.0;
        for (int i = 0; i < n; ++i) {
            tl += s_l[i];
            tb += s_b[i];
        }
        lse[b] = valid ? tl : NAN;
        maxs[b] = valid ? tb : NAN;
    }
}

// ------------------------------------------------------------------ host side

template <int BT>
static void launch_stream(const TableT *t, const int32_t *orders, int B, hipStream_t st)
{
    dim3 grid((unsigned)(t->n * t->chunks), (unsigned)((B + BT - 1) / BT));
    hipLaunchKernelGGL(k_score_stream<BT>, grid, dim3(kScoreThreads), 0, st, t->d_masks, t->d_scores,
                       t->S_pad, t->chunks, t->chunk_entries, orders, B, t->n,
                       reinterpret_cast<Partial *>(t->d_part));
}

static bnos_status ensure_partials(TableT *t, int B)
{
    if (t->part_orders >= B) return BNOS_OK;
    // A launch still in flight may use the old buffer.
    BNOS_HIP(hipDeviceSynchronize());
    BNOS_HIP(hipFree(t->d_part));
    t->d_part = nullptr;
    t->part_orders = 0;
    int64_t want = B < 64 ? 64 : B;
    hipError_t e = hipMalloc(&t->d_part, (size_t)want * t->n * t->chunks * sizeof(Partial));
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc partials: ") + hipGetErrorString(e));
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
    bnos_status s = ensure_partials(t, B);
    if (s != BNOS_OK) return s;
    if (t->timing) {
        if ((s = record_event(t, true, st)) != BNOS_OK) return s;
    }
    // Orders per block: more orders share each streamed entry.
    if (B >= 4) launch_stream<4>(t, orders, B, st);
    else if (B >= 2) launch_stream<2>(t, orders, B, st);
    else launch_stream<1>(t, orders, B, st);
    BNOS_HIP(hipGetLastError());
    if (t->timing) {
        if ((s = record_event(t, false, st)) != BNOS_OK) return s;
        t->ev_used++;
    }
    hipLaunchKernelGGL(k_score_merge, dim3(B), dim3(64), 0, st, reinterpret_cast<const Partial *>(t->d_part),
                       t->chunks, orders, B, t->n, lse, maxs, best, node_lse, node_second);
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
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_timing_read(bnos_table h, double *total_ms, int64_t *launches)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    for (size_t k = 0; k < t->ev_used; ++k) {
        BNOS_HIP(hipEventSynchronize(t->ev_stop[k]));
        float ms = 0.f;
        BNOS_HIP(hipEventElapsedTime(&ms, t->ev_start[k], t->ev_stop[k]));
        t->timed_ms += ms;
        t->timed_launches += 1;
    }
    t->ev_used = 0;
    if (total_ms) *total_ms = t->timed_ms;
    if (launches) *launches = t->timed_launches;
    return BNOS_OK;
}
