// Order scoring: for every node, stream its (mask, score) entries, keep those
// whose parent set lies inside the node's predecessor set, and reduce them by
// log-sum-exp and by argmax (Sec. III.B, Alg. 1 and Eq. (6)).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "bnos_internal.h"
#include "score_device.h"

namespace bnos {

// One block per order: merge its chunk partials and write the per-order sums.
__global__ __launch_bounds__(kMergeWaves * 64) void k_merge(ScoreArgs A)
{
    __shared__ double s_l[64], s_b[64];
    const int b = blockIdx.x;
    bool valid;
    double l, m;
    merge_block(A, b, s_l, s_b, valid, l, m);
    if (threadIdx.x == 0) {
        A.lse[b] = valid ? l : NAN;
        A.maxs[b] = valid ? m : NAN;
    }
}

// ------------------------------------------------------------------ host side

// Orders per block: a block folds every streamed entry into this many order states.
int pick_bt(const TableT *t, int B)
{
    int bt = B >= 8 ? 8 : (B >= 4 ? 4 : (B >= 2 ? 2 : 1));
    if (t->tuned_bt[0] > 0) {
        // autotuned choice for the batch-size bucket (1, 2-3, 4-7, 8-15, 16+)
        int k = B >= 16 ? 4 : (B >= 8 ? 3 : (B >= 4 ? 2 : (B >= 2 ? 1 : 0)));
        if (t->tuned_bt[k] > 0 && t->tuned_bt[k] <= B) bt = t->tuned_bt[k];
    }
    return bt;
}

// Scoring workspace for up to `B` orders: the chunk partials.
bnos_status ensure_workspace(TableT *t, int B)
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

ScoreArgs score_args(const TableT *t, const int32_t *orders, int B, double *lse, double *maxs,
                     uint64_t *best, double *node_lse, float *node_second)
{
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
    A.wl_count = nullptr;
    A.wl_list = nullptr;
    A.tand = t->tile_skip ? t->d_tand : nullptr;
    A.tiles_loaded = t->timing ? t->d_tiles : nullptr;
    return A;
}

template <int BT>
static void launch_bt(const ScoreArgs &A, int nblocks_x, hipStream_t st)
{
    dim3 grid((unsigned)nblocks_x, (unsigned)((A.B + BT - 1) / BT));
    hipLaunchKernelGGL(k_score<BT>, grid, dim3(kScoreThreads), 0, st, A);
}

// The streaming pass (k_score) with the table's block shape; timed when enabled.
// The workspace must already hold A.B orders.
bnos_status launch_stream(TableT *t, const ScoreArgs &A, hipStream_t st, int bt)
{
    bnos_status s;
    if (bt <= 0) bt = pick_bt(t, A.B);
    if (t->timing) {
        if ((s = record_event(t, true, st)) != BNOS_OK) return s;
    }
    const int nbx = t->n * t->chunks;
    if (bt == 8) launch_bt<8>(A, nbx, st);
    else if (bt == 4) launch_bt<4>(A, nbx, st);
    else if (bt == 2) launch_bt<2>(A, nbx, st);
    else launch_bt<1>(A, nbx, st);
    BNOS_HIP(hipGetLastError());
    if (t->timing) {
        if ((s = record_event(t, false, st)) != BNOS_OK) return s;
        if (t->ev_passes.size() <= t->ev_used) t->ev_passes.resize(t->ev_used + 1);
        t->ev_passes[t->ev_used] = (A.B + bt - 1) / bt;
        t->ev_used++;
    }
    return BNOS_OK;
}

static bnos_status score_impl(TableT *t, const int32_t *orders, int B, double *lse, double *maxs,
                              uint64_t *best, double *node_lse, float *node_second, hipStream_t st)
{
    bnos_status s = ensure_workspace(t, B);
    if (s != BNOS_OK) return s;
    ScoreArgs A = score_args(t, orders, B, lse, maxs, best, node_lse, node_second);
    if ((s = launch_stream(t, A, st, 0)) != BNOS_OK) return s;
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
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipDeviceSynchronize());
    t->timing = enable != 0;
    t->ev_used = 0;
    t->timed_ms = 0.0;
    t->timed_launches = 0;
    t->timed_passes = 0;
    BNOS_HIP(hipMemset(t->d_tiles, 0, sizeof(unsigned long long)));
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_tiles_read(bnos_table h, int64_t *tiles_loaded, int64_t *tiles_per_pass)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipDeviceSynchronize());
    unsigned long long v = 0;
    BNOS_HIP(hipMemcpy(&v, t->d_tiles, sizeof v, hipMemcpyDeviceToHost));
    if (tiles_loaded) *tiles_loaded = (int64_t)v;
    if (tiles_per_pass) *tiles_per_pass = (int64_t)t->n * (t->S_pad / 256);
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_tile_skip(bnos_table h, int32_t enable)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    t->tile_skip = enable != 0;
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
