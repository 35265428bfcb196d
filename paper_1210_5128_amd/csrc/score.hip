// Order scoring: for every node, stream its (mask, score) entries, keep those
// whose parent set lies inside the node's predecessor set, and reduce them by
// log-sum-exp and by argmax (Sec. III.B, Alg. 1 and Eq. (6)).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "bnos_internal.h"
#include "score_device.h"

namespace bnos {

// One block per order: merge its chunk partials and write the per-order sums.
__global__ __launch_bounds__(kMergeWaves * 64) void k_merge(ScoreArgs A)
{
    __shared__ MergeLds L;
    const int b = blockIdx.x;
    bool valid;
    double l, m;
    merge_block(A, b, L, valid, l, m);
    if (threadIdx.x == 0) {
        A.lse[b] = valid ? l : NAN;
        A.maxs[b] = valid ? m : NAN;
    }
}

// The cut of every (order, node) pair of a several-order launch, one wavefront
// per pair, written to A.cut_ws[order][node] before the scoring launch: the
// scoring blocks then read their orders' cuts instead of each recomputing them
// (a node's row is streamed by many blocks).
__global__ __launch_bounds__(kScoreThreads) void k_bound_pre(ScoreArgs A)
{
    const int64_t g = (int64_t)blockIdx.x * (kScoreThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    const int n = A.n;
    if (g >= (int64_t)A.B * n) return;            // uniform per wavefront
    const int b = (int)(g / n), node = (int)(g - (int64_t)b * n);
    bool valid;
    const uint64_t np = ~wave_pred(A.orders + (int64_t)b * n, n, node, lane, valid);
    const float c = wave_bound_cut(view_of(A), node, np, lane);
    if (lane == 0) A.cut_ws[g] = c;
}

// Gather pass: see the comment at kGatherMaxK (score_device.h).
__global__ __launch_bounds__(kScoreThreads) void k_gather(ScoreArgs A, const int64_t *__restrict__ nsets, int K)
{
    __shared__ int64_t s_w[kGatherMaxK][64];
    __shared__ uint64_t s_nb[64];
    __shared__ int s_p;
    __shared__ Acc s_red[kScoreThreads / 64];
    const int n = A.n;
    const int node = blockIdx.x / n;
    const int sub = blockIdx.x - node * n;
    const int ob = blockIdx.y;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (wave == 0) {
        bool valid;
        const uint64_t pred = wave_pred(A.orders + (int64_t)ob * n, n, node, lane, valid);
        if (lane < n && ((pred >> lane) & 1ull)) {
            const int i = __popcll(pred & ((1ull << lane) - 1ull));       // rank among the predecessors
            const int slot = lane < node ? lane : lane - 1;
#pragma unroll
            for (int t = 0; t < kGatherMaxK; ++t) s_w[t][i] = t < K ? nsets[slot * 8 + (K - t)] : 0;
            s_nb[i] = 1ull << lane;
        }
        if (lane == 0) s_p = __popcll(pred);
    }
    __syncthreads();
    const int p = s_p;
    const float *row = A.scores + (int64_t)node * A.S_pad;
    Acc a;
    acc_init(a);
    if (sub == 0) {
        if (threadIdx.x == 0) acc_push(a, row[0], 0ull);                   // the empty set
    } else if (K >= 1 && sub - 1 < p) {
        const int i0 = sub - 1;
        const int64_t base = s_w[0][i0];
        const uint64_t m0 = s_nb[i0];
        if (threadIdx.x == 0) acc_push(a, row[base], m0);                  // {P[i0]}
        if (K >= 2)
            for (int x = threadIdx.x; x < i0; x += kScoreThreads)           // {P[i0], P[x]}
                acc_push(a, row[base + s_w[1][x]], m0 | s_nb[x]);
        if (K >= 3)
            for (int q = threadIdx.x; q < i0 * (i0 - 1) / 2; q += kScoreThreads) {
                int x, y;
                tri_unrank(q, x, y);
                acc_push(a, row[base + s_w[1][x] + s_w[2][y]], m0 | s_nb[x] | s_nb[y]);
            }
        if (K >= 4)
            for (int x = 2 + wave; x < i0; x += kScoreThreads / 64) {       // second member, by wavefront
                const int64_t bx = base + s_w[1][x];
                const uint64_t mx = m0 | s_nb[x];
                for (int q = lane; q < x * (x - 1) / 2; q += 64) {
                    int y, z;
                    tri_unrank(q, y, z);
                    acc_push(a, row[bx + s_w[2][y] + s_w[3][z]], mx | s_nb[y] | s_nb[z]);
                }
            }
    }
    // wavefront butterfly (skipped when nothing was folded), then the waves in order
    Acc r;
    if (__ballot(a.m != -INFINITY) != 0ull) {
        Acc one[1] = {a};
        r = acc_wave_reduce_scatter<1>(one, lane);
    } else {
        acc_init(r);
    }
    if (lane == 0) {
        s_red[wave].m = r.m;
        s_red[wave].s = r.s;
        s_red[wave].best = r.best;
        s_red[wave].sec = r.sec;
        s_red[wave].bm = r.bm;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Acc t;
        t.m = s_red[0].m;
        t.s = s_red[0].s;
        t.best = s_red[0].best;
        t.sec = s_red[0].sec;
        t.bm = s_red[0].bm;
#pragma unroll
        for (int w = 1; w < kScoreThreads / 64; ++w) {
            Acc o;
            o.m = s_red[w].m;
            o.s = s_red[w].s;
            o.best = s_red[w].best;
            o.sec = s_red[w].sec;
            o.bm = s_red[w].bm;
            acc_merge(t, o);
        }
        Partial pt;
        pt.m = t.m;
        pt.s = t.s;
        pt.best = t.best;
        pt.second = t.sec;
        pt.bmask = t.bm;
        A.part[((int64_t)ob * n + sub) * n + node] = pt;
    }
}

// ------------------------------------------------------------------ host side

// Orders per block: a block folds every streamed entry into this many order states.
int pick_bt(const TableT *t, int B)
{
    // 4 orders per block for 4 or more (256 chains at n=40 step 4-8% faster than with 8, whose
    // 95 registers per lane leave 5 wavefronts per SIMD resident instead of 7; at n=60 8 is 3-5%
    // faster, which the autotuners pick per table and batch-size bucket)
    int bt = B >= 4 ? 4 : (B >= 2 ? 2 : 1);
    // autotuned choice for the batch-size bucket, if any
    const int k = TableT::bucket(B);
    if (t->tuned_bt[k] > 0 && t->tuned_bt[k] <= B) bt = t->tuned_bt[k];
    return bt;
}

// Scoring workspace for up to `B` orders: the chunk partials.
bnos_status ensure_workspace(TableT *t, int B)
{
    const int64_t need = t->workspace_bytes_for(B);
    if (t->part_bytes >= need) return BNOS_OK;
    // A launch still in flight may use the old buffer.
    BNOS_HIP(hipDeviceSynchronize());
    BNOS_HIP(hipFree(t->d_part));
    t->d_part = nullptr;
    t->part_bytes = 0;
    const int64_t want = need > t->workspace_bytes_for(64) ? need : t->workspace_bytes_for(64);
    hipError_t e = hipMalloc(&t->d_part, (size_t)want);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc scoring workspace: ") + hipGetErrorString(e));
        t->d_part = nullptr;
        return e == hipErrorOutOfMemory ? BNOS_E_NOMEM : BNOS_E_DEVICE;
    }
    t->part_bytes = want;
    return BNOS_OK;
}

// Adds the oldest timed launch in the ring to the totals and frees its slot.
static bnos_status harvest_oldest(TableT *t)
{
    const size_t k = t->ev_head;
    BNOS_HIP(hipEventSynchronize(t->ev_stop[k]));
    float ms = 0.f;
    BNOS_HIP(hipEventElapsedTime(&ms, t->ev_start[k], t->ev_stop[k]));
    t->timed_ms += ms;
    t->timed_launches += 1;
    t->timed_passes += t->ev_passes[k];
    t->ev_head = (k + 1) % TableT::kEventRing;
    t->ev_count--;
    return BNOS_OK;
}

// The event pair for the next timed launch, which makes `passes` passes over
// the table.  With the ring full, the oldest launch (kEventRing launches back,
// long finished in a stream of launches) is read first.
static bnos_status next_events(TableT *t, hipEvent_t &e0, hipEvent_t &e1, int64_t passes)
{
    bnos_status s;
    if (t->ev_start.size() < TableT::kEventRing) {
        BNOS_HIP(hipSetDevice(t->device));
        while (t->ev_start.size() < TableT::kEventRing) {
            hipEvent_t a, b;
            BNOS_HIP(hipEventCreate(&a));
            if (hipEventCreate(&b) != hipSuccess) {
                hipEventDestroy(a);
                set_error("hipEventCreate failed");
                return BNOS_E_DEVICE;
            }
            t->ev_start.push_back(a);
            t->ev_stop.push_back(b);
        }
        t->ev_passes.assign(TableT::kEventRing, 0);
    }
    if (t->ev_count == TableT::kEventRing && (s = harvest_oldest(t)) != BNOS_OK) return s;
    const size_t k = (t->ev_head + t->ev_count) % TableT::kEventRing;
    t->ev_passes[k] = passes;
    t->ev_count++;
    e0 = t->ev_start[k];
    e1 = t->ev_stop[k];
    return BNOS_OK;
}

ScoreArgs score_args(const TableT *t, const int32_t *orders, int B, double *lse, double *maxs,
                     uint64_t *best, double *node_lse, float *node_second)
{
    ScoreArgs A;
    A.masks = t->d_masks;
    A.scores = t->d_scores;
    A.S_pad = t->S_pad;
    A.chunks = t->chunks_for(B);
    A.chunk_entries = t->chunk_entries_for(B);
    A.sum_chunks = t->S_pad / ((int64_t)t->pad_steps * kEntriesPerStep);
    A.sum_steps = t->pad_steps;
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
    A.tsub = t->d_tsub;
    A.anchor = t->computed_masks ? t->d_anchor : nullptr;
    const bool bound = t->score_bound && t->tile_skip;
    A.tmax = bound ? t->d_tmax : nullptr;
    A.cmask = bound ? t->d_cmask : nullptr;
    A.cscore = bound ? t->d_cscore : nullptr;
    A.cuts = nullptr;
    A.cut_ws = t->d_part ? reinterpret_cast<float *>(static_cast<char *>(t->d_part) + t->cuts_offset_for(B))
                         : nullptr;
    A.K = t->K;
    return A;
}

template <void (*KERNEL)(ScoreArgs)>
static void launch_one(dim3 grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1, const ScoreArgs &A)
{
    if (e0) hipExtLaunchKernelGGL(KERNEL, grid, dim3(kScoreThreads), 0, st, e0, e1, 0, A);
    else hipLaunchKernelGGL(KERNEL, grid, dim3(kScoreThreads), 0, st, A);
}

// With events, they take the kernel's own start and end (hipExtLaunchKernel),
// without the gap an event record on either side of the launch would add.
template <int BT>
static void launch_bt(const ScoreArgs &A, int nblocks_x, hipStream_t st, hipEvent_t e0, hipEvent_t e1)
{
    nblocks_x = (nblocks_x + kXcds - 1) / kXcds * kXcds;      // padded for xcd_block
    dim3 grid((unsigned)nblocks_x, (unsigned)((A.B + BT - 1) / BT));
    // without the saturation test when three steps cannot pass 2^64 (with K = 1 a step from
    // a single slot doubles the mask); with tile skipping a wavefront folds few tiles and waits
    // on their loads, so six are kept in flight, while the full scan streams the row and keeps
    // three (fewer registers, more wavefronts resident)
    const bool deep = A.tand != nullptr;
    if (BT == 1 && A.anchor && ((A.K >= 2 && A.n <= 63) || (A.K == 1 && A.n <= 61))) {
        if (deep) launch_one<k_score<1, true, true, 6>>(grid, st, e0, e1, A);
        else launch_one<k_score<1, true, true, 3>>(grid, st, e0, e1, A);
        return;
    }
    if (BT == 1 && A.anchor) {
        if (deep) launch_one<k_score<1, true, false, 6>>(grid, st, e0, e1, A);
        else launch_one<k_score<1, true, false, 3>>(grid, st, e0, e1, A);
        return;
    }
    if (e0) hipExtLaunchKernelGGL(k_score<BT>, grid, dim3(kScoreThreads), 0, st, e0, e1, 0, A);
    else hipLaunchKernelGGL(k_score<BT>, grid, dim3(kScoreThreads), 0, st, A);
}

// The streaming pass (k_score) with the table's block shape; timed when enabled.
// The workspace must already hold A.B orders.
bnos_status launch_stream(TableT *t, const ScoreArgs &A, hipStream_t st, int bt, bool allow_timing)
{
    bnos_status s;
    if (bt <= 0) bt = pick_bt(t, A.B);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (allow_timing && t->timing && t->timing_seen++ % t->timing_every == 0) {
        if ((s = next_events(t, e0, e1, (A.B + bt - 1) / bt)) != BNOS_OK) return s;
    }
    const int nbx = t->n * A.chunks;
    ScoreArgs A2 = A;
    if (bt > 1 && A.tmax && A.tand && A.cut_ws) {
        // every (order, node) cut once, before the blocks that stream the node's row
        const int64_t pairs = (int64_t)A.B * A.n;
        hipLaunchKernelGGL(k_bound_pre, dim3((unsigned)((pairs + kScoreThreads / 64 - 1) / (kScoreThreads / 64))),
                           dim3(kScoreThreads), 0, st, A);
        A2.cuts = A.cut_ws;
    }
    if (bt == 8) launch_bt<8>(A2, nbx, st, e0, e1);
    else if (bt == 4) launch_bt<4>(A2, nbx, st, e0, e1);
    else if (bt == 2) launch_bt<2>(A2, nbx, st, e0, e1);
    else launch_bt<1>(A2, nbx, st, e0, e1);
    BNOS_HIP(hipGetLastError());
    return BNOS_OK;
}

// The gather pass (k_gather) over B orders; A.chunks becomes n (one partial
// slot per top member plus the empty set).  Timed when enabled.
bnos_status launch_gather(TableT *t, ScoreArgs &A, hipStream_t st, bool allow_timing)
{
    bnos_status s;
    A.chunks = t->n;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (allow_timing && t->timing && t->timing_seen++ % t->timing_every == 0) {
        if ((s = next_events(t, e0, e1, 0)) != BNOS_OK) return s;
    }
    dim3 grid((unsigned)(t->n * t->n), (unsigned)A.B);
    if (e0) hipExtLaunchKernelGGL(k_gather, grid, dim3(kScoreThreads), 0, st, e0, e1, 0, A, t->d_nsets, t->K);
    else hipLaunchKernelGGL(k_gather, grid, dim3(kScoreThreads), 0, st, A, t->d_nsets, t->K);
    BNOS_HIP(hipGetLastError());
    return BNOS_OK;
}

// The per-order merge of a scoring launch's partials.
bnos_status launch_merge(const ScoreArgs &A, hipStream_t st)
{
    hipLaunchKernelGGL(k_merge, dim3(A.B), dim3(kMergeWaves * 64), 0, st, A);
    BNOS_HIP(hipGetLastError());
    return BNOS_OK;
}

static bnos_status score_impl(TableT *t, const int32_t *orders, int B, double *lse, double *maxs,
                              uint64_t *best, double *node_lse, float *node_second, hipStream_t st)
{
    bnos_status s = ensure_workspace(t, B);
    if (s != BNOS_OK) return s;
    ScoreArgs A = score_args(t, orders, B, lse, maxs, best, node_lse, node_second);
    if (t->gather_for(B)) s = launch_gather(t, A, st);
    else s = launch_stream(t, A, st, 0);
    if (s != BNOS_OK) return s;
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
    if (enable < 0) { set_error("timing: enable must be >= 0"); return BNOS_E_RANGE; }
    t->timing = enable != 0;
    t->timing_every = enable > 0 ? enable : 1;
    t->timing_seen = 0;
    t->ev_head = 0;
    t->ev_count = 0;
    t->timed_ms = 0.0;
    t->timed_launches = 0;
    t->timed_passes = 0;
    if (t->timing) {                 // create the event ring now, outside any timed launch
        hipEvent_t e0, e1;
        bnos_status s = next_events(t, e0, e1, 0);
        t->ev_count = 0;
        if (s != BNOS_OK) return s;
    }
    return BNOS_OK;
}

template <int BT>
static void launch_count(const ScoreArgs &A, int nbx, unsigned *counts)
{
    dim3 grid((unsigned)nbx, (unsigned)((A.B + BT - 1) / BT));
    hipLaunchKernelGGL(k_count_tiles<BT>, grid, dim3(kScoreThreads), 0, 0, A, counts);
}

extern "C" bnos_status bnos_table_count_tiles(bnos_table h, const int32_t *orders, int32_t B, int64_t *tiles_read,
                                              int64_t *tiles_per_pass)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (!orders) { set_error("NULL argument"); return BNOS_E_INVALID; }
    if (B < 1 || B > (1 << 20)) { set_error("B outside [1, 2^20]"); return BNOS_E_RANGE; }
    BNOS_HIP(hipSetDevice(t->device));
    ScoreArgs A = score_args(t, orders, B, nullptr, nullptr, nullptr, nullptr, nullptr);
    A.tand = t->d_tand;
    const int bt = pick_bt(t, B);
    const int nbx = t->n * A.chunks;
    const int64_t blocks = (int64_t)nbx * ((B + bt - 1) / bt);
    unsigned *d = nullptr;
    BNOS_HIP(hipMalloc((void **)&d, sizeof(unsigned) * blocks));
    if (bt == 8) launch_count<8>(A, nbx, d);
    else if (bt == 4) launch_count<4>(A, nbx, d);
    else if (bt == 2) launch_count<2>(A, nbx, d);
    else launch_count<1>(A, nbx, d);
    std::vector<unsigned> hc((size_t)blocks);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipMemcpy(hc.data(), d, sizeof(unsigned) * blocks, hipMemcpyDeviceToHost);
    hipFree(d);
    if (e != hipSuccess) { set_error(std::string("count tiles: ") + hipGetErrorString(e)); return BNOS_E_DEVICE; }
    int64_t tot = 0;
    for (unsigned v : hc) tot += v;
    if (tiles_read) *tiles_read = tot;
    if (tiles_per_pass) *tiles_per_pass = (int64_t)t->n * (t->S_pad / 64);
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_tile_skip(bnos_table h, int32_t enable)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    t->tile_skip = enable != 0;
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_score_bound(bnos_table h, int32_t enable)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    t->score_bound = enable != 0;
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_computed_masks(bnos_table h, int32_t enable)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    t->computed_masks = enable != 0;
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_timing_read(bnos_table h, double *total_ms, int64_t *launches,
                                              int64_t *table_passes)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    bnos_status s;
    while (t->ev_count > 0)
        if ((s = harvest_oldest(t)) != BNOS_OK) return s;
    if (total_ms) *total_ms = t->timed_ms;
    if (launches) *launches = t->timed_launches;
    if (table_passes) *table_passes = t->timed_passes;
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_autotune(bnos_table h, const int32_t *orders, int32_t B, int32_t reps, void *stream,
                                           int32_t *chunk_steps, int32_t *orders_per_block, int32_t *gather,
                                           double *ms_per_launch)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (!orders) { set_error("NULL argument"); return BNOS_E_INVALID; }
    if (B < 1 || B > (1 << 20) || reps < 1 || reps > 1000) { set_error("B or reps out of range"); return BNOS_E_RANGE; }
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipDeviceSynchronize());
    const int bk = TableT::bucket(B);
    const int old_cs = t->tuned_cs[bk], old_bt = t->tuned_bt[bk], old_g = t->tuned_gather[bk];
    t->tuned_gather[bk] = 0;
    const bool old_timing = t->timing;
    t->timing = false;
    double *d_out = nullptr;
    uint64_t *d_best = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void **)&d_out, sizeof(double) * 2 * (size_t)B);
    if (e == hipSuccess) e = hipMalloc((void **)&d_best, sizeof(uint64_t) * (size_t)B * t->n);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    double best_ms = 1e300;
    int best_cs = t->chunk_entries / kEntriesPerStep, best_bt = pick_bt(t, B);
    bnos_status s = BNOS_OK;
    for (int cs = 1; cs <= t->pad_steps && e == hipSuccess && s == BNOS_OK; cs <<= 1) {
        t->tuned_cs[bk] = cs;
        if ((s = ensure_workspace(t, B)) != BNOS_OK) break;
        for (int bt = 1; bt <= 8 && bt <= B && s == BNOS_OK; bt <<= 1) {
            ScoreArgs A = score_args(t, orders, B, d_out, d_out + B, d_best, nullptr, nullptr);
            for (int r = 0; r <= reps && s == BNOS_OK; ++r) {
                if (r == 1) e = hipEventRecord(e0, st);
                if ((s = launch_stream(t, A, st, bt)) != BNOS_OK) break;
                hipLaunchKernelGGL(k_merge, dim3(B), dim3(kMergeWaves * 64), 0, st, A);
            }
            if (s != BNOS_OK) break;
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && ms / reps < best_ms) {
                best_ms = ms / reps;
                best_cs = cs;
                best_bt = bt;
            }
        }
    }
    // the gather pass (enumerating the consistent sets), where the table allows it
    int best_g = 0;
    if (t->K <= kGatherMaxK && e == hipSuccess && s == BNOS_OK) {
        t->tuned_cs[bk] = best_cs;
        if ((s = ensure_workspace(t, B)) == BNOS_OK) {
            ScoreArgs A = score_args(t, orders, B, d_out, d_out + B, d_best, nullptr, nullptr);
            for (int r = 0; r <= reps && s == BNOS_OK; ++r) {
                if (r == 1) e = hipEventRecord(e0, st);
                if ((s = launch_gather(t, A, st)) != BNOS_OK) break;
                hipLaunchKernelGGL(k_merge, dim3(B), dim3(kMergeWaves * 64), 0, st, A);
            }
            if (e == hipSuccess && s == BNOS_OK) e = hipEventRecord(e1, st);
            if (e == hipSuccess && s == BNOS_OK) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess && s == BNOS_OK) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && s == BNOS_OK && ms / reps < best_ms) {
                best_ms = ms / reps;
                best_g = 1;
            }
        }
    }
    if (e0) hipEventDestroy(e0);
    if (e1) hipEventDestroy(e1);
    hipFree(d_out);
    hipFree(d_best);
    t->timing = old_timing;
    if (s != BNOS_OK || e != hipSuccess) {
        t->tuned_cs[bk] = old_cs;
        t->tuned_bt[bk] = old_bt;
        t->tuned_gather[bk] = old_g;
        if (s == BNOS_OK) { set_error(std::string("autotune: ") + hipGetErrorString(e)); s = BNOS_E_DEVICE; }
        return s;
    }
    t->tuned_cs[bk] = best_cs;
    t->tuned_bt[bk] = best_bt;
    t->tuned_gather[bk] = best_g;
    if ((s = ensure_workspace(t, B)) != BNOS_OK) return s;
    if (chunk_steps) *chunk_steps = best_cs;
    if (orders_per_block) *orders_per_block = best_bt;
    if (gather) *gather = best_g;
    if (ms_per_launch) *ms_per_launch = best_ms;
    return BNOS_OK;
}

extern "C" bnos_status bnos_table_set_launch(bnos_table h, int32_t B, int32_t gather, int32_t chunk_steps,
                                             int32_t orders_per_block)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (B < 1 || B > (1 << 20)) { set_error("B outside [1, 2^20]"); return BNOS_E_RANGE; }
    if (gather != 0 && gather != 1) { set_error("gather must be 0 or 1"); return BNOS_E_INVALID; }
    if (gather && t->K > kGatherMaxK) { set_error("the gather pass needs K <= 4"); return BNOS_E_RANGE; }
    if (chunk_steps != 0 && (chunk_steps < 1 || chunk_steps > t->pad_steps || (chunk_steps & (chunk_steps - 1)) != 0)) {
        set_error("chunk_steps must be 0 or a power of two dividing the row padding");
        return BNOS_E_RANGE;
    }
    if (orders_per_block != 0 && orders_per_block != 1 && orders_per_block != 2 && orders_per_block != 4 &&
        orders_per_block != 8) {
        set_error("orders_per_block must be 0, 1, 2, 4 or 8");
        return BNOS_E_RANGE;
    }
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipDeviceSynchronize());        // launches in flight keep their shapes and workspace
    const int bk = TableT::bucket(B);
    t->tuned_gather[bk] = gather;
    t->tuned_cs[bk] = chunk_steps;
    t->tuned_bt[bk] = orders_per_block;
    return ensure_workspace(t, B);
}

// ------------------------------------------------------------------ scoring without allocation

namespace bnos {

// Partials of bnos_score_orders_noalloc: one fixed device array per GPU (every
// device the library runs on holds its own copy until the process ends).  In
// host code `scratch` names a host-side stand-in, not device memory: only the
// address hipGetSymbolAddress returns for the current device may reach a
// kernel or a copy.
constexpr size_t kNoAllocScratchBytes = size_t(16) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxScratchDevices] = {};

// Device address of `scratch` on `device` (which must be current), resolved on
// the first call for that device.
static bnos_status scratch_on(int device, void **out)
{
    if (device < 0 || device >= kMaxScratchDevices) {
        set_error("device id above the library's scratch table");
        return BNOS_E_RANGE;
    }
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error(std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
            return BNOS_E_DEVICE;
        }
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return BNOS_OK;
}

}  // namespace bnos

extern "C" bnos_status bnos_score_orders_noalloc(bnos_table h, const int32_t *orders, int32_t B, double *lse,
                                                 double *maxs, uint64_t *best, double *node_lse,
                                                 float *node_second, void *stream)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (B < 1 || B > (1 << 20)) { set_error("B outside [1, 2^20]"); return BNOS_E_RANGE; }
    if (!orders || !lse || !maxs || !best) { set_error("NULL argument"); return BNOS_E_INVALID; }
    // partials [B][slots][n]: one slot per chunk, or per top member + the empty set in the gather pass
    // and after them (256-byte aligned) each order's score-bound cut per node
    const int64_t slots = t->gather_for(B) ? t->n : t->chunks_for(B);
    const int64_t part_bytes = (int64_t)B * slots * t->n * (int64_t)sizeof(Partial);
    const int64_t cuts_off = (part_bytes + 255) & ~(int64_t)255;
    const int64_t need = cuts_off + (int64_t)B * t->n * (int64_t)sizeof(float);
    if (need > (int64_t)kNoAllocScratchBytes) {
        set_error("B = " + std::to_string(B) + " orders need " + std::to_string(need) +
                  " bytes of scoring partials and cuts, above the fixed " + std::to_string(kNoAllocScratchBytes) +
                  "-byte scratch array of the allocation-free call");
        return BNOS_E_RANGE;
    }
    BNOS_HIP(hipSetDevice(t->device));
    void *part = nullptr;
    bnos_status s = scratch_on(t->device, &part);
    if (s != BNOS_OK) return s;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    ScoreArgs A = score_args(t, orders, B, lse, maxs, best, node_lse, node_second);
    A.part = reinterpret_cast<Partial *>(part);
    A.cut_ws = reinterpret_cast<float *>(static_cast<char *>(part) + cuts_off);
    if (t->gather_for(B)) s = launch_gather(t, A, st, false);
    else s = launch_stream(t, A, st, 0, false);
    if (s != BNOS_OK) return s;
    return launch_merge(A, st);
}
