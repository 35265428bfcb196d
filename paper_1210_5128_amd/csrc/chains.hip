// Metropolis-Hastings over node orders on the device (Sec. III.C): batched
// chains, one streaming pass per iteration for all chains' proposals, the
// merge + accept/reject + best-graph record + next proposal fused into one
// kernel, and sweeps of iterations captured as HIP graphs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "bnos_internal.h"
#include "score_device.h"
#include "mlp_device.h"

namespace bnos {

// ------------------------------------------------------------------ random numbers

// SplitMix64 finalizer (Steele, Lea & Flood, OOPSLA 2014).
__device__ __forceinline__ uint64_t sm64_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// One draw per (seed, chain, purpose, step); purposes: 0 shuffle, 1/2 swap
// positions, 3 acceptance uniform.
__device__ __forceinline__ uint64_t rng_draw(uint64_t seed, uint64_t chain, uint64_t purpose, uint64_t step)
{
    const uint64_t key = sm64_mix(seed ^ sm64_mix(chain * 8ull + purpose + 1ull));
    return sm64_mix(key + (step + 1ull) * 0x9E3779B97F4A7C15ull);
}

__device__ __forceinline__ uint32_t rng_below(uint64_t x, uint32_t m)
{
    return (uint32_t)(((x >> 32) * (uint64_t)m) >> 32);
}

__device__ __forceinline__ double rng_unit_open(uint64_t x)
{
    return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

__device__ __forceinline__ void rng_pair(uint64_t seed, uint64_t chain, int n, uint64_t step, int &a, int &b)
{
    uint32_t x = rng_below(rng_draw(seed, chain, 1, step), (uint32_t)n);
    uint32_t y = rng_below(rng_draw(seed, chain, 2, step), (uint32_t)(n - 1));
    y += (y >= x) ? 1u : 0u;
    a = (int)x;
    b = (int)y;
}

// ------------------------------------------------------------------ kernels

// Chains of one table.  Kernels take an array of these (one per table) and
// find their table from prefix bases over the grid.
struct ChainView {
    int n, C, target;
    uint64_t seed;
    int64_t chain0;            // RNG stream id of this table's chain 0
    int64_t t_first, t_last;   // iterations done before this call; last iteration to run
    int32_t *cur;              // [C][n] current orders (state)
    int32_t *prop;             // [C][n] orders being scored
    double *score;             // [C] target score of the current order (state)
    double *best_score;        // [C] (state)
    uint64_t *best_graph;      // [C][n] (state)
    int64_t *accepted;         // [C] (state)
    int64_t *t;                // [C] iteration whose proposal is being scored
    double *node_l;            // [C][n] per-node log-sum-exp of the current order
    double *node_m;            // [C][n] per-node best score of the current order
    uint64_t *node_best;       // [C][n] per-node best parent set of the current order
    uint64_t *wmask;           // [C] nodes whose predecessor set the proposal changes
    int32_t *wl_count;         // [n] chains listing each node in their window
    int32_t *wl_list;          // [n][C]
    uint8_t *ppos;             // [C][n] position of each node in the order being scored
    float *cuts;               // [C][n] score-bound cut of each window node of the proposal, or null
    double *trace;             // [C][trace_len] or null
    int trace_every;
    int64_t trace_len;
    uint8_t *flags;            // [C][iterations] or null
    int64_t iterations;
    double *node_sec;          // [C][n] per-node second-best score of the current order
    const double *nstat;       // [n][5] static node features of the table
    // learned proposal
    int proposal;              // 0 uniform, 1 learned
    double eps;
    MlpView mlp;
    float *cur_logit;          // [C][n] network scores of the current order
    double *lq_fwd;            // [C] ln q(pending pair | current order)
    int32_t *pend;             // [C][2] node ids of the pending pair
    // harvest of accepted moves
    float *hv_feat;            // [C][hv_cap][n][8] or null
    int32_t *hv_pair;          // [C][hv_cap][2]
    int64_t *hv_count;         // [C]
    int64_t hv_cap;
    // edges traced per iteration (mixing diagnostics)
    int n_edges;               // 0 = off
    const int32_t *edge_cp;    // [n_edges][2] (child, parent), device copy
    uint32_t *edge_trace;      // [C][trace_len]
    // record of the best distinct graphs
    int topk;                  // 0 = off
    uint64_t *top_graph;       // [C][topk][n]
    double *top_score;         // [C][topk]
    int32_t *top_count;        // [C]
};

__device__ __forceinline__ uint64_t all_nodes(int n) { return n == 64 ? ~0ull : ((1ull << n) - 1ull); }

// Block per chain.  Fresh start: the initial order (iteration 0 adopts it).
// Resume: the saved current order is re-scored first to rebuild the per-node
// caches (same arithmetic, so the same values), then iteration t_first+1 follows.
__global__ __launch_bounds__(64) void k_chain_init(const ChainView *__restrict__ views,
                                                   const int64_t *__restrict__ chain_base, int T)
{
    const int k = find_segment(chain_base, T, (int64_t)blockIdx.x);
    const ChainView &H = views[k];
    const int c = (int)((int64_t)blockIdx.x - chain_base[k]);
    const int lane = threadIdx.x;
    const int n = H.n;
    const uint64_t chain = (uint64_t)(H.chain0 + c);
    if (H.t_first == 0) {
        if (lane == 0) {
            int32_t ord[64];
            for (int p = 0; p < n; ++p) ord[p] = p;
            for (int p = n - 1; p >= 1; --p) {
                uint32_t j = rng_below(rng_draw(H.seed, chain, 0, (uint64_t)p), (uint32_t)(p + 1));
                int32_t tmp = ord[p];
                ord[p] = ord[j];
                ord[j] = tmp;
            }
            for (int p = 0; p < n; ++p) {
                H.prop[(int64_t)c * n + p] = ord[p];
                H.ppos[(int64_t)c * n + ord[p]] = (uint8_t)p;
            }
            H.accepted[c] = 0;
            if (H.topk > 0) H.top_count[c] = 0;
        }
    } else {
        if (lane < n) {
            const int32_t v = H.cur[(int64_t)c * n + lane];
            H.prop[(int64_t)c * n + lane] = v;
            H.ppos[(int64_t)c * n + v] = (uint8_t)lane;
        }
        if (lane == 0 && H.trace) H.trace[(int64_t)c * H.trace_len] = H.score[c];
    }
    if (lane == 0) {
        H.t[c] = H.t_first;
        H.wmask[c] = all_nodes(n);
    }
}

// Block per (table, node): the chains whose proposal window contains the node,
// grouped by the node's position in their proposals (kPosBins ranges of
// positions, in increasing order; chain order within a range).  A scoring block
// takes consecutive listed chains, and chains where the node sits at similar
// positions have predecessor sets of similar size, so the union of the tiles
// they need is smaller.  The grouping changes no result: a tile no consistent
// entry of a chain lies in leaves that chain's state unchanged.
constexpr int kListThreads = 1024;
constexpr int kPosBins = 8;
__device__ __forceinline__ void worklist_block(const ChainView *__restrict__ views,
                                               const int64_t *__restrict__ node_base, int T, int64_t blk)
{
    __shared__ int s_cnt[kPosBins][kListThreads / 64];   // per bin, chains listed by each wave
    __shared__ int s_run[kPosBins];                       // per bin, list position reached
    const int k = find_segment(node_base, T, blk);
    const ChainView &H = views[k];
    const int node = (int)(blk - node_base[k]);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // the bin of chain c for this node, or -1 if its window does not hold the node
    auto bin_of = [&](int c) -> int {
        if (c >= H.C || !((H.wmask[c] >> node) & 1ull)) return -1;
        return (int)H.ppos[(int64_t)c * H.n + node] * kPosBins / H.n;
    };
    // pass 1: chains per bin, so that each bin's run of the list starts where the
    // previous bins' end (the list is bin by bin, chains ascending within a bin)
    if (threadIdx.x < kPosBins) s_run[threadIdx.x] = 0;
    __syncthreads();
    for (int base = 0; base < H.C; base += kListThreads) {
        const int bn = bin_of(base + threadIdx.x);
#pragma unroll
        for (int b = 0; b < kPosBins; ++b) {
            const int cnt = __popcll(__ballot(bn == b));
            if (lane == 0 && cnt) atomicAdd(&s_run[b], cnt);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int start = 0;
        for (int b = 0; b < kPosBins; ++b) {
            const int c = s_run[b];
            s_run[b] = start;
            start += c;
        }
        H.wl_count[node] = start;
    }
    __syncthreads();
    // pass 2: each listed chain at its bin's next free place, in chain order
    for (int base = 0; base < H.C; base += kListThreads) {
        const int bn = bin_of(base + threadIdx.x);
        int rank = 0;
#pragma unroll
        for (int b = 0; b < kPosBins; ++b) {
            const uint64_t bal = __ballot(bn == b);
            if (bn == b) rank = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == 0) s_cnt[b][wave] = __popcll(bal);
        }
        __syncthreads();
        if (bn >= 0) {
            int off = s_run[bn] + rank;
            for (int w = 0; w < wave; ++w) off += s_cnt[bn][w];
            H.wl_list[(int64_t)node * H.C + off] = base + threadIdx.x;
        }
        __syncthreads();
        if (threadIdx.x < kPosBins) {
            int tot = 0;
            for (int w = 0; w < kListThreads / 64; ++w) tot += s_cnt[threadIdx.x][w];
            s_run[threadIdx.x] += tot;
        }
        __syncthreads();
    }
}

// Score bound of the proposals: the wavefront of (chain, node) pair g over all
// tables (node g mod the total node count, chain g div it) computes the cut of
// the chain's proposal for that node when the node is in the chain's window, so
// that the scoring blocks read it instead of each computing it.
__device__ __forceinline__ void chain_cut_wave(const TabView *__restrict__ tviews,
                                               const ChainView *__restrict__ views,
                                               const int64_t *__restrict__ node_base, int T, int C, int64_t g,
                                               int lane)
{
    const int64_t nodes = node_base[T];
    if (g >= nodes * C) return;                              // uniform per wavefront
    const int c = (int)(g / nodes);
    const int64_t gn = g - (int64_t)c * nodes;
    const int k = find_segment(node_base, T, gn);
    const ChainView &H = views[k];
    const int node = (int)(gn - node_base[k]);
    if (!H.cuts || !((H.wmask[c] >> node) & 1ull)) return;  // uniform
    const int n = H.n;
    const int64_t ci = (int64_t)c * n + node;
    // Once the chain holds an adopted order (after its first iteration in this
    // call), the node's best parent set in that order and its score are cached;
    // if the proposal still allows that set, its score bounds the proposal's best
    // from below, often far more tightly than the listed candidates (the node's
    // predecessors change by at most the two swapped nodes).  The three reads are
    // issued with the positions' and used only once the caches are valid.
    const bool cached = H.t[c] > H.t_first;
    const uint64_t bset = H.node_best[ci];
    const double bscore = H.node_m[ci];                      // an FP32 score held in FP64: exact
    const uint8_t *pp = H.ppos + (int64_t)c * n;
    const int pv = pp[node];
    const int pu = pp[lane < n ? lane : n - 1];              // every lane loads (no branch)
    const uint64_t pred = __ballot(lane < n && pu < pv);
    const bool use = cached && (bset & ~pred) == 0ull;
    const float cut = wave_bound_cut(tviews[k], node, ~pred, lane, use ? (float)bscore : -INFINITY,
                                     use ? bset : ~0ull);
    if (lane == 0) H.cuts[ci] = cut;
}

// One launch per iteration before the scoring: blocks below the total node count
// build the work lists (a block per (table, node)); with the score bound, the
// blocks after them compute the cuts (16 (chain, node) pairs per block, one per
// wavefront).  Both parts only read the chains' windows and positions, which
// the previous iteration's k_chain_step wrote, so they run side by side instead
// of as two launches.
__global__ __launch_bounds__(kListThreads) void k_worklist(const TabView *__restrict__ tviews,
                                                           const ChainView *__restrict__ views,
                                                           const int64_t *__restrict__ node_base, int T, int C)
{
    const int64_t nodes = node_base[T];
    const int64_t blk = blockIdx.x;
    if (blk < nodes) worklist_block(views, node_base, T, blk);   // uniform per block
    else   // the wavefront index read as uniform, so the pair's reads go through scalar loads
        chain_cut_wave(tviews, views, node_base, T, C,
                       (blk - nodes) * (kListThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6),
                       threadIdx.x & 63);
}

// Offer graph g (lane i holds node i's parent mask) with max score M to chain
// c's record of best distinct graphs (wave 0, all lanes).  Records are sorted
// by decreasing score; the new graph goes after every record scoring >= M.  An
// identical graph has the identical score (the same FP32 entries summed in the
// same order), so only records of equal score are compared for duplicates.
__device__ __forceinline__ void topk_offer(const ChainView &H, int c, int n, int lane, double M, uint64_t g)
{
    const int K = H.topk;
    uint64_t *G = H.top_graph + (int64_t)c * K * n;
    double *Sc = H.top_score + (int64_t)c * K;
    const int cnt = H.top_count[c];
    const double mine = lane < cnt ? Sc[lane] : 0.0;
    const int pos = __popcll(__ballot(lane < cnt && mine >= M));
    if (pos >= K) return;
    uint64_t eq = __ballot(lane < cnt && mine == M);
    bool dup = false;
    while (eq) {
        const int r = __builtin_ctzll(eq);
        eq &= eq - 1;
        const uint64_t x = lane < n ? G[(int64_t)r * n + lane] : 0ull;
        dup = dup || (__ballot(lane < n && x != g) == 0ull);
    }
    if (dup) return;
    const int last = cnt < K ? cnt : K - 1;
    if (lane < n) {
        for (int r = last; r > pos; --r) G[(int64_t)r * n + lane] = G[(int64_t)(r - 1) * n + lane];
        G[(int64_t)pos * n + lane] = g;
    }
    const bool shift = lane > pos && lane <= last;
    const double prev = shift ? Sc[lane - 1] : 0.0;
    if (shift) Sc[lane] = prev;
    if (lane == pos) Sc[pos] = M;
    if (lane == 0 && cnt < K) H.top_count[c] = cnt + 1;
}

// Block per chain: merge the chunk partials of the window nodes, combine with
// the cached values of the other nodes (per-order sums in node order with a
// fixed butterfly, as a full rescoring would), take the MH decision (with the
// proposal ratio q(pair|new)/q(pair|old) for the learned proposal), update the
// caches and the best-graph record, harvest the accepted move, and draw the
// next proposal.
constexpr int kStepWaves = 16;

__global__ __launch_bounds__(kStepWaves * 64) void k_chain_step(const TabView *__restrict__ tviews,
                                                                 const ChainView *__restrict__ views,
                                                                 const int64_t *__restrict__ chain_base, int T)
{
    __shared__ double s_l[64], s_b[64], s_s[64];
    __shared__ uint64_t s_bm[64];
    __shared__ int s_nodes[64], s_posp[64], s_posc[64];
    __shared__ int s_cnt;
    __shared__ float s_feat[64 * kF];
    __shared__ MlpLds s_mlp;
    __shared__ MergeLds s_merge;
    const int k = find_segment(chain_base, T, (int64_t)blockIdx.x);
    const ChainView &H = views[k];
    const TabView &V = tviews[k];
    const int c = (int)((int64_t)blockIdx.x - chain_base[k]);
    const int n = H.n;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int chunks = V.chunks;
    const int64_t row = (int64_t)c * n;
    const uint64_t wm = H.wmask[c];
    const bool learned = H.proposal == 1;
    const bool harvest = H.hv_feat != nullptr;
    // wave 0's reads of the chain's cached values and counters, requested before
    // the merge so that their latency overlaps it (only this block reads or
    // writes chain c's rows)
    double l0 = 0.0, m0 = 0.0, s0 = 0.0, score0 = 0.0, best0 = 0.0;
    int64_t t0 = 0, nacc0 = 0;
    if (wave == 0) {
        if (lane < n) {
            l0 = H.node_l[row + lane];
            m0 = H.node_m[row + lane];
            s0 = H.node_sec[row + lane];
        }
        t0 = H.t[c];
        score0 = H.score[c];
        best0 = H.best_score[c];
        nacc0 = H.accepted[c];
        const bool in = lane < n && ((wm >> lane) & 1ull);
        const uint64_t bal = __ballot(in);
        if (in) s_nodes[__popcll(bal & ((1ull << lane) - 1ull))] = lane;
        if (lane == 0) s_cnt = __popcll(bal);
        if (lane < n) {
            s_posp[H.prop[row + lane]] = lane;
            s_posc[H.cur[row + lane]] = lane;
        }
    }
    __syncthreads();
    const int cnt = s_cnt;
    {
        // lane j of the merging waves takes window node s_nodes[j]
        const Acc r = merge_nodes(V.part + (int64_t)c * chunks * n, n, chunks, lane < cnt ? s_nodes[lane] : -1,
                                  s_merge);
        if (wave == 0 && lane < cnt) {
            const int i = s_nodes[lane];
            s_l[i] = (double)r.m + log((double)r.s);
            s_b[i] = (double)r.best;
            s_s[i] = (double)r.sec;
            s_bm[i] = r.bm;
        }
    }
    __syncthreads();
    if (learned) {
        // features of the proposal order, then its node scores
        if (tid < n) {
            const int i = tid;
            const bool in = (wm >> i) & 1ull;
            const double best = in ? s_b[i] : m0;   // tid < n: wave 0, lane i
            const double sec = in ? s_s[i] : s0;
            float *f = s_feat + i * kF;
            f[0] = (float)s_posp[i] / (float)n;
            f[1] = (float)best;
            f[2] = isinf(sec) ? 0.f : (float)(best - sec);
#pragma unroll
            for (int j = 0; j < 5; ++j) f[3 + j] = (float)H.nstat[i * 5 + j];
        }
        __syncthreads();
        mlp_forward_block(H.mlp, s_feat, n, s_mlp, nullptr);
    }
    if (wave != 0) return;

    const bool in = lane < n && ((wm >> lane) & 1ull);
    const double li = lane < n ? (in ? s_l[lane] : l0) : 0.0;
    const double mi = lane < n ? (in ? s_b[lane] : m0) : 0.0;
    const double si = lane < n ? (in ? s_s[lane] : s0) : 0.0;
    const double L = wave_sum_f64(li, lane);
    const double M = wave_sum_f64(mi, lane);
    const uint64_t chain = (uint64_t)(H.chain0 + c);
    const int64_t t = t0;
    const double nv = H.target ? M : L;
    int acc = 0, imp = 0, slot = -1;
    if (lane == 0) {
        if (t == H.t_first) {            // adopt the initial (or re-scored saved) order
            acc = 1;
            H.score[c] = nv;
            if (H.t_first == 0) {
                imp = 1;
                H.best_score[c] = M;
                if (H.trace) H.trace[(int64_t)c * H.trace_len] = nv;
            }
        } else {
            double ratio = nv - score0;
            if (learned) ratio += pair_logq_dev(s_mlp.logit, n, H.pend[2 * c], H.pend[2 * c + 1], H.eps) - H.lq_fwd[c];
            const double u = rng_unit_open(rng_draw(H.seed, chain, 3, (uint64_t)t));
            acc = log(u) < ratio;
            if (acc) {
                H.score[c] = nv;
                H.accepted[c] = nacc0 + 1;
                if (M > best0) {
                    H.best_score[c] = M;
                    imp = 1;
                }
                if (harvest && H.hv_count[c] < H.hv_cap) {
                    slot = (int)H.hv_count[c];
                    H.hv_count[c] += 1;
                    H.hv_pair[((int64_t)c * H.hv_cap + slot) * 2] = H.pend[2 * c];
                    H.hv_pair[((int64_t)c * H.hv_cap + slot) * 2 + 1] = H.pend[2 * c + 1];
                }
            }
            if (H.flags) H.flags[(int64_t)c * H.iterations + (t - H.t_first - 1)] = (uint8_t)acc;
            const int64_t kk = t - H.t_first;
            if (H.trace && kk % H.trace_every == 0)
                H.trace[(int64_t)c * H.trace_len + kk / H.trace_every] = acc ? nv : score0;   // the chain's score now
        }
    }
    acc = __shfl(acc, 0, 64);
    imp = __shfl(imp, 0, 64);
    slot = __shfl(slot, 0, 64);
    if (slot >= 0 && lane < n) {
        // raw features of the order before the move (current caches)
        float *f = H.hv_feat + (((int64_t)c * H.hv_cap + slot) * n + lane) * kF;
        const double best = m0, sec = s0;   // the caches before this step's update
        f[0] = (float)s_posc[lane] / (float)n;
        f[1] = (float)best;
        f[2] = isinf(sec) ? 0.f : (float)(best - sec);
#pragma unroll
        for (int j = 0; j < 5; ++j) f[3 + j] = (float)H.nstat[lane * 5 + j];
    }
    if (H.n_edges > 0) {
        const int64_t kk = t - H.t_first;
        if (kk % H.trace_every == 0) {
            // the current order's greedy graph after this step: the proposal's parents in
            // the window if accepted, else the cached ones
            const uint64_t gb = lane < n ? ((acc && in) ? s_bm[lane] : H.node_best[row + lane]) : 0ull;
            const int ech = lane < H.n_edges ? H.edge_cp[2 * lane] : 0;
            const int epa = lane < H.n_edges ? H.edge_cp[2 * lane + 1] : 0;
            const uint64_t gch = (uint64_t)__shfl((unsigned long long)gb, ech, 64);
            const uint64_t bits = __ballot(lane < H.n_edges && ((gch >> epa) & 1ull));
            if (lane == 0) H.edge_trace[(int64_t)c * H.trace_len + kk / H.trace_every] = (uint32_t)bits;
        }
    }
    int32_t v = 0;
    if (lane < n) {
        v = acc ? H.prop[row + lane] : H.cur[row + lane];
        if (acc) {
            H.cur[row + lane] = v;
            H.node_l[row + lane] = li;
            H.node_m[row + lane] = mi;
            H.node_sec[row + lane] = si;
            if (in) H.node_best[row + lane] = s_bm[lane];
            if (learned) H.cur_logit[row + lane] = s_mlp.logit[lane];
        }
    }
    if (imp && lane < n) H.best_graph[row + lane] = in ? s_bm[lane] : H.node_best[row + lane];
    if (H.topk > 0 && acc && !(t == H.t_first && H.t_first > 0))
        topk_offer(H, c, n, lane, M, lane < n ? (in ? s_bm[lane] : H.node_best[row + lane]) : 0ull);
    const int64_t t1 = t + 1;
    const bool next = t1 <= H.t_last;
    int a = 0, b = 0;
    if (next) {
        if (!learned) {
            rng_pair(H.seed, chain, n, (uint64_t)t1, a, b);
            const int na = __shfl(v, a, 64), nb = __shfl(v, b, 64);
            if (harvest && lane == 0) {
                H.pend[2 * c] = na;
                H.pend[2 * c + 1] = nb;
            }
        } else {
            // q: with probability eps a uniform pair of positions, else node a ~ p,
            // then node b ~ p without a (inverse CDF in node order, FP64).
            // The current order's scores: this step's if accepted, else unchanged.
            const float *lg = acc ? s_mlp.logit : H.cur_logit + row;
            const int *pos = acc ? s_posp : s_posc;
            const double mix = rng_unit_open(rng_draw(H.seed, chain, 4, (uint64_t)t1));
            int na = 0, nb = 0;
            if (mix < H.eps) {
                rng_pair(H.seed, chain, n, (uint64_t)t1, a, b);
                na = __shfl(v, a, 64);
                nb = __shfl(v, b, 64);
            } else if (lane == 0) {
                // p_i = exp(l_i - max) / sum, recomputed in each pass (no per-lane array)
                double mx = -1e300;
                for (int i = 0; i < n; ++i) mx = (double)lg[i] > mx ? (double)lg[i] : mx;
                double sum = 0.0;
                for (int i = 0; i < n; ++i) sum += exp((double)lg[i] - mx);
                const double u = rng_unit_open(rng_draw(H.seed, chain, 5, (uint64_t)t1));
                na = n - 1;
                double cu = 0.0;
                for (int i = 0; i < n; ++i) {
                    cu += exp((double)lg[i] - mx) / sum;
                    if (u < cu) { na = i; break; }
                }
                const double pna = exp((double)lg[na] - mx) / sum;
                const double w2 = rng_unit_open(rng_draw(H.seed, chain, 6, (uint64_t)t1)) * (1.0 - pna);
                nb = (na == n - 1) ? n - 2 : n - 1;
                cu = 0.0;
                for (int i = 0; i < n; ++i) {
                    if (i == na) continue;
                    cu += exp((double)lg[i] - mx) / sum;
                    if (w2 < cu) { nb = i; break; }
                }
                a = pos[na];
                b = pos[nb];
            }
            a = __shfl(a, 0, 64);
            b = __shfl(b, 0, 64);
            na = __shfl(na, 0, 64);
            nb = __shfl(nb, 0, 64);
            if (lane == 0) {
                H.pend[2 * c] = na;
                H.pend[2 * c + 1] = nb;
                H.lq_fwd[c] = pair_logq_dev(lg, n, na, nb, H.eps);
            }
        }
    }
    const int src = (lane == a) ? b : ((lane == b) ? a : lane);
    const int32_t w = __shfl(v, src, 64);
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    uint64_t bits = (next && lane >= lo && lane <= hi && lane < n) ? (1ull << v) : 0ull;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) bits |= (uint64_t)__shfl_xor((unsigned long long)bits, off, 64);
    if (next && lane < n) {
        H.prop[row + lane] = w;
        H.ppos[row + w] = (uint8_t)lane;
    }
    if (lane == 0) {
        H.t[c] = t1;
        H.wmask[c] = bits;
    }
}

}  // namespace bnos

using namespace bnos;

namespace {

bnos_status validate_cfg(const bnos_chain_cfg *cfg)
{
    if (!cfg) { set_error("NULL cfg"); return BNOS_E_INVALID; }
    if (cfg->chains < 1 || cfg->chains > 65536) { set_error("chains outside [1, 65536]"); return BNOS_E_RANGE; }
    if (cfg->target != 0 && cfg->target != 1) { set_error("target must be 0 or 1"); return BNOS_E_INVALID; }
    if (cfg->iterations < 0 || cfg->first_iteration < 0) { set_error("negative iteration count"); return BNOS_E_RANGE; }
    if (cfg->trace_every < 1) { set_error("trace_every must be >= 1"); return BNOS_E_RANGE; }
    if (cfg->sweep_len < 0) { set_error("sweep_len < 0"); return BNOS_E_RANGE; }
    if (cfg->chain_offset < 0) { set_error("chain_offset < 0"); return BNOS_E_RANGE; }
    for (int r = 0; r < 2; ++r)
        if (cfg->reserved[r] != 0) { set_error("cfg.reserved must be zero"); return BNOS_E_INVALID; }
    if (cfg->proposal != 0 && cfg->proposal != 1) { set_error("proposal must be 0 or 1"); return BNOS_E_INVALID; }
    if (cfg->topk < 0 || cfg->topk > 64) { set_error("topk outside [0, 64]"); return BNOS_E_RANGE; }
    if (cfg->trace_edges < 0 || cfg->trace_edges > 32) { set_error("trace_edges outside [0, 32]"); return BNOS_E_RANGE; }
    if (cfg->trace_edges > 0 && !cfg->edges) { set_error("trace_edges > 0 needs edges"); return BNOS_E_INVALID; }
    if (cfg->proposal == 1) {
        if (!mlp_handle_live(cfg->mlp)) { set_error("learned proposal needs a live network handle"); return BNOS_E_STATE; }
        if (!(cfg->eps >= 0.f && cfg->eps <= 1.f)) { set_error("eps outside [0, 1]"); return BNOS_E_RANGE; }
    }
    return BNOS_OK;
}

}  // namespace

// The sweep of bnos_run_chains_multi; with replay_ms, the device time of the
// iterations (graph replays and the remainder, not the set-up) is returned there.
static bnos_status run_chains_impl(const bnos_table *hs, int32_t T, const bnos_chain_cfg *cfg,
                                   bnos_chain_state *states, void *stream, float *replay_ms)
{
    if (!hs || !states) { set_error("NULL argument"); return BNOS_E_INVALID; }
    if (T < 1 || T > 4096) { set_error("T outside [1, 4096]"); return BNOS_E_RANGE; }
    bnos_status s = validate_cfg(cfg);
    if (s != BNOS_OK) return s;
    std::vector<TableT *> tabs(T);
    for (int k = 0; k < T; ++k) {
        tabs[k] = reinterpret_cast<TableT *>(hs[k]);
        if (!handle_live(tabs[k])) { set_error("invalid table handle"); return BNOS_E_STATE; }
        for (int j = 0; j < k; ++j)
            if (tabs[j] == tabs[k]) { set_error("a table appears twice"); return BNOS_E_INVALID; }
        if (tabs[k]->device != tabs[0]->device) { set_error("tables on different devices"); return BNOS_E_INVALID; }
        if (tabs[k]->n < 2) { set_error("chains need n >= 2 (a swap needs two positions)"); return BNOS_E_RANGE; }
        const bnos_chain_state &st = states[k];
        if (!st.orders || !st.scores || !st.best_graphs || !st.best_scores || !st.accepted) {
            set_error("NULL state array");
            return BNOS_E_INVALID;
        }
        if (st.harvest_feats && (!st.harvest_pairs || !st.harvest_count || st.harvest_cap < 1)) {
            set_error("harvest needs feats, pairs, count and cap >= 1");
            return BNOS_E_INVALID;
        }
        if (cfg->proposal == 1 && tabs[k]->n > 64) { set_error("n > 64"); return BNOS_E_RANGE; }
        if (cfg->topk > 0 && (!st.top_graphs || !st.top_scores || !st.top_count)) {
            set_error("topk > 0 needs top_graphs, top_scores and top_count");
            return BNOS_E_INVALID;
        }
        if (cfg->trace_edges > 0) {
            if (!st.edge_trace) { set_error("trace_edges > 0 needs edge_trace"); return BNOS_E_INVALID; }
            for (int e = 0; e < cfg->trace_edges; ++e) {
                const int ch = cfg->edges[2 * e], pa = cfg->edges[2 * e + 1];
                if (ch < 0 || ch >= tabs[k]->n || pa < 0 || pa >= tabs[k]->n || ch == pa) {
                    set_error("traced edge outside the table's nodes");
                    return BNOS_E_RANGE;
                }
            }
        }
    }
    // scoring steps: the adoption of the starting order (fresh: iteration 0; resume: the
    // saved order, re-scored to rebuild the per-node caches) and one per iteration
    if (cfg->iterations == 0 && cfg->first_iteration > 0) return BNOS_OK;
    const int64_t steps = cfg->iterations + 1;
    const int C = cfg->chains;
    hipStream_t us = reinterpret_cast<hipStream_t>(stream);
    BNOS_HIP(hipSetDevice(tabs[0]->device));
    for (int k = 0; k < T; ++k)
        if ((s = ensure_workspace(tabs[k], C)) != BNOS_OK) return s;

    // per-call workspace: descriptors + per table: per-node caches, proposals,
    // windows, work lists, iteration counters
    size_t bytes = sizeof(TabView) * T + sizeof(ChainView) * T + 3 * sizeof(int64_t) * (T + 1) + 256;
    const size_t edges_off = bytes;
    bytes += 64 * sizeof(int32_t) + 256;                                        // traced edges
    std::vector<size_t> off(T);
    for (int k = 0; k < T; ++k) {
        const size_t n = tabs[k]->n, cn = (size_t)C * n;
        off[k] = bytes;
        bytes += cn * 24 + (size_t)C * 16 + cn * 4 + n * C * 4 + n * 4 + 256;   // caches, windows, lists
        bytes += cn * 8 + cn * 4 + (size_t)C * 8 + (size_t)C * 8 + 256;         // second best, logits, q, pair
        bytes += cn + 256;                                                       // node positions
        bytes += cn * 4 + 256;                                                   // score-bound cuts
        bytes = (bytes + 255) & ~(size_t)255;
    }
    char *ws = nullptr;
    hipError_t e = hipMalloc((void **)&ws, bytes);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc chain workspace: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? BNOS_E_NOMEM : BNOS_E_DEVICE;
    }
    std::vector<TabView> tv(T);
    std::vector<ChainView> cv(T);
    std::vector<int64_t> blk_base(T + 1, 0), chain_base(T + 1, 0), node_base(T + 1, 0);
    int64_t max_groups_c = C;
    for (int k = 0; k < T; ++k) {
        TableT *t = tabs[k];
        const int n = t->n;
        const size_t cn = (size_t)C * n;
        char *p = ws + off[k];
        ChainView &H = cv[k];
        H.n = n;
        H.C = C;
        H.target = cfg->target;
        H.seed = cfg->seed;
        H.chain0 = cfg->chain_offset + (int64_t)k * C;
        H.t_first = cfg->first_iteration;
        H.t_last = cfg->first_iteration + cfg->iterations;
        H.node_l = reinterpret_cast<double *>(p);       p += cn * 8;
        H.node_m = reinterpret_cast<double *>(p);       p += cn * 8;
        H.node_best = reinterpret_cast<uint64_t *>(p);  p += cn * 8;
        H.wmask = reinterpret_cast<uint64_t *>(p);      p += (size_t)C * 8;
        H.t = reinterpret_cast<int64_t *>(p);           p += (size_t)C * 8;
        H.prop = reinterpret_cast<int32_t *>(p);        p += cn * 4;
        H.wl_list = reinterpret_cast<int32_t *>(p);     p += (size_t)n * C * 4;
        H.wl_count = reinterpret_cast<int32_t *>(p);    p += (size_t)n * 4;
        p = ws + ((size_t)(p - ws + 255) & ~(size_t)255);
        H.node_sec = reinterpret_cast<double *>(p);     p += cn * 8;
        H.lq_fwd = reinterpret_cast<double *>(p);       p += (size_t)C * 8;
        H.cur_logit = reinterpret_cast<float *>(p);     p += cn * 4;
        H.pend = reinterpret_cast<int32_t *>(p);       p += (size_t)C * 8;
        H.ppos = reinterpret_cast<uint8_t *>(p);       p += cn;
        p = ws + ((size_t)(p - ws + 255) & ~(size_t)255);
        const bool bound = t->score_bound && t->tile_skip;
        H.cuts = bound ? reinterpret_cast<float *>(p) : nullptr;
        H.nstat = t->d_nstat;
        H.proposal = cfg->proposal;
        H.eps = cfg->eps > 0.f ? (double)cfg->eps : 0.5;
        if (cfg->proposal == 1) H.mlp = mlp_view(cfg->mlp);
        else std::memset(&H.mlp, 0, sizeof(H.mlp));
        const bnos_chain_state &st = states[k];
        H.cur = st.orders;
        H.score = st.scores;
        H.best_score = st.best_scores;
        H.best_graph = st.best_graphs;
        H.accepted = st.accepted;
        H.trace = st.trace;
        H.trace_every = cfg->trace_every;
        H.trace_len = cfg->iterations / cfg->trace_every + 1;
        H.flags = st.accept_flags;
        H.iterations = cfg->iterations;
        H.hv_feat = st.harvest_feats;
        H.hv_pair = st.harvest_pairs;
        H.hv_count = st.harvest_count;
        H.hv_cap = st.harvest_feats ? st.harvest_cap : 0;
        H.n_edges = cfg->trace_edges;
        H.edge_cp = reinterpret_cast<const int32_t *>(ws + edges_off);
        H.edge_trace = st.edge_trace;
        H.topk = cfg->topk;
        H.top_graph = st.top_graphs;
        H.top_score = st.top_scores;
        H.top_count = st.top_count;
        TabView &V = tv[k];
        V.masks = t->d_masks;
        V.scores = t->d_scores;
        V.S_pad = t->S_pad;
        V.chunks = t->chain_chunks_for(C);
        V.chunk_entries = t->chain_chunk_entries_for(C);
        V.sum_chunks = t->S_pad / ((int64_t)t->pad_steps * kEntriesPerStep);
        V.sum_steps = t->pad_steps;
        V.n = n;
        V.B = C;
        V.orders = H.prop;
        V.part = reinterpret_cast<Partial *>(t->d_part);
        V.wl_count = H.wl_count;
        V.wl_list = H.wl_list;
        V.tand = t->tile_skip ? t->d_tand : nullptr;
        V.tsub = t->d_tsub;
        V.anchor = nullptr;            // chain blocks read the stored masks
        V.tmax = bound ? t->d_tmax : nullptr;
        V.cmask = bound ? t->d_cmask : nullptr;
        V.cscore = bound ? t->d_cscore : nullptr;
        V.cuts = H.cuts;               // computed by k_worklist before each scoring launch
        V.K = t->K;
        blk_base[k + 1] = blk_base[k] + (int64_t)n * V.chunks;
        chain_base[k + 1] = chain_base[k] + C;
        node_base[k + 1] = node_base[k] + n;
    }
    TabView *d_tv = reinterpret_cast<TabView *>(ws);
    ChainView *d_cv = reinterpret_cast<ChainView *>(ws + sizeof(TabView) * T);
    int64_t *d_blk = reinterpret_cast<int64_t *>(ws + sizeof(TabView) * T + sizeof(ChainView) * T);
    int64_t *d_chain = d_blk + (T + 1);
    int64_t *d_node = d_chain + (T + 1);

    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    auto cleanup = [&]() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (cs) hipStreamDestroy(cs);
        if (ev0) hipEventDestroy(ev0);
        if (ev1) hipEventDestroy(ev1);
        hipFree(ws);
    };
#define CK(call) if ((e = (call)) != hipSuccess) { set_error(std::string(#call) + ": " + hipGetErrorString(e)); cleanup(); return BNOS_E_DEVICE; }
    if (cfg->trace_edges > 0)
        CK(hipMemcpy(ws + edges_off, cfg->edges, sizeof(int32_t) * 2 * cfg->trace_edges, hipMemcpyHostToDevice));
    CK(hipMemcpy(d_tv, tv.data(), sizeof(TabView) * T, hipMemcpyHostToDevice));
    CK(hipMemcpy(d_cv, cv.data(), sizeof(ChainView) * T, hipMemcpyHostToDevice));
    CK(hipMemcpy(d_blk, blk_base.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice));
    CK(hipMemcpy(d_chain, chain_base.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice));
    CK(hipMemcpy(d_node, node_base.data(), sizeof(int64_t) * (T + 1), hipMemcpyHostToDevice));
    // orders per scoring block: the chain-sweep shape of C's bucket if set (one per launch,
    // from the first table), else the scoring rule for a batch of C orders
    const int tb_bt = tabs[0]->chain_bt[TableT::bucket(C)];
    const int bt = (tb_bt > 0 && tb_bt <= C) ? tb_bt : pick_bt(tabs[0], C);
    const unsigned groups = (unsigned)((max_groups_c + bt - 1) / bt);
    const unsigned total_chains = (unsigned)chain_base[T];
    bool any_bound = false;
    for (int k = 0; k < T; ++k) any_bound = any_bound || cv[k].cuts != nullptr;
    // blocks of k_worklist that compute the score-bound cuts after the list blocks
    const int64_t cut_blocks = any_bound ? (node_base[T] * (int64_t)C + kListThreads / 64 - 1) / (kListThreads / 64) : 0;
    if ((node_base[T] + cut_blocks) * kListThreads > (int64_t)UINT32_MAX) {
        set_error("too many (chain, node) pairs for one launch: lower the chains or the tables per call");
        cleanup();
        return BNOS_E_RANGE;
    }
    hipLaunchKernelGGL(k_chain_init, dim3(total_chains), dim3(64), 0, us, d_cv, d_chain, T);
    CK(hipGetLastError());
    auto one_step = [&](hipStream_t q) -> hipError_t {
        hipLaunchKernelGGL(k_worklist, dim3((unsigned)(node_base[T] + cut_blocks)), dim3(kListThreads), 0, q, d_tv, d_cv,
                           d_node, T, C);
        dim3 grid((unsigned)((blk_base[T] + kXcds - 1) / kXcds * kXcds), groups);   // padded for xcd_block
        if (bt == 8) hipLaunchKernelGGL(k_score_multi<8>, grid, dim3(kScoreThreads), 0, q, d_tv, d_blk, T);
        else if (bt == 4) hipLaunchKernelGGL(k_score_multi<4>, grid, dim3(kScoreThreads), 0, q, d_tv, d_blk, T);
        else if (bt == 2) hipLaunchKernelGGL(k_score_multi<2>, grid, dim3(kScoreThreads), 0, q, d_tv, d_blk, T);
        else hipLaunchKernelGGL(k_score_multi<1>, grid, dim3(kScoreThreads), 0, q, d_tv, d_blk, T);
        hipLaunchKernelGGL(k_chain_step, dim3(total_chains), dim3(kStepWaves * 64), 0, q, d_tv, d_cv, d_chain, T);
        return hipGetLastError();
    };
    const int64_t sweep = cfg->sweep_len > 0 ? cfg->sweep_len : 32;
    const int64_t graphs = steps / sweep;
    const int64_t rest = steps - graphs * sweep;
    if (graphs > 0) {
        CK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        CK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int64_t q = 0; q < sweep; ++q) {
            if ((e = one_step(cs)) != hipSuccess) {
                hipGraph_t g2 = nullptr;
                hipStreamEndCapture(cs, &g2);
                if (g2) hipGraphDestroy(g2);
                set_error(std::string("kernel launch during capture: ") + hipGetErrorString(e));
                cleanup();
                return BNOS_E_DEVICE;
            }
        }
        CK(hipStreamEndCapture(cs, &graph));
        CK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
    }
    if (replay_ms) {
        CK(hipEventCreate(&ev0));
        CK(hipEventCreate(&ev1));
        CK(hipEventRecord(ev0, us));
    }
    for (int64_t g = 0; g < graphs; ++g) CK(hipGraphLaunch(exec, us));
    for (int64_t q = 0; q < rest; ++q) CK(one_step(us));
    if (replay_ms) CK(hipEventRecord(ev1, us));
    CK(hipStreamSynchronize(us));
    if (replay_ms) CK(hipEventElapsedTime(replay_ms, ev0, ev1));
#undef CK
    cleanup();
    return BNOS_OK;
}

extern "C" bnos_status bnos_run_chains_multi(const bnos_table *hs, int32_t T, const bnos_chain_cfg *cfg,
                                             bnos_chain_state *states, void *stream)
{
    return run_chains_impl(hs, T, cfg, states, stream, nullptr);
}

extern "C" bnos_status bnos_run_chains(bnos_table h, const bnos_chain_cfg *cfg, bnos_chain_state *st,
                                       void *stream)
{
    return run_chains_impl(&h, 1, cfg, st, stream, nullptr);
}

static bnos_status check_chain_shape(const TableT *t, int32_t chunk_steps, int32_t orders_per_block)
{
    if (chunk_steps != 0 && (chunk_steps < 1 || chunk_steps > t->pad_steps || (chunk_steps & (chunk_steps - 1)) != 0)) {
        set_error("chunk_steps must be 0 or a power of two dividing the row padding");
        return BNOS_E_RANGE;
    }
    if (orders_per_block != 0 && orders_per_block != 1 && orders_per_block != 2 && orders_per_block != 4 &&
        orders_per_block != 8) {
        set_error("orders_per_block must be 0, 1, 2, 4 or 8");
        return BNOS_E_RANGE;
    }
    return BNOS_OK;
}

extern "C" bnos_status bnos_chains_set_launch(bnos_table h, int32_t chains, int32_t chunk_steps,
                                              int32_t orders_per_block)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (chains < 1 || chains > 65536) { set_error("chains outside [1, 65536]"); return BNOS_E_RANGE; }
    bnos_status s = check_chain_shape(t, chunk_steps, orders_per_block);
    if (s != BNOS_OK) return s;
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipDeviceSynchronize());        // sweeps in flight keep their shapes and workspace
    const int bk = TableT::bucket(chains);
    t->chain_cs[bk] = chunk_steps;
    t->chain_bt[bk] = orders_per_block;
    return ensure_workspace(t, chains);
}

extern "C" bnos_status bnos_chains_autotune(bnos_table h, const bnos_chain_cfg *cfg, const bnos_chain_state *state,
                                            int32_t reps, void *stream, int32_t *chunk_steps,
                                            int32_t *orders_per_block, double *ms_per_iteration)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    bnos_status s = validate_cfg(cfg);
    if (s != BNOS_OK) return s;
    if (cfg->iterations < 1 || cfg->iterations > (1 << 20)) { set_error("iterations outside [1, 2^20]"); return BNOS_E_RANGE; }
    if (reps < 1 || reps > 100) { set_error("reps outside [1, 100]"); return BNOS_E_RANGE; }
    if (t->n < 2) { set_error("chains need n >= 2 (a swap needs two positions)"); return BNOS_E_RANGE; }
    const bool resume = cfg->first_iteration > 0;
    if (resume && (!state || !state->orders || !state->scores || !state->best_graphs || !state->best_scores ||
                   !state->accepted)) {
        set_error("a resumed tuning run needs the state to start from");
        return BNOS_E_INVALID;
    }
    const int C = cfg->chains, n = t->n;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    BNOS_HIP(hipSetDevice(t->device));
    BNOS_HIP(hipDeviceSynchronize());
    // scratch state: every candidate starts from the same chains and the caller's state is untouched
    const size_t cn = (size_t)C * n;
    char *scr = nullptr;
    const size_t bytes = cn * 4 + cn * 8 + (size_t)C * 8 * 3 + 1024;
    hipError_t e = hipMalloc((void **)&scr, bytes);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc tuning state: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? BNOS_E_NOMEM : BNOS_E_DEVICE;
    }
    bnos_chain_state sc;
    std::memset(&sc, 0, sizeof(sc));
    char *p = scr;
    sc.best_graphs = reinterpret_cast<uint64_t *>(p);  p += cn * 8;
    sc.scores = reinterpret_cast<double *>(p);          p += (size_t)C * 8;
    sc.best_scores = reinterpret_cast<double *>(p);     p += (size_t)C * 8;
    sc.accepted = reinterpret_cast<int64_t *>(p);       p += (size_t)C * 8;
    sc.orders = reinterpret_cast<int32_t *>(p);
    bnos_chain_cfg c2 = *cfg;
    c2.topk = 0;
    c2.trace_edges = 0;
    c2.edges = nullptr;
    const int bk = TableT::bucket(C);
    const int old_cs = t->chain_cs[bk], old_bt = t->chain_bt[bk];
    double best_ms = 1e300;
    int best_cs = 0, best_bt = 0;
    for (int cs = 1; cs <= t->pad_steps && s == BNOS_OK; cs <<= 1) {
        for (int bt = 1; bt <= 8 && bt <= C && s == BNOS_OK; bt <<= 1) {
            t->chain_cs[bk] = cs;
            t->chain_bt[bk] = bt;
            if ((s = ensure_workspace(t, C)) != BNOS_OK) break;
            double tot = 0.0;
            for (int r = 0; r <= reps && s == BNOS_OK; ++r) {
                if (resume) {
                    hipMemcpyAsync(sc.orders, state->orders, cn * 4, hipMemcpyDeviceToDevice, st);
                    hipMemcpyAsync(sc.scores, state->scores, (size_t)C * 8, hipMemcpyDeviceToDevice, st);
                    hipMemcpyAsync(sc.best_graphs, state->best_graphs, cn * 8, hipMemcpyDeviceToDevice, st);
                    hipMemcpyAsync(sc.best_scores, state->best_scores, (size_t)C * 8, hipMemcpyDeviceToDevice, st);
                    if ((e = hipMemcpyAsync(sc.accepted, state->accepted, (size_t)C * 8, hipMemcpyDeviceToDevice,
                                            st)) != hipSuccess) {
                        set_error(std::string("tuning state copy: ") + hipGetErrorString(e));
                        s = BNOS_E_DEVICE;
                        break;
                    }
                }
                float ms = 0.f;
                bnos_table hh = h;
                s = run_chains_impl(&hh, 1, &c2, &sc, stream, &ms);
                if (r > 0) tot += ms;                 // the first run is the warm-up
            }
            const double per = tot / ((double)reps * (double)cfg->iterations);
            if (s == BNOS_OK && per < best_ms) {
                best_ms = per;
                best_cs = cs;
                best_bt = bt;
            }
        }
    }
    hipFree(scr);
    if (s != BNOS_OK) {
        t->chain_cs[bk] = old_cs;
        t->chain_bt[bk] = old_bt;
        return s;
    }
    t->chain_cs[bk] = best_cs;
    t->chain_bt[bk] = best_bt;
    if ((s = ensure_workspace(t, C)) != BNOS_OK) return s;
    if (chunk_steps) *chunk_steps = best_cs;
    if (orders_per_block) *orders_per_block = best_bt;
    if (ms_per_iteration) *ms_per_iteration = best_ms;
    return BNOS_OK;
}
