// Metropolis-Hastings over node orders on the device (Sec. III.C): batched
// chains, one streaming pass per iteration for all chains' proposals, the
// merge + accept/reject + best-graph record + next proposal fused into one
// kernel, and sweeps of iterations captured as HIP graphs.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <string>

#include "bnos_internal.h"
#include "score_device.h"

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

struct ChainArgs {
    int n, C, target;
    uint64_t seed;
    int64_t chain0;
    int64_t t_first, t_last;   // iterations already done before this call; last iteration to run
    int32_t *cur;              // [C][n] current orders (state)
    int32_t *prop;             // [C][n] orders being scored
    double *score;             // [C] target score of the current order (state)
    double *best_score;        // [C] (state)
    uint64_t *best_graph;      // [C][n] (state)
    uint64_t *prop_best;       // [C][n] greedy graph of the proposal
    int64_t *accepted;         // [C] (state)
    int64_t *t;                // [C] iteration whose proposal is being scored
    double *trace;             // [C][trace_len] or null
    int trace_every;
    int64_t trace_len;
    uint8_t *flags;            // [C][iterations] or null
    int64_t iterations;
};

// Block per chain: the initial order (fresh start) or the first proposal after
// the saved state (resume).
__global__ __launch_bounds__(64) void k_chain_init(ChainArgs H)
{
    const int c = blockIdx.x;
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
            for (int p = 0; p < n; ++p) H.prop[(int64_t)c * n + p] = ord[p];
            H.t[c] = 0;
            H.accepted[c] = 0;
        }
    } else {
        const int64_t t1 = H.t_first + 1;
        int a = 0, b = 0;
        rng_pair(H.seed, chain, n, (uint64_t)t1, a, b);
        if (lane < n) {
            const int src = (lane == a) ? b : ((lane == b) ? a : lane);
            H.prop[(int64_t)c * n + lane] = H.cur[(int64_t)c * n + src];
        }
        if (lane == 0) {
            H.t[c] = t1;
            if (H.trace) H.trace[(int64_t)c * H.trace_len] = H.score[c];
        }
    }
}

// Block per chain: merge the proposal's chunk partials, take the MH decision,
// update the best-graph record, and write the next proposal.
__global__ __launch_bounds__(kMergeWaves * 64) void k_chain_step(ScoreArgs A, ChainArgs H)
{
    __shared__ double s_l[64], s_b[64];
    __shared__ int s_acc, s_imp, s_a, s_b2, s_next;
    const int c = blockIdx.x;
    const int n = H.n;
    bool valid;
    double l, m;
    merge_block(A, c, s_l, s_b, valid, l, m);
    if (threadIdx.x == 0) {
        const uint64_t chain = (uint64_t)(H.chain0 + c);
        const int64_t t = H.t[c];
        const double nv = H.target ? m : l;
        int acc = 0, imp = 0;
        if (t == 0) {
            acc = 1;
            imp = 1;
            H.score[c] = nv;
            H.best_score[c] = m;
        } else {
            const double u = rng_unit_open(rng_draw(H.seed, chain, 3, (uint64_t)t));
            acc = log(u) < nv - H.score[c];
            if (acc) {
                H.score[c] = nv;
                H.accepted[c] += 1;
                if (m > H.best_score[c]) {
                    H.best_score[c] = m;
                    imp = 1;
                }
            }
            if (H.flags) H.flags[(int64_t)c * H.iterations + (t - H.t_first - 1)] = (uint8_t)acc;
        }
        const int64_t k = t - H.t_first;
        if (H.trace && k % H.trace_every == 0) H.trace[(int64_t)c * H.trace_len + k / H.trace_every] = H.score[c];
        const int64_t t1 = t + 1;
        int a = 0, b = 0;
        const int next = t1 <= H.t_last;
        if (next) rng_pair(H.seed, chain, n, (uint64_t)t1, a, b);
        H.t[c] = t1;
        s_acc = acc;
        s_imp = imp;
        s_a = a;
        s_b2 = b;
        s_next = next;
    }
    __syncthreads();
    const int lane = threadIdx.x;
    if (lane < 64) {
        const int64_t row = (int64_t)c * n;
        int32_t v = 0;
        if (lane < n) {
            v = s_acc ? H.prop[row + lane] : H.cur[row + lane];
            H.cur[row + lane] = v;
            if (s_imp) H.best_graph[row + lane] = H.prop_best[row + lane];
        }
        const int a = s_a, b = s_b2;
        const int src = (lane == a) ? b : ((lane == b) ? a : lane);
        const int32_t w = __shfl(v, src, 64);
        if (s_next && lane < n) H.prop[row + lane] = w;
    }
}

}  // namespace bnos

using namespace bnos;

extern "C" bnos_status bnos_run_chains(bnos_table h, const bnos_chain_cfg *cfg, bnos_chain_state *st,
                                       void *stream)
{
    TableT *t = reinterpret_cast<TableT *>(h);
    if (!handle_live(t)) { set_error("invalid table handle"); return BNOS_E_STATE; }
    if (!cfg || !st) { set_error("NULL argument"); return BNOS_E_INVALID; }
    const int n = t->n;
    const int C = cfg->chains;
    if (C < 1 || C > 65536) { set_error("chains outside [1, 65536]"); return BNOS_E_RANGE; }
    if (cfg->target != 0 && cfg->target != 1) { set_error("target must be 0 or 1"); return BNOS_E_INVALID; }
    if (cfg->iterations < 0 || cfg->first_iteration < 0) { set_error("negative iteration count"); return BNOS_E_RANGE; }
    if (cfg->trace_every < 1) { set_error("trace_every must be >= 1"); return BNOS_E_RANGE; }
    if (cfg->sweep_len < 0) { set_error("sweep_len < 0"); return BNOS_E_RANGE; }
    if (cfg->chain_offset < 0) { set_error("chain_offset < 0"); return BNOS_E_RANGE; }
    for (int r = 0; r < 6; ++r)
        if (cfg->reserved[r] != 0) { set_error("cfg.reserved must be zero"); return BNOS_E_INVALID; }
    if (!st->orders || !st->scores || !st->best_graphs || !st->best_scores || !st->accepted) {
        set_error("NULL state array");
        return BNOS_E_INVALID;
    }
    if (n < 2) { set_error("chains need n >= 2 (a swap needs two positions)"); return BNOS_E_RANGE; }
    const bool fresh = cfg->first_iteration == 0;
    // scoring steps: fresh runs t = 0..iterations, a resume runs t = first+1..first+iterations
    const int64_t steps = fresh ? cfg->iterations + 1 : cfg->iterations;
    if (steps == 0) return BNOS_OK;
    hipStream_t us = reinterpret_cast<hipStream_t>(stream);
    BNOS_HIP(hipSetDevice(t->device));
    bnos_status s = ensure_workspace(t, C);
    if (s != BNOS_OK) return s;

    // per-call workspace: proposals, their greedy graphs and scores, iteration counters
    char *ws = nullptr;
    const size_t b_prop = sizeof(int32_t) * (size_t)C * n;
    const size_t b_pbest = sizeof(uint64_t) * (size_t)C * n;
    const size_t b_pl = sizeof(double) * (size_t)C;
    const size_t b_t = sizeof(int64_t) * (size_t)C;
    hipError_t e = hipMalloc((void **)&ws, b_prop + b_pbest + 2 * b_pl + b_t + 256);
    if (e != hipSuccess) {
        set_error(std::string("hipMalloc chain workspace: ") + hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? BNOS_E_NOMEM : BNOS_E_DEVICE;
    }
    uint64_t *prop_best = reinterpret_cast<uint64_t *>(ws);
    double *prop_l = reinterpret_cast<double *>(ws + b_pbest);
    double *prop_m = prop_l + C;
    int64_t *tcount = reinterpret_cast<int64_t *>(ws + b_pbest + 2 * b_pl);
    int32_t *prop = reinterpret_cast<int32_t *>(ws + b_pbest + 2 * b_pl + b_t);

    ChainArgs H;
    H.n = n;
    H.C = C;
    H.target = cfg->target;
    H.seed = cfg->seed;
    H.chain0 = cfg->chain_offset;
    H.t_first = cfg->first_iteration;
    H.t_last = cfg->first_iteration + cfg->iterations;
    H.cur = st->orders;
    H.prop = prop;
    H.score = st->scores;
    H.best_score = st->best_scores;
    H.best_graph = st->best_graphs;
    H.prop_best = prop_best;
    H.accepted = st->accepted;
    H.t = tcount;
    H.trace = st->trace;
    H.trace_every = cfg->trace_every;
    H.trace_len = cfg->iterations / cfg->trace_every + 1;
    H.flags = st->accept_flags;
    H.iterations = cfg->iterations;
    ScoreArgs A = score_args(t, prop, C, prop_l, prop_m, prop_best, nullptr, nullptr);
    const int bt = pick_bt(t, C);

    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    auto cleanup = [&]() {
        if (exec) hipGraphExecDestroy(exec);
        if (graph) hipGraphDestroy(graph);
        if (cs) hipStreamDestroy(cs);
        hipFree(ws);
    };
#define CK(call) if ((e = (call)) != hipSuccess) { set_error(std::string(#call) + ": " + hipGetErrorString(e)); cleanup(); return BNOS_E_DEVICE; }
    hipLaunchKernelGGL(k_chain_init, dim3(C), dim3(64), 0, us, H);
    CK(hipGetLastError());
    auto one_step = [&](hipStream_t q) -> bnos_status {
        bnos_status r = launch_stream(t, A, q, bt);
        if (r != BNOS_OK) return r;
        hipLaunchKernelGGL(k_chain_step, dim3(C), dim3(kMergeWaves * 64), 0, q, A, H);
        BNOS_HIP(hipGetLastError());
        return BNOS_OK;
    };
    const int64_t sweep = cfg->sweep_len > 0 ? cfg->sweep_len : 32;
    const int64_t graphs = steps / sweep;
    const int64_t rest = steps - graphs * sweep;
    if (graphs > 0) {
        // Capture one sweep on a private stream (timing events are not captured).
        const bool timing = t->timing;
        t->timing = false;
        CK(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        CK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        for (int64_t k = 0; k < sweep; ++k) {
            if ((s = one_step(cs)) != BNOS_OK) {
                hipGraph_t g2 = nullptr;
                hipStreamEndCapture(cs, &g2);
                if (g2) hipGraphDestroy(g2);
                t->timing = timing;
                cleanup();
                return s;
            }
        }
        CK(hipStreamEndCapture(cs, &graph));
        t->timing = timing;
        CK(hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0));
        for (int64_t g = 0; g < graphs; ++g) CK(hipGraphLaunch(exec, us));
    }
    for (int64_t k = 0; k < rest; ++k) {
        if ((s = one_step(us)) != BNOS_OK) { cleanup(); return s; }
    }
    CK(hipStreamSynchronize(us));
#undef CK
    cleanup();
    return BNOS_OK;
}
