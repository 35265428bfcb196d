// Device code of order scoring shared by the scoring and the chain kernels:
// per-entry fold (online log-sum-exp + top-2 argmax), fixed-order merges,
// predecessor masks, the streaming kernel k_score<BT> and the per-order merge.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "bnos_internal.h"

namespace bnos {

typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ device helpers

// Wavefront reductions on the data-parallel-primitive (DPP) lane network:
// quad permutes (lane ^ 1, lane ^ 2), row shifts by 4 and 8 and the two row
// broadcasts (lane 15 of a row to the next row, lane 31 to rows 2 and 3) leave
// the reduction of all 64 lanes in lane 63, one VALU instruction per level; a
// lane whose source does not exist reads the identity.  The association is
// fixed, so the result does not depend on scheduling; readlane makes it uniform.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v, uint32_t identity)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)identity, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v, float identity)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, identity),
                                                                 __builtin_bit_cast(int, v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float lane63_f32(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}
__device__ __forceinline__ float wave_max_f32(float v)
{
    v = fmaxf(v, dpp_f32<0xb1>(v, -INFINITY));
    v = fmaxf(v, dpp_f32<0x4e>(v, -INFINITY));
    v = fmaxf(v, dpp_f32<0x114>(v, -INFINITY));
    v = fmaxf(v, dpp_f32<0x118>(v, -INFINITY));
    v = fmaxf(v, dpp_f32<0x142>(v, -INFINITY));
    v = fmaxf(v, dpp_f32<0x143>(v, -INFINITY));
    return lane63_f32(v);
}
__device__ __forceinline__ float wave_sum_f32(float v)
{
    v = v + dpp_f32<0xb1>(v, 0.f);
    v = v + dpp_f32<0x4e>(v, 0.f);
    v = v + dpp_f32<0x114>(v, 0.f);
    v = v + dpp_f32<0x118>(v, 0.f);
    v = v + dpp_f32<0x142>(v, 0.f);
    v = v + dpp_f32<0x143>(v, 0.f);
    return lane63_f32(v);
}
__device__ __forceinline__ uint32_t wave_or_u32(uint32_t v)
{
    v |= dpp_u32<0xb1>(v, 0u);
    v |= dpp_u32<0x4e>(v, 0u);
    v |= dpp_u32<0x114>(v, 0u);
    v |= dpp_u32<0x118>(v, 0u);
    v |= dpp_u32<0x142>(v, 0u);
    v |= dpp_u32<0x143>(v, 0u);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}
__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v)
{
    return ((uint64_t)wave_or_u32((uint32_t)(v >> 32)) << 32) | wave_or_u32((uint32_t)v);
}


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

// Fold a lane's group of 4 consecutive row entries into its state, for a lane
// that sees its entries in ascending mask order (the streaming pass: a row
// lists the masks in ascending order and a lane visits its groups in row
// order).  x[e] is the entry's score if consistent, else -inf; mk[e] its mask.
// The log-sum-exp max is the top-1 score, so one comparison serves both: a
// group that beats the lane's best rescales the sum and takes the new argmax
// (the first entry holding the group's max, i.e. the smallest mask among
// equal scores -- earlier groups hold smaller masks, so an equal score never
// replaces the held best); any other group adds its exp terms and raises the
// second best.  Each term is 2^fl(x log2e - t), t = fl(best log2e): one fma and
// one v_exp_f32 per entry.  Against the exact 2^((x - best) log2e) every term
// carries the same factor 2^(best log2e - t), t's rounding residual, which
// acc_fold_finish divides out; a change of best rescales the sum by 2^(t_old -
// t_new), exact, so the sum always holds that one common factor.  A group with
// no consistent entry changes nothing (it adds exact zeros).
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kScoreFloor = -1.0e38f;   // below every score; keeps best * log2e finite

__device__ __forceinline__ float fold_shift(float best) { return fmaxf(best, kScoreFloor) * kLog2e; }

// t: the caller keeps t == fold_shift(a.best) (initially fold_shift(-inf)).
__device__ __forceinline__ void acc_fold4(Acc &a, float &t, const float (&x)[4], const uint64_t (&mk)[4])
{
#pragma clang fp contract(off)     // t_old - t_new must subtract the two rounded shifts
    const float m01 = fmaxf(x[0], x[1]), n01 = fminf(x[0], x[1]);
    const float m23 = fmaxf(x[2], x[3]), n23 = fminf(x[2], x[3]);
    const float b = fmaxf(m01, m23);
    a.sec = fmaxf(a.sec, b);
    if (b > a.best) {
        // o: the largest of the other three entries (b again if b occurs twice);
        // the argmax: the first entry holding b
        const float o = fmaxf(fminf(m01, m23), fmaxf(n01, n23));
        uint64_t k0 = mk[0], k1 = mk[1], k2 = mk[2], k3 = mk[3];
        asm volatile("" : "+v"(k0), "+v"(k1), "+v"(k2), "+v"(k3));   // selects in registers, not an indexed copy
        uint64_t bmk = k3;
        bmk = x[2] == b ? k2 : bmk;
        bmk = x[1] == b ? k1 : bmk;
        bmk = x[0] == b ? k0 : bmk;
        const float tn = b * kLog2e;
        a.s *= __builtin_amdgcn_exp2f(t - tn);               // 0 when nothing was held
        t = tn;
        a.sec = fmaxf(a.best, o);
        a.best = b;
        a.bm = bmk;
    }
    const float e0 = __builtin_amdgcn_exp2f(fmaf(x[0], kLog2e, -t)), e1 = __builtin_amdgcn_exp2f(fmaf(x[1], kLog2e, -t));
    const float e2 = __builtin_amdgcn_exp2f(fmaf(x[2], kLog2e, -t)), e3 = __builtin_amdgcn_exp2f(fmaf(x[3], kLog2e, -t));
    a.s += (e0 + e1) + (e2 + e3);
}

// The same fold with both updates formed and one selected, no branch: for one
// order per block with computed masks, where some lane of a wavefront nearly
// always takes the first (results bitwise those of acc_fold4; it needs more
// registers, which the blocks that read stored masks cannot spare).
__device__ __forceinline__ void acc_fold4_sel(Acc &a, float &t, const float (&x)[4], const uint64_t (&mk)[4])
{
#pragma clang fp contract(off)     // t_old - t_new must subtract the two rounded shifts
    uint64_t k0 = mk[0], k1 = mk[1], k2 = mk[2], k3 = mk[3];
    asm volatile("" : "+v"(k0), "+v"(k1), "+v"(k2), "+v"(k3));   // keep the masks in registers
    const float m01 = fmaxf(x[0], x[1]), n01 = fminf(x[0], x[1]);
    const float m23 = fmaxf(x[2], x[3]), n23 = fminf(x[2], x[3]);
    const float b = fmaxf(m01, m23);
    const float o = fmaxf(fminf(m01, m23), fmaxf(n01, n23));
    uint64_t bmk = k3;
    bmk = x[2] == b ? k2 : bmk;
    bmk = x[1] == b ? k1 : bmk;
    bmk = x[0] == b ? k0 : bmk;
    const bool nb = b > a.best;
    const float tn = b * kLog2e;
    const float r = __builtin_amdgcn_exp2f(t - tn);
    a.s = nb ? a.s * r : a.s;
    t = nb ? tn : t;
    a.sec = nb ? fmaxf(a.best, o) : fmaxf(a.sec, b);
    a.bm = nb ? bmk : a.bm;
    a.best = nb ? b : a.best;
    const float e0 = __builtin_amdgcn_exp2f(fmaf(x[0], kLog2e, -t)), e1 = __builtin_amdgcn_exp2f(fmaf(x[1], kLog2e, -t));
    const float e2 = __builtin_amdgcn_exp2f(fmaf(x[2], kLog2e, -t)), e3 = __builtin_amdgcn_exp2f(fmaf(x[3], kLog2e, -t));
    a.s += (e0 + e1) + (e2 + e3);
}

// After the last acc_fold4: divide out 2^(best log2e - t) (the residual of t =
// fl(best log2e), exact by fma) and make the state an ordinary (m, s) pair.
__device__ __forceinline__ void acc_fold_finish(Acc &a)
{
#pragma clang fp contract(off)
    if (a.best > -INFINITY) {
        const float t = a.best * kLog2e;
        a.s *= __builtin_amdgcn_exp2f(-fmaf(a.best, kLog2e, -t));
    }
    a.m = a.best;
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

// Select one of two states field by field (no dynamic struct copies).
__device__ __forceinline__ Acc acc_sel(bool c, const Acc &x, const Acc &y)
{
    Acc r;
    r.m = c ? x.m : y.m;
    r.s = c ? x.s : y.s;
    r.best = c ? x.best : y.best;
    r.sec = c ? x.sec : y.sec;
    r.bm = c ? x.bm : y.bm;
    return r;
}

// Reduction of one state per lane whose log-sum-exp max is its top-1 score
// (m == best, as the streaming fold leaves it) over the 64 lanes: the max;
// each lane's sum rescaled to it and summed; the argmax as the smallest mask
// among the lanes holding the max (read from the one lane holding it, else a
// butterfly minimum); the second best as that max when two lanes hold it,
// else the max over the other lanes' best and the holder's second.  Fixed
// trees, so the result does not depend on scheduling; every lane returns it.
__device__ __forceinline__ Acc acc_wave_reduce_one(const Acc &a)
{
    const float M = wave_max_f32(a.best);
    const float s = wave_sum_f32((a.best == -INFINITY) ? 0.f : a.s * __expf(a.best - M));
    const bool top = a.best == M;
    const uint64_t tops = __ballot(top);
    Acc r;
    r.m = M;
    r.s = s;
    r.best = M;
    if (__popcll(tops) == 1) {                               // uniform: one lane holds the max
        const int w = __builtin_ctzll(tops);
        r.bm = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(a.bm >> 32), w) << 32) |
               (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)a.bm, w);
        r.sec = wave_max_f32(top ? a.sec : a.best);
    } else {                                                 // a tie: the smallest mask among the holders
        uint64_t bm = top ? a.bm : ~0ull;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t o = (uint64_t)__shfl_xor((unsigned long long)bm, off, 64);
            bm = o < bm ? o : bm;
        }
        r.bm = bm;
        r.sec = M;
    }
    return r;
}

// Reduction of BT per-lane states over the 64 lanes of a wavefront, as a
// reduce-scatter: while more than one state is left, lanes split by the next
// high lane bit (32, 16, ...) keep one half of the states, receive the
// partner's copy of that half and merge; then a plain butterfly over the
// remaining low lane bits.  Every merge takes the lower lane's state as the
// left operand, so the result does not depend on scheduling.  Returns the
// lane's state; the full reduction of state j is held by the lanes whose top
// log2(BT) bits equal j (e.g. lane j * 64 / BT).  Costs log2(BT) + 6 - log2(BT)
// levels with BT - 1 + (6 - log2 BT) merges per lane, against 6 * BT for BT
// separate butterflies.
template <int BT>
__device__ __forceinline__ Acc acc_wave_reduce_scatter(Acc (&a)[BT], int lane)
{
    constexpr int kLevels = BT >= 8 ? 3 : (BT >= 4 ? 2 : (BT >= 2 ? 1 : 0));
#pragma unroll
    for (int lvl = 0; lvl < kLevels; ++lvl) {
        const int off = 32 >> lvl;
        const int h = (BT >> lvl) / 2;
        const bool up = (lane & off) != 0;
#pragma unroll
        for (int i = 0; i < BT / 2; ++i) {
            if (i >= h) break;
            const Acc keep = acc_sel(up, a[i + h], a[i]);
            const Acc send = acc_sel(up, a[i], a[i + h]);
            const Acc recv = acc_shfl_xor(send, off);
            Acc lo = acc_sel(up, recv, keep);
            const Acc hi = acc_sel(up, keep, recv);
            acc_merge(lo, hi);
            a[i] = lo;
        }
    }
    Acc r = a[0];
#pragma unroll
    for (int off = 1; off < (64 >> kLevels); off <<= 1) {
        const Acc o = acc_shfl_xor(r, off);
        const bool up = (lane & off) != 0;
        Acc lo = acc_sel(up, o, r);
        const Acc hi = acc_sel(up, r, o);
        acc_merge(lo, hi);
        r = lo;
    }
    return r;
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
    const uint64_t before = wave_or_u64((lane < pos) ? bit : 0ull);
    const uint64_t all = wave_or_u64(bit);
    uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    valid = (all == full) && (__ballot(lane < n && !inr) == 0ull);
    return valid ? before : 0ull;
}

// Whether the order is a permutation of 0..n-1, from lane p's entry v (position p),
// by the same test as wave_pred.
__device__ __forceinline__ bool order_valid(int v, int n, int lane)
{
    const bool inr = (v >= 0 && v < n);
    uint64_t all = inr ? (1ull << v) : 0ull;
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) all |= (uint64_t)__shfl_xor((unsigned long long)all, off, 64);
    const uint64_t full = (n == 64) ? ~0ull : ((1ull << n) - 1ull);
    return (all == full) && (__ballot(lane < n && !inr) == 0ull);
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
    int64_t sum_chunks;      // the summaries' layout: chunks of sum_steps steps per row (summary_pos)
    int sum_steps;
    const int32_t *orders;
    int B, n;
    Partial *part;          // [B][chunks][n]
    double *lse, *maxs;
    uint64_t *best;
    double *node_lse;
    float *node_second;
    // Optional work list (chains): node i scores only the wl_count[i] orders listed
    // in wl_list[i * B ...]; a block's slot j takes the (group*BT + j)-th listed order.
    const int32_t *wl_count;   // [n] or null (then slot j of group g is order g*BT + j)
    const int32_t *wl_list;    // [n][B]
    const uint64_t *tand;      // tile summaries, or null
    const uint64_t *tsub;      // sub-tile summaries (with tand)
    const uint64_t *anchor;    // first mask of every 4 entries in slot space, or null
    const float *tmax;         // largest score of each tile (with tand: the score bound), or null
    const uint64_t *cmask;     // [n][kBoundSlots] score-bound candidates of each row (with tmax)
    const float *cscore;
    const float *cuts;         // [B][n] each order's cut per node, computed before the launch, or null
    float *cut_ws;             // [B][n] workspace for those cuts (several-order launches)
    int K;
};

// What one streaming block needs to know about its table and its orders.
struct TabView {
    const uint64_t *masks;
    const float *scores;
    int64_t S_pad;
    int chunks, chunk_entries, n;
    int64_t sum_chunks;         // the summaries' layout: chunks of sum_steps steps per row (summary_pos)
    int sum_steps;
    int B;                      // orders (chains) of this table; row stride of wl_list
    const int32_t *orders;      // [B][n]
    Partial *part;              // [B][chunks][n]
    const int32_t *wl_count;    // [n] or null
    const int32_t *wl_list;     // [n][B]
    const uint64_t *tand;       // [n * S_pad / 256] AND of each 256-entry tile's masks, or null (no skipping)
    const uint64_t *tsub;       // [n * S_pad / 64] the same per 64-entry sub-tile (with tand)
    const uint64_t *anchor;     // [n * S_pad / 4] slot-space first mask of each 4-entry group (computed masks)
    const float *tmax;          // [n * S_pad / 256] largest score of each tile, or null (no score bound)
    const uint64_t *cmask;      // [n][kBoundSlots] score-bound candidates of each row (with tmax)
    const float *cscore;
    const float *cuts;          // [orders][n] each order's (chain's) cut per node, computed by an
                                // earlier launch, or null (the block computes it)
    int K;
};

// A row lists every mask over the node's n - 1 slots (slot s is node s below
// the node, node s + 1 above it) with at most K members, in ascending order.
// The mask after m is m + 1 if that has at most K members, else m plus its
// lowest member (adding it carries the run of members above it into the next
// free slot, and no number in between has few enough members).  Past the last
// mask the result holds a slot >= n - 1, which no predecessor set contains;
// a result not above m (the end of the 64 bits, or K = 0) saturates to ~0.
// (For a mask with at most K members, m + 1 has at most K members exactly when
// m has fewer than K or holds slot 0, and in the second case m + lowest member
// = m + 1; so the step adds 1 or m's lowest member.)
__device__ __forceinline__ uint64_t next_mask(uint64_t m, int K)
{
    const uint64_t r = m + ((__popcll(m) < K) ? 1ull : (m & (0ull - m)));
    return r <= m ? ~0ull : r;
}

// The same without the saturation, for K >= 2 with n <= 63 and for K = 1 with
// n <= 61: starting from a mask of the row or from 2^(n-1) (slot n - 1, which no
// row has: padding and unused lanes), three steps stay below 2^64 (with K = 1
// each step past the row doubles the mask) and every mask past the row keeps a
// slot >= n - 1.
__device__ __forceinline__ uint64_t next_mask_nosat(uint64_t m, int K)
{
    return m + ((__popcll(m) < K) ? 1ull : (m & (0ull - m)));
}

// Node-space mask (bit `node` clear) -> slot space, and back.
__device__ __forceinline__ uint64_t to_slots(uint64_t m, int node)
{
    const uint64_t low = (1ull << node) - 1ull;
    return (m & low) | ((m >> 1) & ~low);
}
__device__ __forceinline__ uint64_t to_nodes(uint64_t s, int node)
{
    const uint64_t low = (1ull << node) - 1ull;
    return (s & low) | ((s & ~low) << 1);
}

// ---- score bound
//
// For each of its orders, a block takes lower bounds on the best and the
// second-best score among the entries the order can use, from candidates kept
// per row at build (lane l of wavefront w holds slot 64 w + l): the singleton
// of slot s (usable if that node precedes), the empty set (always usable) and
// the row's listed top entries of two or more members.  The candidates are
// distinct entries, so the largest usable one bounds the best from below and
// the second largest the second best.  A tile whose largest score is below
// both the second-best bound and the best bound minus kBoundGap holds neither
// result and only terms below e^-kBoundGap of the largest one; the block
// leaves it out for that order (and reads it only if another order needs it),
// and inside a kept tile an entry below the cut counts as unusable.

// This lane's candidate (score, node-space mask); requested before the order
// is read so that the loads overlap.
__device__ __forceinline__ void bound_candidate(const TabView &V, int node, int wave, int lane, float &cv,
                                                uint64_t &cm)
{
    static_assert(kBoundSlots == kScoreThreads, "one candidate per thread of a scoring block");
    const int64_t c = (int64_t)node * kBoundSlots + wave * 64 + lane;
    cv = V.cscore[c];
    cm = V.cmask[c];
}

// b - kBoundGap, or -inf where FP32 cannot hold that gap below b (|b| of order
// 2^31 and above, where the rounded difference could come out closer to b).
__device__ __forceinline__ float gap_below(float b)
{
    const float g = b - kBoundGap;
    return (b - g >= kBoundGap) ? g : -INFINITY;
}

// The score below which a tile is left out, for predecessor complement np
// (node space).  Every thread of the block calls it (it holds a barrier).
__device__ __forceinline__ float bound_cut(float cv, uint64_t cm, uint64_t np, int wave, int lane,
                                           float (&s_lb)[kScoreThreads / 64][2])
{
    const float v = ((cm & np) == 0ull) ? cv : -INFINITY;
    const float m1 = wave_max_f32(v);
    const uint64_t at = __ballot(v == m1);
    const int l1 = at ? __builtin_ctzll(at) : 64;
    const float m2 = wave_max_f32(lane == l1 ? -INFINITY : v);
    if (lane == 0) {
        s_lb[wave][0] = m1;
        s_lb[wave][1] = m2;
    }
    __syncthreads();
    float b = s_lb[0][0];
    int wb = 0;
#pragma unroll
    for (int w = 1; w < kScoreThreads / 64; ++w)
        if (s_lb[w][0] > b) {
            b = s_lb[w][0];
            wb = w;
        }
    float sec = s_lb[wb][1];
#pragma unroll
    for (int w = 0; w < kScoreThreads / 64; ++w)
        if (w != wb) sec = fmaxf(sec, s_lb[w][0]);
    return fminf(gap_below(b), sec);
}

// The cut of one (order, node) pair computed by one wavefront alone (lane l
// holds candidates l, l + 64, l + 128, l + 192), for launches that compute
// every pair's cut before the scoring launch: the same candidates and the same
// top two, so the same value as bound_cut.  A caller that knows one more usable
// entry of the row (score kv, node-space mask km; kv = -inf: none) adds it: the
// candidate with the same mask is left out, so the top two stay two distinct
// entries and both bounds stay bounds.
__device__ __forceinline__ float wave_bound_cut(const TabView &V, int node, uint64_t np, int lane,
                                                float kv = -INFINITY, uint64_t km = ~0ull)
{
    float t1 = -INFINITY, t2 = -INFINITY;      // this lane's top two usable candidates
#pragma unroll
    for (int i = 0; i < kBoundSlots / 64; ++i) {
        const uint32_t c = (uint32_t)node * kBoundSlots + (uint32_t)(i * 64 + lane);   // < 2^14
        const uint64_t cm = V.cmask[c];
        const float cs = V.cscore[c];
        const float x = ((cm & np) == 0ull && cm != km) ? cs : -INFINITY;
        t2 = fmaxf(t2, fminf(t1, x));
        t1 = fmaxf(t1, x);
    }
    if (lane == 0) {
        t2 = fmaxf(t2, fminf(t1, kv));
        t1 = fmaxf(t1, kv);
    }
    const float m1 = wave_max_f32(t1);
    const uint64_t at = __ballot(t1 == m1);
    const int l1 = at ? __builtin_ctzll(at) : 64;
    const float m2 = wave_max_f32(lane == l1 ? t2 : t1);
    return fminf(gap_below(m1), m2);
}

// The same for the BT orders of a several-order block, after the barrier that
// published their predecessor complements: every wavefront takes each order's
// top two usable candidates among its own, and a second barrier combines them.
template <int BT>
__device__ __forceinline__ void bound_cuts(float cv, uint64_t cm, const uint64_t (&npred)[BT], int wave, int lane,
                                           float (&s_lbm)[kScoreThreads / 64][BT][2], float (&cut)[BT])
{
#pragma unroll
    for (int j = 0; j < BT; ++j) {
        const float v = ((cm & npred[j]) == 0ull) ? cv : -INFINITY;
        const float m1 = wave_max_f32(v);
        const uint64_t at = __ballot(v == m1);
        const int l1 = at ? __builtin_ctzll(at) : 64;
        const float m2 = wave_max_f32(lane == l1 ? -INFINITY : v);
        if (lane == 0) {
            s_lbm[wave][j][0] = m1;
            s_lbm[wave][j][1] = m2;
        }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < BT; ++j) {
        float b = s_lbm[0][j][0];
        int wb = 0;
#pragma unroll
        for (int w = 1; w < kScoreThreads / 64; ++w)
            if (s_lbm[w][j][0] > b) {
                b = s_lbm[w][j][0];
                wb = w;
            }
        float sec = s_lbm[wb][j][1];
#pragma unroll
        for (int w = 0; w < kScoreThreads / 64; ++w)
            if (w != wb) sec = fmaxf(sec, s_lbm[w][j][0]);
        cut[j] = fminf(gap_below(b), sec);
    }
}

// One block streams chunk `chunk` of node `node`'s entries once and folds
// each entry into BT order states (group `group` of the batch, or of the node's
// work list); it writes one Partial per order.
//
// CM (one order per block): the masks are not read but computed -- each lane
// reads the slot-space mask of its first entry (V.anchor) and steps to the
// next three with next_mask; the entries are tested against the predecessor
// set in slot space and the best mask goes back to node space for the partial.
// The states and partials are bitwise those of reading the stored masks, for
// 6 bytes per entry read instead of 12.  NOSAT steps without the saturation
// test where next_mask_nosat allows it.
template <int BT, bool CM = false, bool NOSAT = false, int RING = 0>
__device__ __forceinline__ void score_block(const TabView &V, int node, int chunk, int group, int chunks,
                                            int steps)
{
    static_assert(!CM || BT == 1, "computed masks serve one order per block");
    __shared__ uint64_t s_npred[BT];
    __shared__ Acc s_red[kScoreThreads / 64][BT];
    __shared__ int s_ord[BT];
    const int b0 = group * BT;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: scalar order and list reads
    const int n = V.n;
    // orders this block folds: slots b0..b0+BT-1 of the plain batch or of node's work list
    const int count = V.wl_count ? V.wl_count[node] : V.B;
    if (b0 >= count) return;                     // uniform: nothing listed for this group
    // The block's entries are chunk `chunk` of the node's row: the row's
    // 1024-entry steps chunk, chunk + chunks, chunk + 2 * chunks, ...; local
    // tile tl = 4 i + w is tile w of the block's i-th step.  Spread over the
    // row, a block's share of its node's work is about the same for every
    // chunk, wherever the order concentrates that work in the row (the masks
    // whose top member is one predecessor sit together, for example); a step's
    // 16 sub-tile summaries still fill one 128-byte line.
    const int64_t row = (int64_t)node * V.S_pad;             // the node's first entry
    const int64_t trow = row >> 8;                            // and first tile
    // each wavefront owns local tiles wave + 4*i, i < steps (the block's steps: chunk + i * chunks)
    auto gtile = [&](int tl) -> int64_t { return ((chunk + (int64_t)(tl >> 2) * chunks) << 2) + (tl & 3); };
    // where the summaries of this wavefront's tile of the block's step i sit: one
    // run per block when the launch takes the longest chunks
    auto spos = [&](int i) -> int64_t {
        return trow + (chunks == V.sum_chunks ? ((int64_t)chunk * V.sum_steps + i) * 4 + wave
                                              : summary_pos(chunk + (int64_t)i * chunks, wave, V.sum_chunks,
                                                            V.sum_steps));
    };
    const int64_t tpos = spos(lane < steps ? lane : 0);
    // this wavefront's tile summaries, requested before the predecessor masks so the latencies overlap
    uint64_t tsum = 0;
    if (V.tand && lane < steps) tsum = V.tand[tpos];
    // sub-tile summaries (one order per block): lane i holds the 4 of this wavefront's tile i
    u64x2 tsl01 = {0ull, 0ull}, tsl23 = {0ull, 0ull};
    if (BT == 1 && V.tand && lane < steps) {
        const u64x2 *tp = reinterpret_cast<const u64x2 *>(V.tsub + tpos * 4);
        tsl01 = tp[0];
        tsl23 = tp[1];
    }
    // score bound: lane i's tile maximum and this lane's candidate (unless the
    // cuts were computed before the launch)
    const bool bound = V.tmax != nullptr && V.tand != nullptr;
    const bool pre = bound && V.cuts != nullptr;
    __shared__ float s_lb[kScoreThreads / 64][2];
    __shared__ float s_lbm[kScoreThreads / 64][BT][2];
    float tmx = 0.f, cv = -INFINITY;
    uint64_t cm = ~0ull;
    if (bound) {
        if (lane < steps) tmx = V.tmax[tpos];
        if (!pre) bound_candidate(V, node, wave, lane, cv, cm);
    }

    // with the bound computed here and one order, every wavefront forms the predecessor set itself
    const bool own = BT == 1 && bound && !pre;
    uint64_t np_w = ~0ull;
    for (int j = own ? 0 : wave; j < BT; j += kScoreThreads / 64) {
        uint64_t np = ~0ull;   // no order in this slot: nothing is consistent
        int ob = -1;
        if (b0 + j < count) {
            ob = V.wl_count ? V.wl_list[(int64_t)node * V.B + b0 + j] : b0 + j;
            bool valid;
            uint64_t pred = wave_pred(V.orders + (int64_t)ob * n, n, node, lane, valid);
            np = ~pred;        // invalid order: only the empty set is consistent
        }
        if (lane == 0 && (!own || wave == 0)) {
            s_npred[j] = np;
            s_ord[j] = ob;
        }
        np_w = np;
    }
    // tiles whose largest score is below cut[j] are left out for order j
    float cut[BT];
#pragma unroll
    for (int j = 0; j < BT; ++j) cut[j] = -INFINITY;
    if (own) cut[0] = bound_cut(cv, cm, np_w, wave, lane, s_lb);   // holds the block barrier
    else __syncthreads();
    uint64_t npred[BT];
    Acc a[BT];
    float tt[BT];        // fold_shift(a[j].best), kept by acc_fold4
#pragma unroll
    for (int j = 0; j < BT; ++j) {
        npred[j] = uniform_u64(s_npred[j]);
        acc_init(a[j]);
        tt[j] = fold_shift(-INFINITY);
    }
    if (pre) {
#pragma unroll
        for (int j = 0; j < BT; ++j) {
            const int ob = s_ord[j];
            cut[j] = ob >= 0 ? V.cuts[(int64_t)ob * n + node] : -INFINITY;
        }
    } else if (BT > 1 && bound) {
        bound_cuts<BT>(cv, cm, npred, wave, lane, s_lbm, cut);   // a second barrier
    }

    const u64x2 *mp = reinterpret_cast<const u64x2 *>(V.masks + row);
    const f32x4 *sp = reinterpret_cast<const f32x4 *>(V.scores + row);
    const uint64_t *ap = CM ? V.anchor + (row >> 2) : nullptr;
    // slot-space predecessor complement, with every slot >= n - 1 (none exists) included
    const uint64_t npred_s = CM ? (to_slots(npred[0], node) | (~0ull << (n - 1))) : 0ull;
    const uint64_t dead = 1ull << (n - 1);   // anchor of a lane that reads nothing: slot n - 1
    // Tile skipping: if the AND of a tile's masks holds a node outside an
    // order's predecessor set, every entry of the tile does, and the order
    // skips the tile; tiles no order of the block needs are not read.  Each
    // wavefront compacts its needed tiles (kept in tile order, so the fold
    // order of the entries that matter is the same as without skipping) so
    // that every iteration loads one tile.
    __shared__ int s_tile[kScoreThreads / 64][kMaxStepsPerChunk];
    __shared__ uint32_t s_tneed[kScoreThreads / 64][kMaxStepsPerChunk];
    __shared__ int s_ntile[kScoreThreads / 64];
    {
        uint32_t m = 0;
        if (lane < steps) {
            if (V.tand) {
#pragma unroll
                for (int j = 0; j < BT; ++j)
                    m |= ((tsum & npred[j]) == 0ull && !(bound && tmx < cut[j])) ? (1u << j) : 0u;
            } else {
                m = (1u << BT) - 1u;
            }
        }
        const uint64_t bal = __ballot(m != 0u);
        if (m != 0u) {
            const int pos = __popcll(bal & ((1ull << lane) - 1ull));
            s_tile[wave][pos] = (int)gtile(lane * 4 + wave);  // the tile's index in the row
            s_tneed[wave][pos] = m | ((uint32_t)lane << 8);   // the orders that need it, and its step
        }
        if (lane == 0) s_ntile[wave] = __popcll(bal);
    }
    __syncthreads();
    const int nt = s_ntile[wave];
    // With one order per block, a lane reads its 4 entries only if the order
    // can use its 64-entry sub-tile; otherwise its masks read as ~0 (consistent
    // with nothing), so the fold is unchanged and the sub-tile's bytes are not
    // fetched.  (With several orders the union rarely skips a sub-tile and the
    // test costs more than it saves.)  Lane i holds the summaries of the
    // wavefront's i-th step tile, so four ballots give, for each sub-tile s,
    // the tiles whose sub-tile s is needed; a lane reads sub-tile lane / 16 of
    // every tile, so it keeps that ballot: bit i of `my_ok`.
    uint64_t my_ok = ~0ull;
    if (BT == 1 && V.tand) {
        const uint64_t np0 = npred[0];
        const uint64_t b0 = __ballot(lane < steps && (tsl01.x & np0) == 0ull);
        const uint64_t b1 = __ballot(lane < steps && (tsl01.y & np0) == 0ull);
        const uint64_t b2 = __ballot(lane < steps && (tsl23.x & np0) == 0ull);
        const uint64_t b3 = __ballot(lane < steps && (tsl23.y & np0) == 0ull);
        const int my_sub = lane >> 4;
        my_ok = my_sub == 0 ? b0 : (my_sub == 1 ? b1 : (my_sub == 2 ? b2 : b3));
    }
    // This lane's 4-entry group of the tile with row index gt, as an index into
    // the node's row of groups (below 2^30: rows hold fewer than 2^32 entries).
    // Prefetch ring over this wavefront's needed tiles: while the tile in
    // slot d is folded, the loads of the next D - 1 tiles are in flight; the
    // slot is refilled (with the tile D places on) right after its fold, and
    // the loop is unrolled by D so that every slot keeps its own registers.
    // RING > 0 fixes the depth; by default three slots with one order per
    // block and two with several.
    constexpr int D = RING > 0 ? RING : ((BT == 1) ? 3 : 2);
    u64x2 r01[D], r23[D];
    f32x4 rsc[D];
    uint32_t rneed[D];
#define BNOS_ISSUE(d, kk)                                                                       \
    if ((kk) < nt) {                                                                            \
        const uint32_t q_ = ((uint32_t)s_tile[wave][(kk)] << 6) | (uint32_t)lane;              \
        const uint32_t nd_ = s_tneed[wave][(kk)];                                               \
        rneed[d] = nd_ & 0xffu;                                                                 \
        r01[d] = (u64x2){CM ? dead : ~0ull, ~0ull};                                             \
        r23[d] = (u64x2){~0ull, ~0ull};                                                         \
        if ((my_ok >> (nd_ >> 8)) & 1ull) {                                                     \
            if (CM) {                                                                           \
                r01[d].x = __builtin_nontemporal_load(&ap[q_]);                                 \
            } else {                                                                            \
                r01[d] = __builtin_nontemporal_load(&mp[2 * q_]);                               \
                r23[d] = __builtin_nontemporal_load(&mp[2 * q_ + 1]);                           \
            }                                                                                   \
            rsc[d] = __builtin_nontemporal_load(&sp[q_]);                                       \
        }                                                                                       \
    }
#pragma unroll
    for (int d = 0; d < D; ++d) {
        rsc[d] = (f32x4){0.f, 0.f, 0.f, 0.f};
        rneed[d] = 0u;
        BNOS_ISSUE(d, d)
    }
    for (int k0 = 0; k0 < nt; k0 += D) {
#pragma unroll
        for (int d = 0; d < D; ++d) {
            const int k = k0 + d;
            if (k >= nt) break;                              // uniform
            uint64_t mk[4] = {r01[d].x, r01[d].y, r23[d].x, r23[d].y};
            if (CM) {
                mk[1] = NOSAT ? next_mask_nosat(mk[0], V.K) : next_mask(mk[0], V.K);
                mk[2] = NOSAT ? next_mask_nosat(mk[1], V.K) : next_mask(mk[1], V.K);
                mk[3] = NOSAT ? next_mask_nosat(mk[2], V.K) : next_mask(mk[2], V.K);
            }
            const float x[4] = {rsc[d].x, rsc[d].y, rsc[d].z, rsc[d].w};
            const uint32_t need_c = rneed[d];
#pragma unroll
            for (int j = 0; j < BT; ++j) {
                if (!((need_c >> j) & 1u)) continue;         // uniform
                const uint64_t np = CM ? npred_s : npred[j];
                float xs[4];
                bool any = false;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    // an entry below the order's cut is left out like the tiles below it (it is
                    // neither result and its term is below e^-60 of the largest); cut[j] = -inf
                    // without the bound
                    const bool ok = (mk[e] & np) == 0ull && !(x[e] < cut[j]);
                    xs[e] = ok ? x[e] : -INFINITY;
                    any |= ok;
                }
                if (__ballot(any) == 0ull) continue;         // uniform: nothing to fold in the wavefront
                if (BT == 1 && CM) {
                    acc_fold4_sel(a[j], tt[j], xs, mk);
                } else if (BT == 1) {
                    acc_fold4(a[j], tt[j], xs, mk);
                } else {                                     // registers: recompute the shift
                    float t = fold_shift(a[j].best);
                    acc_fold4(a[j], t, xs, mk);
                }
            }
            BNOS_ISSUE(d, k + D)
        }
    }
#undef BNOS_ISSUE
#pragma unroll
    for (int j = 0; j < BT; ++j) acc_fold_finish(a[j]);

    {
        // a wavefront that folded nothing (no needed tile, or no consistent entry)
        // holds identity states: skip the reduction, whose result would be the identity
        bool any = false;
#pragma unroll
        for (int j = 0; j < BT; ++j) any |= a[j].m != -INFINITY;
        Acc r;
        if (__ballot(any) != 0ull) r = (BT == 1) ? acc_wave_reduce_one(a[0]) : acc_wave_reduce_scatter<BT>(a, lane);
        else acc_init(r);
        if ((lane & (64 / BT - 1)) == 0) {
            const int j = lane / (64 / BT);
            s_red[wave][j].m = r.m;
            s_red[wave][j].s = r.s;
            s_red[wave][j].best = r.best;
            s_red[wave][j].sec = r.sec;
            s_red[wave][j].bm = r.bm;
        }
    }
    __syncthreads();
    if (threadIdx.x < BT) {
        const int j = threadIdx.x;
        if (b0 + j < count) {
            const int ob = s_ord[j];
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
            p.bmask = (CM && r.m != -INFINITY) ? to_nodes(r.bm, node) : r.bm;
            V.part[((int64_t)ob * V.chunks + chunk) * n + node] = p;
        }
    }
}

__device__ __forceinline__ TabView view_of(const ScoreArgs &A)
{
    TabView V;
    V.masks = A.masks;
    V.scores = A.scores;
    V.S_pad = A.S_pad;
    V.chunks = A.chunks;
    V.chunk_entries = A.chunk_entries;
    V.sum_chunks = A.sum_chunks;
    V.sum_steps = A.sum_steps;
    V.n = A.n;
    V.B = A.B;
    V.orders = A.orders;
    V.part = A.part;
    V.wl_count = A.wl_count;
    V.wl_list = A.wl_list;
    V.tand = A.tand;
    V.tsub = A.tsub;
    V.anchor = A.anchor;
    V.tmax = A.tmax;
    V.cmask = A.cmask;
    V.cscore = A.cscore;
    V.cuts = A.cuts;
    V.K = A.K;
    return V;
}

// Measurement only: how many 256-entry tiles k_score<BT> reads for these
// orders with tile skipping (same grid, same tests, no data loads).  One
// count per block, written to counts[blockIdx.y * gridDim.x + blockIdx.x].
template <int BT>
__global__ __launch_bounds__(kScoreThreads) void k_count_tiles(ScoreArgs A, unsigned *__restrict__ counts)
{
    __shared__ uint64_t s_np[BT];
    __shared__ unsigned s_c[kScoreThreads / 64];
    const int node = blockIdx.x / A.chunks;
    const int chunk = blockIdx.x - node * A.chunks;
    const int b0 = blockIdx.y * BT;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = A.n;
    const int count = A.B;
    const TabView V = view_of(A);
    const bool bound = A.tmax != nullptr && A.tand != nullptr;
    const bool own = BT == 1 && bound;
    __shared__ float s_lb[kScoreThreads / 64][2];
    __shared__ float s_lbm[kScoreThreads / 64][BT][2];
    float cv = -INFINITY;
    uint64_t cm = ~0ull;
    if (bound) bound_candidate(V, node, wave, lane, cv, cm);
    uint64_t np_w = ~0ull;
    for (int j = own ? 0 : wave; j < BT; j += kScoreThreads / 64) {
        uint64_t np = ~0ull;
        if (b0 + j < count) {
            bool valid;
            np = ~wave_pred(A.orders + (int64_t)(b0 + j) * n, n, node, lane, valid);
        }
        if (lane == 0 && (!own || wave == 0)) s_np[j] = np;
        np_w = np;
    }
    float cut[BT];
    for (int j = 0; j < BT; ++j) cut[j] = -INFINITY;
    if (own) cut[0] = bound_cut(cv, cm, np_w, wave, lane, s_lb);
    else __syncthreads();
    if (BT > 1 && bound) {
        uint64_t np_all[BT];
        for (int j = 0; j < BT; ++j) np_all[j] = s_np[j];
        bound_cuts<BT>(cv, cm, np_all, wave, lane, s_lbm, cut);
    }
    const int64_t trow = (int64_t)node * (A.S_pad >> 8);
    const int steps = A.chunk_entries / kEntriesPerStep;
    // 64-entry sub-tiles read: of the needed tiles, those the order can use (one
    // order per block) or all four (several)
    unsigned c = 0;
    if (b0 < count) {
        for (int it = 0; it < steps; ++it) {
            const int64_t tile = trow + summary_pos(chunk + (int64_t)it * A.chunks, wave, A.sum_chunks,
                                                    A.sum_steps);   // the summaries score_block reads
            const uint64_t sm = A.tand[tile];
            const float tm = bound ? A.tmax[tile] : 0.f;
            bool any = false;
            for (int j = 0; j < BT; ++j) any |= (sm & s_np[j]) == 0ull && !(bound && tm < cut[j]);
            if (!any) continue;
            if (BT > 1) {                  // several orders: the whole tile is read
                c += 4u;
                continue;
            }
            for (int s = 0; s < 4; ++s) c += ((A.tsub[tile * 4 + s] & s_np[0]) == 0ull) ? 1u : 0u;
        }
    }
    if (lane == 0) s_c[wave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned tot = 0;
        for (int w = 0; w < kScoreThreads / 64; ++w) tot += s_c[w];
        counts[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = tot;
    }
}

// Workgroups go to the 8 XCDs round robin by linear id, each XCD with its own
// L2.  Grids of the scoring kernels have their x extent padded to a multiple of
// 8; xcd_block maps linear id L to the column x = 8 * (l / G) + L % 8 and the
// group y = l % G (l = L / 8, G = gridDim.y), so the G groups of orders that read
// the same rows run back to back on one XCD and share its L2.  A bijection on
// the padded grid; returns false for the padding columns (x >= real_x).
constexpr int kXcds = 8;
__device__ __forceinline__ bool xcd_block(int64_t real_x, int &x, int &y)
{
    const int64_t L = blockIdx.x + (int64_t)blockIdx.y * gridDim.x;
    const int64_t l = L / kXcds;
    x = (int)((l / gridDim.y) * kXcds + L % kXcds);
    y = (int)(l % gridDim.y);
    return x < real_x;
}

// Grid: x = node * chunks + chunk, y = group of BT orders.  With one order
// per block, x runs over the order's positions from the last one down: the
// node at the last position has the most predecessors, hence the most tiles
// to read, so the longest blocks are dispatched first and the shortest fill
// the tail.  (An entry that is not a node id keeps the plain mapping; such an
// order is invalid and scores NaN anyway.)
template <int BT, bool CM = false, bool NOSAT = false, int RING = 0>
__global__ __launch_bounds__(kScoreThreads) void k_score(ScoreArgs A)
{
    int x, y;
    if (!xcd_block((int64_t)A.n * A.chunks, x, y)) return;
    int node = x / A.chunks;
    const int chunk = x - node * A.chunks;
    if (BT == 1) {
        const int v = A.orders[(int64_t)y * A.n + (A.n - 1 - node)];
        node = (v >= 0 && v < A.n) ? v : node;
    }
    score_block<BT, CM, NOSAT, RING>(view_of(A), node, chunk, y, A.chunks, A.chunk_entries / kEntriesPerStep);
}

// Index of the segment holding x, for prefix bases base[0] = 0 < ... < base[T].
__device__ __forceinline__ int find_segment(const int64_t *__restrict__ base, int T, int64_t x)
{
    int lo = 0, hi = T - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (base[mid] <= x) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Many tables in one grid: x runs over every table's (node, chunk) blocks
// (table k owns x in [blk_base[k], blk_base[k+1])), y = group of BT orders.
template <int BT>
__global__ __launch_bounds__(kScoreThreads) void k_score_multi(const TabView *__restrict__ views,
                                                              const int64_t *__restrict__ blk_base, int T)
{
    int x, y;
    if (!xcd_block(blk_base[T], x, y)) return;
    const int k = find_segment(blk_base, T, (int64_t)x);
    const TabView V = views[k];
    const int local = (int)((int64_t)x - blk_base[k]);
    const int node = local / V.chunks;
    const int chunk = local - node * V.chunks;
    score_block<BT>(V, node, chunk, y, V.chunks, V.chunk_entries / kEntriesPerStep);
}

// ------------------------------------------------------------------ gather scoring
//
// The predecessor-set enumeration of the paper's parent-set traversal, on the
// dense table: instead of streaming a node's whole row and testing every mask,
// a block enumerates the consistent parent sets themselves (the subsets of the
// node's predecessors with at most K members, K <= 4) and reads only their
// scores, at the set's rank in the row.  Ranks: the row holds the masks over the
// n-1 slots with <= K bits in ascending order, so a set with slots
// b_0 > b_1 > ... has rank sum_t nsets[b_t][K - t]; with the predecessors'
// slots P[0] < P[1] < ... the weights w_t[i] = nsets[P[i]][K - t] make a rank
// a sum of table lookups.  Block (x = node * n + s, y = order): s = 0 takes the
// empty set, s = i0 + 1 the sets whose top member is P[i0]; each writes one
// partial (order, s, node) in the layout k_merge reads with chunks = n.
constexpr int kGatherMaxK = 4;

// pair index q -> (a > b) with q = a (a - 1) / 2 + b
__device__ __forceinline__ void tri_unrank(int q, int &a, int &b)
{
    int x = (int)((1.0f + sqrtf(1.0f + 8.0f * (float)q)) * 0.5f);
    if (x * (x - 1) / 2 > q) --x;
    if ((x + 1) * x / 2 <= q) ++x;
    a = x;
    b = q - x * (x - 1) / 2;
}

constexpr int kMergeWaves = 8;

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

// LDS for the cross-wave step of merge_nodes.
struct MergeLds {
    float m[kMergeWaves][64], s[kMergeWaves][64], best[kMergeWaves][64], sec[kMergeWaves][64];
    uint64_t bm[kMergeWaves][64];
};

// Merge of one order's chunk partials (base: that order's [chunks][n] block),
// node-parallel: lane j of every one of the first kMergeWaves wavefronts
// takes node node_j (< 0: none) and folds the chunks wave, wave + W, ...
// in increasing order; the waves' states are then combined through LDS in a
// fixed tree (lower wave always the left operand).  The merged state of node
// node_j is valid in lane j of wave 0.  All threads of the block must call it.
__device__ __forceinline__ Acc merge_nodes(const Partial *__restrict__ base, int n, int chunks, int node_j,
                                           MergeLds &L)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    Acc a;
    acc_init(a);
    if (wave < kMergeWaves && node_j >= 0) {
        const Partial *p = base + node_j;
        int c = wave;
        // four loads in flight per step
        for (; c + 3 * kMergeWaves < chunks; c += 4 * kMergeWaves) {
            const Acc x0 = load_partial(p + (int64_t)c * n);
            const Acc x1 = load_partial(p + (int64_t)(c + kMergeWaves) * n);
            const Acc x2 = load_partial(p + (int64_t)(c + 2 * kMergeWaves) * n);
            const Acc x3 = load_partial(p + (int64_t)(c + 3 * kMergeWaves) * n);
            acc_merge(a, x0);
            acc_merge(a, x1);
            acc_merge(a, x2);
            acc_merge(a, x3);
        }
        for (; c < chunks; c += kMergeWaves) acc_merge(a, load_partial(p + (int64_t)c * n));
    }
    if (wave < kMergeWaves) {
        L.m[wave][lane] = a.m;
        L.s[wave][lane] = a.s;
        L.best[wave][lane] = a.best;
        L.sec[wave][lane] = a.sec;
        L.bm[wave][lane] = a.bm;
    }
    __syncthreads();
#pragma unroll
    for (int h = kMergeWaves / 2; h >= 1; h >>= 1) {
        if (wave < h) {
            Acc o;
            o.m = L.m[wave + h][lane];
            o.s = L.s[wave + h][lane];
            o.best = L.best[wave + h][lane];
            o.sec = L.sec[wave + h][lane];
            o.bm = L.bm[wave + h][lane];
            acc_merge(a, o);
            L.m[wave][lane] = a.m;
            L.s[wave][lane] = a.s;
            L.best[wave][lane] = a.best;
            L.sec[wave][lane] = a.sec;
            L.bm[wave][lane] = a.bm;
        }
        __syncthreads();
    }
    return a;
}

// Per-order merge (k_merge): node-parallel merge_nodes, then lane i of wave 0
// forms LSE_i = m + ln s in FP64, writes the node outputs, and the wave sums
// the per-node terms in FP64 with a fixed butterfly; the sums are valid in
// lane 0 of wave 0.
__device__ __forceinline__ void merge_block(const ScoreArgs &A, int b, MergeLds &L, bool &valid, double &lse_out,
                                            double &max_out)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int n = A.n;
    // the order's entries are requested first and checked after the merge, so the
    // two loads overlap
    const int v = lane < n ? A.orders[(int64_t)b * n + lane] : -1;
    const Acc r = merge_nodes(A.part + (int64_t)b * A.chunks * n, n, A.chunks, lane < n ? lane : -1, L);
    valid = order_valid(v, n, lane);
    lse_out = 0.0;
    max_out = 0.0;
    if (wave == 0) {
        double li = 0.0, mi = 0.0;
        if (lane < n) {
            li = (double)r.m + log((double)r.s);
            mi = (double)r.best;
            const int64_t o = (int64_t)b * n + lane;
            A.best[o] = valid ? r.bm : 0ull;
            if (A.node_lse) A.node_lse[o] = valid ? li : NAN;
            if (A.node_second) A.node_second[o] = valid ? r.sec : NAN;
        }
        lse_out = wave_sum_f64(li, lane);
        max_out = wave_sum_f64(mi, lane);
    }
}

// ---- host-side helpers (score.hip)
int pick_bt(const TableT *t, int B);
bnos_status ensure_workspace(TableT *t, int B);
ScoreArgs score_args(const TableT *t, const int32_t *orders, int B, double *lse, double *maxs,
                     uint64_t *best, double *node_lse, float *node_second);
bnos_status launch_stream(TableT *t, const ScoreArgs &A, hipStream_t st, int bt, bool allow_timing = true);
bnos_status launch_gather(TableT *t, ScoreArgs &A, hipStream_t st, bool allow_timing = true);
bnos_status launch_merge(const ScoreArgs &A, hipStream_t st);

}  // namespace bnos
