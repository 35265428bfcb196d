/*
 * CPU oracle for order-space Bayesian-network structure learning.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, FP64 restatement of
 * what the method computes, used to check the GPU library.  It shares no code,
 * header, table or constant with the GPU path, and the product never links it.
 *
 * What it follows (Wang, Zhang, Qian, Yuan, "A Novel Learning Algorithm for
 * Bayesian Network and Its Efficient Implementation on GPU"):
 *   - counts N_ijk over complete discrete data and the Bayesian-Dirichlet local
 *     score with structure penalty gamma^|pi| (Sec. II, Eq. (3); log form
 *     Sec. III.A, Eq. (4)), with the BDeu choice of Dirichlet parameters;
 *   - the pairwise prior added per present edge (Sec. IV, Eq. (7)-(9)) through
 *     the cubic prior function of Eq. (10);
 *   - scoring an order: for every node, all parent sets of size <= s drawn from
 *     the nodes that precede it (Sec. III.B, Alg. 1), reduced by max / argmax
 *     (Eq. (6)) and by the sum over consistent graphs used as the alternative
 *     order score (the sum-based score discussed in Sec. III.B);
 *   - the Metropolis-Hastings walk over orders with two-node swaps
 *     (Sec. III.C) and the best-graph record (Sec. III.C).
 *
 * Readings where the paper is silent (all natural logs; BDeu alpha; argmax
 * tie rule; RNG) are stated next to the code that takes them.
 *
 * Parity status: every function here is pinned by the CPU test suite
 * (exact rational arithmetic, closed forms, score equivalence, brute force
 * over all DAGs for n <= 5, exact stationarity for n <= 4).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ */
/* Binomials and parent-set counts                                     */
/* ------------------------------------------------------------------ */

static int64_t orc_binom(int a, int b)
{
    if (b < 0 || a < 0 || b > a) return 0;
    int64_t r = 1;
    for (int t = 1; t <= b; ++t) r = r * (a - b + t) / t;   /* exact at every step */
    return r;
}

/* Number of subsets of a set of size m with at most K members. */
int64_t orc_num_sets(int m, int K)
{
    int64_t s = 0;
    for (int j = 0; j <= K && j <= m; ++j) s += orc_binom(m, j);
    return s;
}

/* ------------------------------------------------------------------ */
/* Counts N_ijk (Sec. II, below Eq. (3): "counted from experimental data") */
/* ------------------------------------------------------------------ */

/*
 * Cell layout: the members of pi listed ascending m1 < m2 < ... < md give the
 * parent configuration k = ((x_m1 * r_m2 + x_m2) * r_m3 + ...), lowest id most
 * significant; the cell of (k, child state j) is k * r_i + j.
 * Returns the number of cells q_i * r_i.
 */
int64_t orc_counts(const int8_t *data, int64_t N, int n, const int32_t *ar,
                   int node, uint64_t pmask, uint32_t *counts)
{
    int64_t q = 1;
    for (int m = 0; m < n; ++m)
        if ((pmask >> m) & 1ULL) q *= ar[m];
    int64_t cells = q * ar[node];
    for (int64_t c = 0; c < cells; ++c) counts[c] = 0;
    for (int64_t t = 0; t < N; ++t) {
        const int8_t *row = data + t * (int64_t)n;
        int64_t k = 0;
        for (int m = 0; m < n; ++m)
            if ((pmask >> m) & 1ULL) k = k * ar[m] + row[m];
        counts[k * ar[node] + row[node]] += 1;
    }
    return cells;
}

/* ------------------------------------------------------------------ */
/* Pairwise prior function (Sec. IV)                                    */
/* ------------------------------------------------------------------ */

/*
 * Eq. (10): PPF = 100 (R - 0.5)^3, a log10 quantity (Eq. (8)-(9) add
 * log10 p(i,m)).  All scores here are natural logs, so the added term is
 * ln(10) * PPF.  mode 0: the caller gives w in [-1,1] with R = (1 + w) / 2;
 * mode 1: the caller gives the paper's R in [0,1] directly.
 */
double orc_ppf_nats(double v, int mode)
{
    double R = (mode == 0) ? 0.5 * (1.0 + v) : v;
    double d = R - 0.5;
    return log(10.0) * 100.0 * d * d * d;
}

/* ------------------------------------------------------------------ */
/* Local score (Eq. (3)/(4) in natural logs, plus Eq. (9) prior terms) */
/* ------------------------------------------------------------------ */

/*
 * ls(i,pi) = |pi| ln(gamma)
 *          + sum_k [ lnG(a_ik) - lnG(a_ik + N_ik)
 *                    + sum_j ( lnG(N_ijk + a_ijk) - lnG(a_ijk) ) ]
 * with BDeu parameters a_ijk = ess / (q_i r_i), a_ik = ess / q_i.
 * A configuration k with N_ik = 0, and a cell with N_ijk = 0, contribute
 * lnG(a) - lnG(a) = 0 exactly, so they are skipped without changing the sum.
 * prior: n x n floats, row = child i, column = parent m (edge m -> i), or NULL.
 */
double orc_local_score(const int8_t *data, int64_t N, int n, const int32_t *ar,
                       int node, uint64_t pmask, double ess, double log_gamma,
                       const float *prior, int prior_mode)
{
    int64_t q = 1;
    int size = 0;
    for (int m = 0; m < n; ++m)
        if ((pmask >> m) & 1ULL) { q *= ar[m]; ++size; }
    int r = ar[node];
    uint32_t *counts = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(q * r));
    orc_counts(data, N, n, ar, node, pmask, counts);
    double a_ijk = ess / (double)(q * r);
    double a_ik = ess / (double)q;
    double ls = size * log_gamma;
    for (int64_t k = 0; k < q; ++k) {
        int64_t Nik = 0;
        for (int j = 0; j < r; ++j) Nik += counts[k * r + j];
        if (Nik == 0) continue;
        ls += lgamma(a_ik) - lgamma(a_ik + (double)Nik);
        for (int j = 0; j < r; ++j) {
            uint32_t c = counts[k * r + j];
            if (c == 0) continue;
            ls += lgamma((double)c + a_ijk) - lgamma(a_ijk);
        }
    }
    free(counts);
    if (prior) {
        for (int m = 0; m < n; ++m)
            if ((pmask >> m) & 1ULL) ls += orc_ppf_nats((double)prior[(int64_t)node * n + m], prior_mode);
    }
    return ls;
}

/* ------------------------------------------------------------------ */
/* Rank-indexed table (the oracle's own layout, no hashing)             */
/* ------------------------------------------------------------------ */

/*
 * The candidate parents of node i are the n-1 other nodes, renumbered as
 * slots 0..n-2 (node id m -> slot m if m < i else m - 1).  A subset of slots
 * {c_1 < ... < c_j} gets the dense index
 *     offset(j) + sum_t C(c_t, t)      (combinatorial number system),
 * offset(j) = sum_{j' < j} C(n-1, j').
 */
static int slot_of(int node, int m) { return m < node ? m : m - 1; }
static int node_of(int node, int s) { return s < node ? s : s + 1; }

int64_t orc_rank(int n, int K, int node, uint64_t pmask)
{
    int cs[64];
    int j = 0;
    for (int m = 0; m < n; ++m)
        if ((pmask >> m) & 1ULL) cs[j++] = slot_of(node, m);
    if (j > K) return -1;
    int64_t idx = 0;
    for (int jj = 0; jj < j; ++jj) idx += orc_binom(n - 1, jj);
    for (int t = 0; t < j; ++t) idx += orc_binom(cs[t], t + 1);
    return idx;
}

/* Inverse of orc_rank: the node-id mask of the subset with dense index idx. */
uint64_t orc_unrank(int n, int K, int node, int64_t idx)
{
    int j = 0;
    while (j <= K && idx >= orc_binom(n - 1, j)) { idx -= orc_binom(n - 1, j); ++j; }
    uint64_t mask = 0;
    int top = n - 2;
    for (int t = j; t >= 1; --t) {
        /* largest c with C(c, t) <= idx */
        int c = top;
        while (orc_binom(c, t) > idx) --c;
        idx -= orc_binom(c, t);
        mask |= 1ULL << node_of(node, c);
        top = c - 1;
    }
    return mask;
}

/* Part of one node's row: out[rank] = s(node, unrank(rank)) for r0 <= rank < r1. */
void orc_build_row(const int8_t *data, int64_t N, int n, const int32_t *ar, int K, double ess,
                   double log_gamma, const float *prior, int prior_mode, int node,
                   int64_t r0, int64_t r1, double *out)
{
    for (int64_t r = r0; r < r1; ++r)
        out[r] = orc_local_score(data, N, n, ar, node, orc_unrank(n, K, node, r), ess, log_gamma,
                                 prior, prior_mode);
}

/* Full table: out[node * S + rank] = s(node, unrank(rank)), S = S(n-1, K). */
void orc_build_table(const int8_t *data, int64_t N, int n, const int32_t *ar, int K,
                     double ess, double log_gamma, const float *prior, int prior_mode,
                     double *out)
{
    int64_t S = orc_num_sets(n - 1, K);
    for (int i = 0; i < n; ++i)
        for (int64_t r = 0; r < S; ++r)
            out[(int64_t)i * S + r] = orc_local_score(data, N, n, ar, i, orc_unrank(n, K, i, r),
                                                      ess, log_gamma, prior, prior_mode);
}

/* ------------------------------------------------------------------ */
/* Order scoring by enumeration (Sec. III.B, Alg. 1 and Eq. (6))        */
/* ------------------------------------------------------------------ */

/*
 * Argmax tie rule (the paper's loop keeps the first of equal scores, and its
 * enumeration order is unspecified): the larger score wins; on equal scores
 * the numerically smaller parent mask wins.  This rule does not depend on any
 * storage order.
 */
static int beats(double s, uint64_t m, double bs, uint64_t bm)
{
    return s > bs || (s == bs && m < bm);
}

typedef struct {
    double *vals;      /* every consistent score, in enumeration order */
    uint64_t *masks;
    int64_t cnt, cap;
} orc_list;

static void list_push(orc_list *L, double v, uint64_t m)
{
    if (L->cnt == L->cap) {
        L->cap = L->cap ? 2 * L->cap : 1024;
        L->vals = (double *)realloc(L->vals, sizeof(double) * (size_t)L->cap);
        L->masks = (uint64_t *)realloc(L->masks, sizeof(uint64_t) * (size_t)L->cap);
    }
    L->vals[L->cnt] = v;
    L->masks[L->cnt] = m;
    L->cnt++;
}

/* Reduce a node's list of consistent scores: LSE (two-pass, max shifted),
 * argmax with the tie rule, and the best score among the other entries. */
static void reduce_node(const orc_list *L, double *lse, double *best, uint64_t *best_mask,
                        double *second)
{
    double mx = -INFINITY;
    for (int64_t t = 0; t < L->cnt; ++t) if (L->vals[t] > mx) mx = L->vals[t];
    double sum = 0.0;
    for (int64_t t = 0; t < L->cnt; ++t) sum += exp(L->vals[t] - mx);
    *lse = mx + log(sum);
    double bs = -INFINITY;
    uint64_t bm = ~0ULL;
    int64_t bt = -1;
    for (int64_t t = 0; t < L->cnt; ++t)
        if (beats(L->vals[t], L->masks[t], bs, bm)) { bs = L->vals[t]; bm = L->masks[t]; bt = t; }
    double sec = -INFINITY;
    for (int64_t t = 0; t < L->cnt; ++t)
        if (t != bt && L->vals[t] > sec) sec = L->vals[t];
    *best = bs;
    *best_mask = bm;
    *second = sec;
}

/* Round to the nearest FP32 value (ties to even), returned as a double. */
static double to_f32(double v) { return (double)(float)v; }

/* Recursively list every subset of preds[from..] of size <= left, added to cur. */
typedef struct {
    const double *row;   /* the node's table row, or NULL for direct scoring */
    int n, K, node;
    int round_f32;
    const int8_t *data; int64_t N; const int32_t *ar;
    double ess, log_gamma; const float *prior; int prior_mode;
} orc_ctx;

static void enum_sets(const orc_ctx *c, const int *preds, int np, int from, int left,
                      uint64_t cur, orc_list *L)
{
    double v;
    if (c->row) v = c->row[orc_rank(c->n, c->K, c->node, cur)];
    else v = orc_local_score(c->data, c->N, c->n, c->ar, c->node, cur, c->ess, c->log_gamma,
                             c->prior, c->prior_mode);
    if (c->round_f32) v = to_f32(v);
    list_push(L, v, cur);
    if (left == 0) return;
    for (int t = from; t < np; ++t)
        enum_sets(c, preds, np, t + 1, left - 1, cur | (1ULL << preds[t]), L);
}

static void score_node(const orc_ctx *c, uint64_t pred, double *lse, double *best,
                       uint64_t *best_mask, double *second)
{
    int preds[64];
    int np = 0;
    for (int m = 0; m < c->n; ++m)
        if ((pred >> m) & 1ULL) preds[np++] = m;
    orc_list L = {0};
    enum_sets(c, preds, np, 0, c->K, 0ULL, &L);
    reduce_node(&L, lse, best, best_mask, second);
    free(L.vals);
    free(L.masks);
}

/*
 * Score one order against a rank-indexed table (n x S doubles).
 * order[p] = node id at position p.  Outputs (natural logs):
 *   *lse  = sum_i ln sum_{pi consistent} exp s(i,pi)   (sum-based order score)
 *   *mx   = sum_i max_{pi consistent} s(i,pi)           (Eq. (6))
 *   best_masks[i]  = the greedy best parent set of node i (by node id)
 *   node_lse[i], node_second[i] (may be NULL).
 * With round_f32 != 0 every table value is first rounded to FP32, the
 * precision in which the GPU stores scores and takes its argmax.
 */
void orc_score_order(const double *table, int n, int K, const int32_t *order, int round_f32,
                     double *lse, double *mx, uint64_t *best_masks, double *node_lse,
                     double *node_best, double *node_second)
{
    int64_t S = orc_num_sets(n - 1, K);
    uint64_t pred = 0;
    double tl = 0.0, tm = 0.0;
    for (int p = 0; p < n; ++p) {
        int i = order[p];
        orc_ctx c = {0};
        c.row = table + (int64_t)i * S;
        c.n = n; c.K = K; c.node = i; c.round_f32 = round_f32;
        double l, b, s2;
        uint64_t bm;
        score_node(&c, pred, &l, &b, &bm, &s2);
        tl += l;
        tm += b;
        if (best_masks) best_masks[i] = bm;
        if (node_lse) node_lse[i] = l;
        if (node_best) node_best[i] = b;
        if (node_second) node_second[i] = s2;
        pred |= 1ULL << i;
    }
    *lse = tl;
    *mx = tm;
}

/* Score one node against its own table row, given its predecessor mask. */
void orc_score_node_row(const double *row, int n, int K, int node, uint64_t pred, int round_f32,
                        double *lse, double *best, uint64_t *best_mask, double *second)
{
    orc_ctx c = {0};
    c.row = row; c.n = n; c.K = K; c.node = node; c.round_f32 = round_f32;
    score_node(&c, pred, lse, best, best_mask, second);
}

/*
 * Score one node straight from the data (no table): the same enumeration,
 * with every local score computed on demand.  For spot checks of large n.
 */
void orc_score_node_direct(const int8_t *data, int64_t N, int n, const int32_t *ar, int K,
                           double ess, double log_gamma, const float *prior, int prior_mode,
                           int node, uint64_t pred, int round_f32,
                           double *lse, double *best, uint64_t *best_mask, double *second)
{
    orc_ctx c = {0};
    c.row = NULL; c.n = n; c.K = K; c.node = node; c.round_f32 = round_f32;
    c.data = data; c.N = N; c.ar = ar; c.ess = ess; c.log_gamma = log_gamma;
    c.prior = prior; c.prior_mode = prior_mode;
    score_node(&c, pred, lse, best, best_mask, second);
}

/* ------------------------------------------------------------------ */
/* Counter-based random numbers (SplitMix64 finalizer)                  */
/* ------------------------------------------------------------------ */

/*
 * One 64-bit draw per (seed, chain, purpose, step), from the finalizer of
 * Steele, Lea & Flood's SplitMix64 (OOPSLA 2014):
 *     mix(z) = z ^ (z >> 31) after z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9,
 *              z = (z ^ (z >> 27)) * 0x94D049BB133111EB
 *     key    = mix(seed ^ mix(chain * 8 + purpose + 1))
 *     draw   = mix(key + (step + 1) * 0x9E3779B97F4A7C15)
 * Purposes: 0 initial shuffle, 1 first swap position, 2 second swap
 * position, 3 acceptance uniform.
 */
static uint64_t orc_mix(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t orc_draw(uint64_t seed, uint64_t chain, uint64_t purpose, uint64_t step)
{
    uint64_t key = orc_mix(seed ^ orc_mix(chain * 8 + purpose + 1));
    return orc_mix(key + (step + 1) * 0x9E3779B97F4A7C15ULL);
}

/* Integer in [0, m): high 32 bits scaled by m (multiply-shift). */
static uint32_t below(uint64_t x, uint32_t m) { return (uint32_t)(((x >> 32) * (uint64_t)m) >> 32); }

/* Uniform double in the open interval (0, 1) from the top 53 bits. */
static double unit_open(uint64_t x) { return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

/* Initial order: identity shuffled by Fisher-Yates, j drawn for p = n-1..1. */
void orc_initial_order(uint64_t seed, uint64_t chain, int n, int32_t *order)
{
    for (int p = 0; p < n; ++p) order[p] = p;
    for (int p = n - 1; p >= 1; --p) {
        uint32_t j = below(orc_draw(seed, chain, 0, (uint64_t)p), (uint32_t)(p + 1));
        int32_t t = order[p]; order[p] = order[j]; order[j] = t;
    }
}

/* The two distinct positions swapped at step t (uniform over unordered pairs). */
void orc_swap_pair(uint64_t seed, uint64_t chain, int n, uint64_t step, int *a, int *b)
{
    uint32_t x = below(orc_draw(seed, chain, 1, step), (uint32_t)n);
    uint32_t y = below(orc_draw(seed, chain, 2, step), (uint32_t)(n - 1));
    if (y >= x) y += 1;
    *a = (int)x;
    *b = (int)y;
}

double orc_accept_uniform(uint64_t seed, uint64_t chain, uint64_t step)
{
    return unit_open(orc_draw(seed, chain, 3, step));
}

/* ------------------------------------------------------------------ */
/* Metropolis-Hastings over orders (Sec. III.C)                          */
/* ------------------------------------------------------------------ */

/*
 * Record of the k best distinct graphs seen by a chain (Sec. III.C keeps a
 * number of best graphs): offered the greedy graph of the initial order and of
 * every accepted order.  Kept in decreasing order of score; a graph equal to a
 * recorded one is not added again; among equal scores the earlier record stays
 * ahead; when full, a new graph enters only with a score strictly above the
 * last one, which then drops out.  graphs [k][n], scores [k].
 */
void orc_topk_offer(int n, int k, uint64_t *graphs, double *scores, int32_t *count, const uint64_t *g, double s)
{
    int cnt = *count;
    for (int r = 0; r < cnt; ++r)
        if (memcmp(graphs + (size_t)r * n, g, sizeof(uint64_t) * (size_t)n) == 0) return;
    int pos = 0;
    while (pos < cnt && scores[pos] >= s) ++pos;
    if (pos >= k) return;
    int last = cnt < k ? cnt : k - 1;
    for (int r = last; r > pos; --r) {
        memcpy(graphs + (size_t)r * n, graphs + (size_t)(r - 1) * n, sizeof(uint64_t) * (size_t)n);
        scores[r] = scores[r - 1];
    }
    memcpy(graphs + (size_t)pos * n, g, sizeof(uint64_t) * (size_t)n);
    scores[pos] = s;
    if (cnt < k) *count = cnt + 1;
}

/*
 * One chain of `iters` iterations on a rank-indexed table.
 *   target 0: the order score is the log-sum-exp score; 1: the max score of
 *   Eq. (6).  An iteration (t = 1..iters) proposes a swap of two distinct
 *   positions, scores the new order and accepts iff ln u < new - old (strict).
 *   The best-graph record starts from the initial order's greedy graph and is
 *   replaced, after an accepted move, when that order's max score is strictly
 *   larger.
 * Outputs: final order (order_out[n]); trace[t] = target score of the current
 * order after iteration t (trace[0] = initial); acc[t-1] = 1 if accepted;
 * best graph (parent mask per node id) and its score; accepted count; with
 * topk > 0 the record of the topk best distinct graphs (orc_topk_offer).
 */
void orc_run_chain(const double *table, int n, int K, uint64_t seed, uint64_t chain,
                   int64_t iters, int target, int round_f32,
                   int32_t *order_out, double *trace, uint8_t *acc,
                   uint64_t *best_graph, double *best_score, int64_t *accepted,
                   int topk, uint64_t *top_graphs, double *top_scores, int32_t *top_count)
{
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *prop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    orc_initial_order(seed, chain, n, cur);
    double l, m;
    orc_score_order(table, n, K, cur, round_f32, &l, &m, best_graph, NULL, NULL, NULL);
    double cur_score = target == 0 ? l : m;
    *best_score = m;
    if (topk > 0) {
        *top_count = 0;
        orc_topk_offer(n, topk, top_graphs, top_scores, top_count, best_graph, m);
    }
    int64_t nacc = 0;
    if (trace) trace[0] = cur_score;
    for (int64_t t = 1; t <= iters; ++t) {
        int a, b;
        orc_swap_pair(seed, chain, n, (uint64_t)t, &a, &b);
        memcpy(prop, cur, sizeof(int32_t) * (size_t)n);
        int32_t tmp = prop[a]; prop[a] = prop[b]; prop[b] = tmp;
        double pl, pm;
        orc_score_order(table, n, K, prop, round_f32, &pl, &pm, g, NULL, NULL, NULL);
        double new_score = target == 0 ? pl : pm;
        double u = orc_accept_uniform(seed, chain, (uint64_t)t);
        int ok = log(u) < new_score - cur_score;
        if (ok) {
            memcpy(cur, prop, sizeof(int32_t) * (size_t)n);
            cur_score = new_score;
            ++nacc;
            if (pm > *best_score) {
                *best_score = pm;
                memcpy(best_graph, g, sizeof(uint64_t) * (size_t)n);
            }
            if (topk > 0) orc_topk_offer(n, topk, top_graphs, top_scores, top_count, g, pm);
        }
        if (acc) acc[t - 1] = (uint8_t)ok;
        if (trace) trace[t] = cur_score;
    }
    memcpy(order_out, cur, sizeof(int32_t) * (size_t)n);
    *accepted = nacc;
    free(cur);
    free(prop);
    free(g);
}

/* ------------------------------------------------------------------ */
/* Learned swap proposal (exact MH correction)                          */
/* ------------------------------------------------------------------ */

/*
 * A small network scores every node of the current order; the scores define
 * a distribution over unordered node pairs, and the two nodes' positions are
 * swapped.  Because the proposal is not symmetric, the acceptance test uses
 * the Metropolis-Hastings ratio with q evaluated in both directions:
 *     accept iff ln u < [score(new) - score(old)] + ln q(pair | new) - ln q(pair | old).
 *
 * Per-node features (8), for node i in order o:
 *   0 position / n; 1 best consistent local score s(i, best_i);
 *   2 gap best - second best (0 when the empty set is the only candidate);
 *   3 sum_m prior(i, m) (prior terms in nats, row); 4 sum_j prior(j, i) (column);
 *   5, 6, 7 max, mean, standard deviation of s(i, .) over all candidate sets.
 * They enter the network z-scored: z = (f - mu) / sd.
 * Network: h1 = relu(W1 z + b1), h2 = relu(W2 h1 + b2), l = w3 . h2 + b3, with
 * W1 128x8, W2 128x128; parameters flattened as W1, b1, W2, b2, w3, b3 (17,793).
 * Pair distribution, p = softmax(l) over the n nodes, eps mixing weight:
 *   q({a,b}) = (1 - eps) p_a p_b (1/(1 - p_a) + 1/(1 - p_b)) + eps * 2 / (n (n - 1)),
 * i.e. with probability eps a uniform pair, else a ~ p then b ~ p without a.
 */
#define ORC_H 128
#define ORC_F 8
#define ORC_NPARAM (ORC_H * ORC_F + ORC_H + ORC_H * ORC_H + ORC_H + ORC_H + 1)

int orc_mlp_num_params(void) { return ORC_NPARAM; }

/* max, mean, population standard deviation of each node's row (FP32-rounded values if round_f32). */
void orc_table_stats(const double *table, int n, int K, int round_f32, double *stats /*[n][3]*/)
{
    int64_t S = orc_num_sets(n - 1, K);
    for (int i = 0; i < n; ++i) {
        double mx = -INFINITY, sum = 0.0, sq = 0.0;
        for (int64_t r = 0; r < S; ++r) {
            double v = table[(int64_t)i * S + r];
            if (round_f32) v = to_f32(v);
            if (v > mx) mx = v;
            sum += v;
        }
        double mean = sum / (double)S;
        for (int64_t r = 0; r < S; ++r) {
            double v = table[(int64_t)i * S + r];
            if (round_f32) v = to_f32(v);
            sq += (v - mean) * (v - mean);
        }
        stats[i * 3 + 0] = mx;
        stats[i * 3 + 1] = mean;
        stats[i * 3 + 2] = sqrt(sq / (double)S);
    }
}

/* Raw features of every node (by node id) for an order, from its per-node
 * best / second-best scores (as orc_score_order returns them). */
void orc_features(int n, const int32_t *order, const double *node_best, const double *node_second,
                  const double *prior_nats /*[n][n] or NULL*/, const double *stats, double *f /*[n][8]*/)
{
    for (int p = 0; p < n; ++p) f[order[p] * ORC_F + 0] = (double)p / (double)n;
    for (int i = 0; i < n; ++i) {
        double *r = f + i * ORC_F;
        r[1] = node_best[i];
        r[2] = isinf(node_second[i]) ? 0.0 : node_best[i] - node_second[i];
        double row = 0.0, col = 0.0;
        if (prior_nats)
            for (int m = 0; m < n; ++m) {
                if (m == i) continue;
                row += prior_nats[i * n + m];
                col += prior_nats[m * n + i];
            }
        r[3] = row;
        r[4] = col;
        r[5] = stats[i * 3 + 0];
        r[6] = stats[i * 3 + 1];
        r[7] = stats[i * 3 + 2];
    }
}

/* Forward pass for n nodes: z [n][8] (already normalised) -> logits [n].
 * pre1/pre2 [n][128] (optional) receive the pre-activations. */
void orc_mlp_forward(const double *prm, int n, const double *z, double *logits, double *pre1, double *pre2)
{
    const double *W1 = prm, *b1 = W1 + ORC_H * ORC_F, *W2 = b1 + ORC_H, *b2 = W2 + ORC_H * ORC_H;
    const double *w3 = b2 + ORC_H, *b3 = w3 + ORC_H;
    double h1[ORC_H], h2[ORC_H];
    for (int i = 0; i < n; ++i) {
        for (int u = 0; u < ORC_H; ++u) {
            double a = b1[u];
            for (int k = 0; k < ORC_F; ++k) a += W1[u * ORC_F + k] * z[i * ORC_F + k];
            if (pre1) pre1[i * ORC_H + u] = a;
            h1[u] = a > 0.0 ? a : 0.0;
        }
        for (int u = 0; u < ORC_H; ++u) {
            double a = b2[u];
            for (int k = 0; k < ORC_H; ++k) a += W2[u * ORC_H + k] * h1[k];
            if (pre2) pre2[i * ORC_H + u] = a;
            h2[u] = a > 0.0 ? a : 0.0;
        }
        double l = b3[0];
        for (int u = 0; u < ORC_H; ++u) l += w3[u] * h2[u];
        logits[i] = l;
    }
}

static void softmax(const double *l, int n, double *p)
{
    double mx = -INFINITY;
    for (int i = 0; i < n; ++i) if (l[i] > mx) mx = l[i];
    double s = 0.0;
    for (int i = 0; i < n; ++i) { p[i] = exp(l[i] - mx); s += p[i]; }
    for (int i = 0; i < n; ++i) p[i] /= s;
}

/* ln q({a, b}) for nodes a != b. */
double orc_pair_logq(const double *logits, int n, int a, int b, double eps)
{
    double p[64];
    softmax(logits, n, p);
    double Q = p[a] * p[b] * (1.0 / (1.0 - p[a]) + 1.0 / (1.0 - p[b]));
    return log((1.0 - eps) * Q + eps * 2.0 / ((double)n * (n - 1)));
}

/*
 * Loss -ln q({a,b} | z) of one sample and its gradient, added to grad[]
 * (same layout as prm).  Returns the loss.
 */
double orc_mlp_loss_grad(const double *prm, int n, const double *z, int a, int b, double eps, double *grad)
{
    const double *W1 = prm, *b1 = W1 + ORC_H * ORC_F, *W2 = b1 + ORC_H, *b2 = W2 + ORC_H * ORC_H;
    const double *w3 = b2 + ORC_H;
    (void)b1; (void)b2;
    double *gW1 = grad, *gb1 = gW1 + ORC_H * ORC_F, *gW2 = gb1 + ORC_H, *gb2 = gW2 + ORC_H * ORC_H;
    double *gw3 = gb2 + ORC_H, *gb3 = gw3 + ORC_H;
    double logits[64], p[64], dl[64];
    double *pre1 = (double *)malloc(sizeof(double) * (size_t)n * ORC_H);
    double *pre2 = (double *)malloc(sizeof(double) * (size_t)n * ORC_H);
    orc_mlp_forward(prm, n, z, logits, pre1, pre2);
    softmax(logits, n, p);
    double pa = p[a], pb = p[b];
    double Q = pa * pb * (1.0 / (1.0 - pa) + 1.0 / (1.0 - pb));
    double U = 2.0 / ((double)n * (n - 1));
    double q = (1.0 - eps) * Q + eps * U;
    /* dQ/dp_a = p_b (1/(1-p_a)^2 + 1/(1-p_b)), dQ/dp_b symmetric; through the softmax:
       dQ/dl_k = [k=a] g_a + [k=b] g_b - p_k (g_a + g_b), g_x = p_x dQ/dp_x. */
    double ga = pa * pb * (1.0 / ((1.0 - pa) * (1.0 - pa)) + 1.0 / (1.0 - pb));
    double gb = pb * pa * (1.0 / ((1.0 - pb) * (1.0 - pb)) + 1.0 / (1.0 - pa));
    for (int k = 0; k < n; ++k) {
        double dQ = -p[k] * (ga + gb) + (k == a ? ga : 0.0) + (k == b ? gb : 0.0);
        dl[k] = -(1.0 - eps) * dQ / q;
    }
    for (int i = 0; i < n; ++i) {
        double h1[ORC_H], h2[ORC_H], d2[ORC_H], d1[ORC_H];
        for (int u = 0; u < ORC_H; ++u) {
            h1[u] = pre1[i * ORC_H + u] > 0.0 ? pre1[i * ORC_H + u] : 0.0;
            h2[u] = pre2[i * ORC_H + u] > 0.0 ? pre2[i * ORC_H + u] : 0.0;
        }
        gb3[0] += dl[i];
        for (int u = 0; u < ORC_H; ++u) {
            gw3[u] += dl[i] * h2[u];
            d2[u] = pre2[i * ORC_H + u] > 0.0 ? dl[i] * w3[u] : 0.0;
            gb2[u] += d2[u];
        }
        for (int u = 0; u < ORC_H; ++u)
            for (int k = 0; k < ORC_H; ++k) gW2[u * ORC_H + k] += d2[u] * h1[k];
        for (int k = 0; k < ORC_H; ++k) {
            double s = 0.0;
            for (int u = 0; u < ORC_H; ++u) s += W2[u * ORC_H + k] * d2[u];
            d1[k] = pre1[i * ORC_H + k] > 0.0 ? s : 0.0;
            gb1[k] += d1[k];
        }
        for (int u = 0; u < ORC_H; ++u)
            for (int k = 0; k < ORC_F; ++k) gW1[u * ORC_F + k] += d1[u] * z[i * ORC_F + k];
    }
    free(pre1);
    free(pre2);
    return -log(q);
}

/* Draw an unordered node pair from q at iteration `step` (purposes 4: mixture
 * choice, 5: first node, 6: second node, 1/2: uniform positions); returns the
 * two POSITIONS to swap. */
void orc_learned_pair(uint64_t seed, uint64_t chain, int n, uint64_t step, const double *logits,
                      const int32_t *order, double eps, int *pa_out, int *pb_out)
{
    double mix = unit_open(orc_draw(seed, chain, 4, step));
    if (mix < eps) { orc_swap_pair(seed, chain, n, step, pa_out, pb_out); return; }
    double p[64];
    softmax(logits, n, p);
    double u = unit_open(orc_draw(seed, chain, 5, step));
    int a = n - 1;
    double c = 0.0;
    for (int i = 0; i < n; ++i) { c += p[i]; if (u < c) { a = i; break; } }
    double v = unit_open(orc_draw(seed, chain, 6, step)) * (1.0 - p[a]);
    int b = (a == n - 1) ? n - 2 : n - 1;
    c = 0.0;
    for (int i = 0; i < n; ++i) {
        if (i == a) continue;
        c += p[i];
        if (v < c) { b = i; break; }
    }
    int pos_a = 0, pos_b = 0;
    for (int q = 0; q < n; ++q) { if (order[q] == a) pos_a = q; if (order[q] == b) pos_b = q; }
    *pa_out = pos_a;
    *pb_out = pos_b;
}

static void node_of_positions(const int32_t *order, int pa, int pb, int *a, int *b) { *a = order[pa]; *b = order[pb]; }

/*
 * MH chain with the learned proposal (same conventions as orc_run_chain).
 * prm: network parameters; mu, sd: feature normalisation; prior_nats: [n][n]
 * prior terms or NULL; stats: [n][3] table statistics.
 */
void orc_run_chain_learned(const double *table, int n, int K, uint64_t seed, uint64_t chain, int64_t iters,
                           int target, int round_f32, const double *prm, const double *mu, const double *sd,
                           const double *prior_nats, const double *stats, double eps,
                           int32_t *order_out, double *trace, uint8_t *acc, uint64_t *best_graph,
                           double *best_score, int64_t *accepted,
                           int topk, uint64_t *top_graphs, double *top_scores, int32_t *top_count)
{
    int32_t *cur = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *prop = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    uint64_t *g = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    double nl[64], nb[64], ns[64], f[64 * ORC_F], z[64 * ORC_F], lc[64], lp[64];
    orc_initial_order(seed, chain, n, cur);
    double l, m;
    orc_score_order(table, n, K, cur, round_f32, &l, &m, best_graph, nl, nb, ns);
    double cur_score = target == 0 ? l : m;
    *best_score = m;
    if (topk > 0) {
        *top_count = 0;
        orc_topk_offer(n, topk, top_graphs, top_scores, top_count, best_graph, m);
    }
    orc_features(n, cur, nb, ns, prior_nats, stats, f);
    for (int k = 0; k < n * ORC_F; ++k) z[k] = (f[k] - mu[k % ORC_F]) / sd[k % ORC_F];
    orc_mlp_forward(prm, n, z, lc, NULL, NULL);
    int64_t nacc = 0;
    if (trace) trace[0] = cur_score;
    for (int64_t t = 1; t <= iters; ++t) {
        int pa, pb, a, b;
        orc_learned_pair(seed, chain, n, (uint64_t)t, lc, cur, eps, &pa, &pb);
        node_of_positions(cur, pa, pb, &a, &b);
        memcpy(prop, cur, sizeof(int32_t) * (size_t)n);
        prop[pa] = cur[pb];
        prop[pb] = cur[pa];
        double pl, pm;
        orc_score_order(table, n, K, prop, round_f32, &pl, &pm, g, nl, nb, ns);
        orc_features(n, prop, nb, ns, prior_nats, stats, f);
        for (int k = 0; k < n * ORC_F; ++k) z[k] = (f[k] - mu[k % ORC_F]) / sd[k % ORC_F];
        orc_mlp_forward(prm, n, z, lp, NULL, NULL);
        double new_score = target == 0 ? pl : pm;
        double ratio = new_score - cur_score + orc_pair_logq(lp, n, a, b, eps) - orc_pair_logq(lc, n, a, b, eps);
        double u = orc_accept_uniform(seed, chain, (uint64_t)t);
        int ok = log(u) < ratio;
        if (ok) {
            memcpy(cur, prop, sizeof(int32_t) * (size_t)n);
            memcpy(lc, lp, sizeof(double) * (size_t)n);
            cur_score = new_score;
            ++nacc;
            if (pm > *best_score) {
                *best_score = pm;
                memcpy(best_graph, g, sizeof(uint64_t) * (size_t)n);
            }
            if (topk > 0) orc_topk_offer(n, topk, top_graphs, top_scores, top_count, g, pm);
        }
        if (acc) acc[t - 1] = (uint8_t)ok;
        if (trace) trace[t] = cur_score;
    }
    memcpy(order_out, cur, sizeof(int32_t) * (size_t)n);
    *accepted = nacc;
    free(cur);
    free(prop);
    free(g);
}
