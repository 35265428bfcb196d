/*
 * bnos — order-space MCMC Bayesian-network structure learning on MI355X.
 *
 * C ABI of libbnos.so.  All scores are natural logarithms.
 *
 * The method (Wang, Zhang, Qian, Yuan, "A Novel Learning Algorithm for
 * Bayesian Network and Its Efficient Implementation on GPU"):
 *   - data are complete samples of discrete variables (Sec. II);
 *   - the local score of node i with parent set pi is the Bayesian-Dirichlet
 *     marginal likelihood with structure penalty gamma^|pi| (Eq. (3), in log
 *     form Eq. (4)), here with the BDeu parameters a_ijk = ess/(q_i r_i),
 *     a_ik = ess/q_i, plus one pairwise-prior term per present edge
 *     (Sec. IV, Eq. (7)-(9)) given by the cubic of Eq. (10);
 *   - parent sets have at most K members (the size limit s of Sec. II/III.B);
 *   - an order is scored by filtering every node's candidate parent sets to
 *     those inside the node's predecessor set (Sec. III.B, Alg. 1), taking the
 *     argmax (the greedy best graph, Eq. (6)) and the log-sum-exp (the
 *     sum-over-consistent-graphs order score that Sec. III.B contrasts with
 *     Eq. (6)) in one pass;
 *   - orders are sampled by Metropolis-Hastings with two-position swaps,
 *     keeping the best graph seen (Sec. III.C).
 *
 * Conventions for every call:
 *   - Return value: BNOS_OK (0) or a negative status; bnos_last_error() then
 *     gives a message (thread-local, valid until the next call on the thread).
 *   - Arguments are validated before any device work; on a validation error
 *     nothing is written.
 *   - Node ids are 0..n-1 with n <= 64; a parent set is a uint64 bit mask of
 *     node ids.  An order is int32[n] mapping position -> node id.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Handles are not thread-safe; distinct handles are independent.
 */
#ifndef BNOS_H
#define BNOS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bnos_status;
#define BNOS_OK        0
#define BNOS_E_INVALID (-1)   /* NULL pointer, non-permutation order, state >= arity, ess <= 0, NaN prior */
#define BNOS_E_RANGE   (-2)   /* n outside [1,64], K outside [0, min(n-1, 6)], arity outside [1,255],
                                 q_i * r_i above 16384, N above 2^31 - 1, B outside [1, 2^20] */
#define BNOS_E_NOMEM   (-3)   /* host or device allocation failed */
#define BNOS_E_DEVICE  (-4)   /* a HIP runtime call failed; the message names it */
#define BNOS_E_STATE   (-5)   /* handle is NULL or already freed */

const char *bnos_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int32_t bnos_version(void);

typedef struct bnos_table_s *bnos_table;

typedef struct {
    double log_gamma;      /* ln(gamma), the per-parent structure penalty of Eq. (3); default 0 */
    int32_t prior_mode;    /* 0: prior entries are weights w in [-1,1], R = (1 + w)/2;
                              1: prior entries are the paper's R in [0,1] (Sec. IV).
                              Either way the added term is ln(10) * 100 * (R - 0.5)^3. */
    int32_t chunk_steps;   /* scoring blocks stream chunk_steps * 1024 entries of one node's row (a
                              chunk: every chunks-th 1024-entry step of the row, chunks = padded
                              row / chunk length); a power of two <= 16 (rows are then padded to
                              a multiple of at least that many steps), or 0 = automatic */
    int32_t count_mode;    /* 0: one joint histogram per node subset U (|U| <= K+1) serves the |U|
                              families (i, U \ {i}); 1: one histogram per family.  Same table, bit
                              for bit; 0 counts about (K+1) times fewer samples.  (0 falls back to 1
                              when the lnGamma lookup of the build would exceed 256 MB.) */
    int32_t data_on_device; /* 0: data is a host array; 1: data is a DEVICE pointer (int8 [N][n],
                              row-major, ready on `stream`); its states are then checked on the
                              device, and an out-of-range state is BNOS_E_INVALID as for host data */
    int32_t reserved[4];   /* must be zero */
} bnos_build_opts;         /* all-zero = defaults */

/*
 * Build the local-score table of one dataset on the device (Sec. III.A:
 * every (node, parent set) scored once, before sampling).
 *   data       host int8 [N][n], row-major, data[t*n + v] in [0, arities[v]).
 *   N          number of samples, 0 <= N <= 2^31 - 1 (N = 0 is allowed).
 *   n          number of nodes, 1..64.
 *   arities    host int32 [n], each 1..255.
 *   K          max parents, 0..min(n-1, 6).
 *   ess        BDeu equivalent sample size, > 0 and finite.
 *   prior      host float [n][n] or NULL; entry [i*n + m] is the confidence in
 *              the edge m -> i (row = child, column = parent); the diagonal is
 *              ignored; see bnos_build_opts.prior_mode.
 *   opts       NULL for defaults.
 *   stream     stream for the build kernels; the call returns after the build
 *              has completed on it.
 *   out        receives the handle; free with bnos_table_free.
 * The library copies what it needs and keeps no caller pointer.
 * Memory cap: if the environment variable BNOS_MAX_DEVICE_BYTES holds a positive
 * integer, a build whose table would hold more device bytes than that (the
 * bnos_table_info figure, before any scoring workspace) returns BNOS_E_NOMEM
 * with a message, before it touches the device.
 * Table layout (device): for node i, entries e = 0..S-1 with
 * S = sum_{j<=K} C(n-1, j) hold (uint64 parent mask, float score); the
 * entries are the parent sets of size <= K over the other n-1 nodes, listed
 * in ascending order of their mask with node i's bit removed.
 */
bnos_status bnos_build_score_table(const int8_t *data, int64_t N, int32_t n,
                                   const int32_t *arities, int32_t K, double ess,
                                   const float *prior, const bnos_build_opts *opts,
                                   void *stream, bnos_table *out);

/* Frees the table's device memory (synchronises the device first).  NULL is a no-op. */
void bnos_table_free(bnos_table t);

/*
 * Shape of a table: n, K, S = entries per node (before padding), and the
 * device bytes the table holds.  Any output pointer may be NULL.
 */
bnos_status bnos_table_info(bnos_table t, int32_t *n, int32_t *K, int64_t *entries_per_node,
                            int64_t *device_bytes);

/*
 * Autotuner: times scoring launches of the B orders (DEVICE int32 [B][n]) for
 * every chunk length (powers of two dividing the row padding) and every
 * number of orders per block (1, 2, 4, 8, at most B), and, when K <= 4, the
 * gather pass (each block enumerates the consistent parent sets of a node
 * with a given top member and reads only their scores, at their ranks in the
 * row: Alg. 2's traversal on the dense table), `reps` launches each after one
 * warm-up, and keeps the fastest for this table and batch size (batch sizes
 * are bucketed as 1, 2-3, 4-7, 8-15, 16+).  Outputs (may be NULL): the chosen
 * chunk steps and orders per block of the streaming pass, whether the gather
 * pass won (1) or not (0), and the mean time per launch in ms.  Both passes and
 * every shape give the same argmax parent sets; log-sum-exp values move in the
 * last bits with the order of the partial sums.  Synchronous on `stream`.
 */
bnos_status bnos_table_autotune(bnos_table t, const int32_t *orders, int32_t B, int32_t reps, void *stream,
                                int32_t *chunk_steps, int32_t *orders_per_block, int32_t *gather,
                                double *ms_per_launch);

/*
 * Fix the launch of scoring batches of B orders (B's bucket, as above):
 * gather = 1 selects the gather pass (needs K <= 4); otherwise the streaming
 * pass with chunk_steps (0 = the build's choice) and orders_per_block (1, 2,
 * 4 or 8; 0 = the default rule).  Waits for launches in flight.
 */
bnos_status bnos_table_set_launch(bnos_table t, int32_t B, int32_t gather, int32_t chunk_steps,
                                  int32_t orders_per_block);

/*
 * Copy node `node`'s entries to host arrays masks[S], scores[S] (S from
 * bnos_table_info; cap = capacity of both arrays in entries, must be >= S).
 * Entry order as described at bnos_build_score_table.  Synchronous.
 */
bnos_status bnos_table_export(bnos_table t, int32_t node, uint64_t *masks, float *scores,
                              int64_t cap);

/*
 * The per-node static features of the learned proposal, host double [n][5]:
 * sum of the node's prior terms as child (row), as parent (column), and the
 * max, mean and population standard deviation of its stored scores.  Sync.
 */
bnos_status bnos_table_node_features(bnos_table t, double *out);

/*
 * Contingency counts N_ijk on the device for Q queries (node[q], parent
 * mask[q]), with the counting code the table's build used: for count_mode 0
 * (the default) the joint histogram of the node subset U = parents + node,
 * read out as the family's cells; for count_mode 1 (or when the build fell
 * back to it) the per-family histogram.
 *   nodes, masks   host arrays [Q]; masks must not contain the query's node
 *                  and hold at most K members.
 *   counts         host uint32 array with cap entries; query q's cells start
 *                  at offset sum_{q'<q} cells(q'), cells = q_i * r_i.
 * Cell layout: the parent ids ascending m1 < ... < md give the configuration
 * k = ((x_m1 * r_m2 + x_m2) * r_m3 + ...), lowest id most significant; the
 * cell of (k, child state j) is k * r_i + j.  Synchronous.
 */
bnos_status bnos_counts(bnos_table t, int32_t Q, const int32_t *nodes, const uint64_t *masks,
                        uint32_t *counts, int64_t cap);

/*
 * Score B orders in one pass over the table (Alg. 1 scoring loop; Eq. (6)).
 * All arrays are DEVICE pointers; the call is asynchronous on `stream`, and
 * reads its inputs until the stream reaches it.
 *   orders       int32 [B][n], position -> node id.
 *   lse          double [B]: sum_i ln sum_{pi consistent} exp s(i,pi).
 *   maxs         double [B]: sum_i max_{pi consistent} s(i,pi)  (Eq. (6)).
 *   best         uint64 [B][n]: greedy best parent set of each node (by node
 *                id); the argmax takes the larger FP32 score, on equal scores
 *                the smaller mask.
 *   node_lse     double [B][n] or NULL: per-node log-sum-exp.
 *   node_second  float [B][n] or NULL: best score among the node's other
 *                consistent sets (-inf if the empty set is the only one).
 * An order that is not a permutation of 0..n-1 yields lse = maxs = NaN and
 * best = 0 for that order; other orders are unaffected.
 * The table owns the scoring workspace (the chunk partials), grown on demand
 * with a device synchronisation: scoring calls on one table that may overlap
 * (different streams, or host threads) race and must be serialised by the
 * caller.
 */
bnos_status bnos_score_orders(bnos_table t, const int32_t *orders, int32_t B, double *lse,
                              double *maxs, uint64_t *best, double *node_lse,
                              float *node_second, void *stream);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * scoring as bnos_score_orders (same arguments, kernels and results, bit for
 * bit), with the chunk partials and the per-(order, node) score-bound cuts
 * in a fixed device array of 16 MiB that the library holds on each GPU it
 * runs on until the process ends, instead of the table's workspace.  It never
 * calls hipMalloc or hipFree; the first call on a device only looks up that
 * array's address (make it before any capture).
 * Limit: B orders need B * n * slots * 24 bytes (rounded up to 256) plus
 * B * n * 4, slots = the launch's chunks per row (n for the gather pass);
 * above 16 MiB the call returns BNOS_E_RANGE before any device work (at
 * n = 60, K = 4, in the default shape for 8+ orders, 30 chunks per row: up to
 * 386 orders in one call).  Every call on a GPU, for any table, uses that GPU's one array:
 * calls that may overlap on one GPU (streams, host threads) race and must be
 * serialised by the caller.  Nothing needs clearing between calls.
 */
bnos_status bnos_score_orders_noalloc(bnos_table t, const int32_t *orders, int32_t B, double *lse,
                                      double *maxs, uint64_t *best, double *node_lse, float *node_second,
                                      void *stream);

/*
 * Host-pointer convenience for one order; synchronous on the null stream.
 * order int32[n]; best_parents uint64[n] (may be NULL).  A non-permutation
 * order is rejected with BNOS_E_INVALID.
 */
bnos_status bnos_score_order(bnos_table t, const int32_t *order, double *lse, double *maxs,
                             uint64_t *best_parents);

/*
 * Learned swap proposal: a network that scores every node of an order; the
 * pair of nodes whose positions are swapped is drawn from
 *   q({a,b}) = (1 - eps) p_a p_b (1/(1 - p_a) + 1/(1 - p_b)) + eps * 2/(n(n-1)),
 * p = softmax of the node scores, and the MH test uses q in both directions,
 * so the chains still sample the posterior over orders (Sec. III.C's
 * acceptance rule with the Metropolis-Hastings proposal ratio).
 *
 * Per-node features (8), raw, in this order: position / n; best consistent
 * local score; best minus second best (0 if the empty set is the only
 * candidate); sum of the node's prior terms as child (row); as parent
 * (column); max, mean and standard deviation of the node's local scores.
 * The network z-scores them with (mu, sd), then computes
 *   h1 = relu(W1 z + b1), h2 = relu(W2 h1 + b2), logit = w3 . h2 + b3,
 * W1 128x8, W2 128x128.  Flat parameter layout (17,793 floats):
 *   W1 [128][8], b1 [128], W2 [128][128], b2 [128], w3 [128], b3 [1].
 * The device keeps FP32 master weights; W1, W2, w3 and the activations enter
 * the matrix cores in BF16 (round to nearest even) with FP32 accumulation.
 */
typedef struct bnos_mlp_s *bnos_mlp;

/* New network on the current device: all parameters 0, mu = 0, sd = 1. */
bnos_status bnos_mlp_create(bnos_mlp *out);
void bnos_mlp_free(bnos_mlp m);

/* Host arrays; params [17793] or NULL (keep), mu/sd [8] or NULL (keep).
 * Setting parameters resets the optimiser state.  Synchronous. */
bnos_status bnos_mlp_set_params(bnos_mlp m, const float *params, const float *mu, const float *sd);
bnos_status bnos_mlp_get_params(bnos_mlp m, float *params, float *mu, float *sd);

/* mu, sd := per-feature mean and population standard deviation of the rows
 * of feats (DEVICE float [rows][8], 16-byte aligned); an sd below 1e-6
 * becomes 1.  Async. */
bnos_status bnos_mlp_fit_norm(bnos_mlp m, const float *feats, int64_t rows, void *stream);

/* logits (DEVICE float [R][n]) of R samples of n nodes (DEVICE float [R][n][8]
 * raw features); 2 <= n <= 64.  Async. */
bnos_status bnos_mlp_forward(bnos_mlp m, const float *feats, int32_t R, int32_t n, float *logits, void *stream);

/* Mean over R samples of -ln q(pair | sample) and its gradient (DEVICE float
 * [17793], flat layout) w.r.t. the FP32 parameters; pairs DEVICE int32 [R][2]
 * node ids (a != b); loss DEVICE double [1] or NULL.  Synchronous. */
bnos_status bnos_mlp_grad(bnos_mlp m, const float *feats, const int32_t *pairs, int32_t R, int32_t n, float eps,
                          float *grad, double *loss, void *stream);

/* Adam (beta1 0.9, beta2 0.999, 1e-8) on the mean loss over minibatches of
 * `batch` samples, `epochs` passes over the count samples, each epoch in a
 * seeded pseudo-random order; loss_trace DEVICE float [steps] or NULL.
 * Synchronous. */
bnos_status bnos_mlp_train(bnos_mlp m, const float *feats, const int32_t *pairs, int64_t count, int32_t n,
                           float eps, int32_t epochs, int32_t batch, float lr, uint64_t seed, float *loss_trace,
                           void *stream);

/*
 * Metropolis-Hastings over orders (Sec. III.C), many chains at once.
 *
 * Iteration t = 0 adopts each chain's initial order (a uniform permutation:
 * Fisher-Yates from the identity with j drawn for p = n-1..1).  Every
 * iteration t >= 1 swaps two distinct positions drawn uniformly, scores the
 * new order on the table, and accepts iff ln u < new - old (u uniform in
 * (0,1)); the best-graph record starts from the initial order's greedy graph
 * and is replaced, after an accepted move, when the new order's max score
 * (Eq. (6)) is strictly larger.  All C proposals of an iteration are scored
 * in one pass over the table; sweep_len iterations are captured in one HIP
 * graph and replayed.
 *
 * Random numbers: one 64-bit draw per (seed, chain, purpose, step) from the
 * SplitMix64 finalizer mix(z) (Steele, Lea & Flood 2014):
 *   key = mix(seed ^ mix(chain*8 + purpose + 1)),
 *   draw = mix(key + (step+1) * 0x9E3779B97F4A7C15);
 * purposes 0 = initial shuffle (step = p), 1/2 = first/second swap position,
 * 3 = acceptance uniform; integers in [0,m) are ((draw >> 32) * m) >> 32; the
 * second position y in [0,n-1) is shifted past the first (y >= x -> y+1);
 * u = ((draw >> 11) + 0.5) * 2^-53.  The chain id is chain_offset + c.
 */
typedef struct {
    int32_t chains;           /* C, 1..65536 */
    int32_t target;           /* 0: log-sum-exp order score; 1: max order score (Eq. (6)) */
    int64_t iterations;       /* MH iterations to run in this call, >= 0 */
    int64_t first_iteration;  /* 0: fresh start; k > 0: resume, the state holds the chains after
                                 iteration k and this call runs k+1 .. k+iterations */
    uint64_t seed;
    int64_t chain_offset;     /* chain c draws from RNG stream chain_offset + c */
    int32_t trace_every;      /* >= 1; trace entry j is the score after iteration
                                 first_iteration + j*trace_every, j = 0..iterations/trace_every */
    int32_t sweep_len;        /* iterations per captured graph; 0 = 32 */
    int32_t proposal;         /* 0: uniform swap of two positions; 1: learned (needs mlp) */
    float eps;                /* learned: weight of the uniform pair in q, (0, 1]; 0 means 0.5 */
    struct bnos_mlp_s *mlp;   /* learned: the network (see bnos_mlp_*), read during the call */
    int32_t topk;             /* 0..64: keep each chain's topk best distinct graphs (Sec. III.C keeps a
                                 number of best graphs); 0 = off */
    int32_t trace_edges;      /* 0..32: edges traced per chain (state.edge_trace), for mixing diagnostics */
    const int32_t *edges;     /* HOST [trace_edges][2] (child, parent) node ids, read during the call */
    int32_t reserved[2];      /* must be zero */
} bnos_chain_cfg;

typedef struct {              /* DEVICE pointers; the chain state, read when resuming, written always */
    int32_t *orders;          /* [C][n] current order of each chain */
    double *scores;           /* [C] target score of the current order */
    uint64_t *best_graphs;    /* [C][n] best graph seen: parent mask per node id */
    double *best_scores;      /* [C] max score (Eq. (6)) of the best graph's order */
    int64_t *accepted;        /* [C] accepted moves since iteration 0 */
    double *trace;            /* [C][iterations/trace_every + 1] or NULL */
    uint8_t *accept_flags;    /* [C][iterations] or NULL: move of iteration first_iteration+1+k accepted */
    /* Harvest of accepted moves (all NULL / 0 = off): chain c stores its k-th
       accepted move, k < harvest_cap, as the raw features [n][8] of the order
       before the move (see the learned proposal above) and the swapped node
       pair; harvest_count[c] counts the stored moves (in/out). */
    float *harvest_feats;     /* [C][harvest_cap][n][8] */
    int32_t *harvest_pairs;   /* [C][harvest_cap][2] node ids */
    int64_t *harvest_count;   /* [C] */
    int64_t harvest_cap;
    /* Record of the best distinct graphs (cfg.topk > 0): the greedy graph of
       the initial order and of every accepted order is offered; records are
       kept in decreasing order of max score (Eq. (6)), a graph already recorded
       is not added again, among equal scores the earlier record stays ahead,
       and when the record is full a graph enters only with a score strictly
       above the last, which drops out.  A fresh start empties the record; a
       resumed call continues the one in the state.  Entry 0 is best_graphs. */
    uint64_t *top_graphs;     /* [C][topk][n] */
    double *top_scores;       /* [C][topk] */
    int32_t *top_count;       /* [C] records held (in/out) */
    /* cfg.trace_edges > 0: bit e of edge_trace[c][j] tells whether edge e of
       cfg.edges (parent -> child) is in the greedy graph of chain c's current
       order after iteration first_iteration + j*trace_every (j = 0: the
       starting order), for effective-sample-size estimates of edge indicators. */
    uint32_t *edge_trace;     /* [C][iterations/trace_every + 1] */
} bnos_chain_state;

/*
 * Run cfg->iterations MH iterations of C chains on `stream` and return when
 * they have completed.  The library allocates a per-call workspace
 * (proposal orders and scores, plus the table's scoring partials for C
 * orders) and frees the per-call part before returning.
 */
bnos_status bnos_run_chains(bnos_table t, const bnos_chain_cfg *cfg, bnos_chain_state *state,
                            void *stream);

/*
 * The same for T datasets of possibly different n at once: every kernel of an
 * iteration spans all T tables (one grid over all tables' (node, chunk)
 * blocks, one block per chain of every table).  tables[k] gets
 * cfg->chains chains whose RNG stream ids are chain_offset + k*chains + c,
 * and its own state states[k] (sized by tables[k]'s n).  Each chain's
 * trajectory is the one bnos_run_chains gives it with that chain id.
 * T is 1..4096; a table may appear once.  With the score bound on, the
 * per-iteration launch that lists each node's chains also holds one
 * wavefront per (chain, node) pair; a call whose pairs (summed over the
 * tables) exceed that launch's 2^32 work-items returns BNOS_E_RANGE before
 * any kernel runs.
 */
bnos_status bnos_run_chains_multi(const bnos_table *tables, int32_t T, const bnos_chain_cfg *cfg,
                                  bnos_chain_state *states, void *stream);

/*
 * Chain-sweep autotuner (Sec. III.C's iterations, batched): times
 * cfg->iterations iterations of cfg->chains chains on this table -- the real
 * sweep: window work lists, the window nodes' scoring pass, the merge and MH
 * decision -- for every chunk length (powers of two dividing the row padding)
 * and every number of chains per scoring block (1, 2, 4, 8, at most C),
 * `reps` timed runs each after one warm-up, and keeps the fastest for this
 * table and the chain count's bucket (1, 2-3, 4-7, 8-15, 16+).  Later sweeps
 * of that many chains on this table (bnos_run_chains, and bnos_run_chains_multi
 * where it is the first table: the chains per block are per launch) use it.
 * With cfg->first_iteration > 0 every timed run resumes from a copy of `state`
 * (orders, scores, best_graphs, best_scores, accepted; e.g. burned-in chains);
 * with 0 they start fresh from cfg->seed and state may be NULL.  The caller's
 * state is never written.  cfg->iterations in [1, 2^20], reps in [1, 100].
 * Outputs (may be NULL): the chosen chunk steps, chains per block, and the
 * device time per iteration in ms.  A shape changes the association of the
 * FP32 log-sum-exp partial sums, not the argmax.  Synchronous.
 */
bnos_status bnos_chains_autotune(bnos_table t, const bnos_chain_cfg *cfg, const bnos_chain_state *state,
                                 int32_t reps, void *stream, int32_t *chunk_steps, int32_t *orders_per_block,
                                 double *ms_per_iteration);

/*
 * Fix the chain-sweep launch for `chains` chains (their bucket, as above):
 * chunk_steps a power of two dividing the row padding or 0 (the scoring
 * shape of a batch of that many orders), orders_per_block 1, 2, 4, 8 or 0
 * (the default rule).  Waits for work in flight.
 */
bnos_status bnos_chains_set_launch(bnos_table t, int32_t chains, int32_t chunk_steps, int32_t orders_per_block);

/*
 * Kernel timing for measurement: while enabled (enable = k >= 1), every k-th
 * order-scoring launch of this table (bnos_score_orders / bnos_score_order),
 * starting with the first, carries a pair of HIP events that take the
 * streaming kernel's own start and end on the launch stream
 * (hipExtLaunchKernel); 0 disables, negative values are E_RANGE.  (A launch
 * with events costs the host about 15 us more than one without: for short
 * launches, sample with k > 1 so that the timed loop is not host-bound.)  bnos_table_timing_read waits for them and
 * returns the sum of the streaming kernels' durations (ms), the number of
 * launches and the number of passes over the table those launches made (a
 * launch scoring B orders streams the table once per group of orders per
 * block) since the last enable, then keeps counting.  Any output pointer may
 * be NULL.  The events form a ring of 256 pairs created by the enable call;
 * when 256 timed launches are pending, the next one first waits for the
 * oldest and adds it to the totals.
 */
bnos_status bnos_table_timing(bnos_table t, int32_t enable);

/*
 * Tile skipping (on by default): the table keeps, for every 256-entry tile
 * and every 64-entry sub-tile, the AND of its masks; a (sub-)tile whose AND
 * contains a node outside an order's predecessor set holds no consistent
 * entry for that order.  A tile no order of a scoring block needs is skipped
 * by the block, and a block scoring one order does not fetch the sub-tiles of
 * its tiles that the order cannot use.  Results are identical with it off.
 * bnos_table_count_tiles (measurement) returns how many 64-entry sub-tiles a
 * scoring launch of these B orders (DEVICE int32 [B][n]) reads with tile
 * skipping, and the sub-tiles of one full pass (n * padded entries / 64).
 * Such a launch also reads every tile summary of each pass (8 B per 256
 * entries) and, with one order per block, every sub-tile summary (8 B per 64
 * entries).  Synchronous.
 */
bnos_status bnos_table_tile_skip(bnos_table t, int32_t enable);

/*
 * Score bound (on by default; acts with tile skipping on): every scoring block
 * (order scoring and chain sweeps) first bounds from below, for each of its
 * orders, the best and the second-best score among the entries of its node
 * that the order can use
 * (Sec. III.B, Eq. (3)-(6)), from entries it can locate without a search: the
 * empty set, the singletons of the node's predecessors, and up to 192 top
 * entries of the row listed at build (sets of two or more members).  It then
 * skips every tile whose largest score (kept per 256-entry tile at build) lies
 * below the second-best bound and 60 nats below the best bound.  Such a tile
 * holds neither the argmax nor the second best, and every one of its terms in
 * the node's log-sum-exp is below e^-60 times the largest term, so the sum
 * changes by less than 2^-60 of itself at n <= 64 (far below FP32 rounding):
 * the max score, the best parent sets and the second best are unchanged, and
 * the log-sum-exp is the same up to that bound (bitwise, in every case tested).
 * A block of several orders reads a tile if any of its orders needs it, and
 * each order folds only the tiles it needs.
 */
bnos_status bnos_table_score_bound(bnos_table t, int32_t enable);

/*
 * Computed masks (on by default): a scoring launch of one order per block
 * does not read the stored masks.  The table keeps, for every 4 entries of a
 * row, the first entry's mask over the node's n - 1 other nodes; the scoring
 * block steps to the next masks itself (a row lists every such mask with at
 * most K members in ascending order), so it reads 6 bytes per entry instead
 * of 12.  Results are bitwise identical with it off.  Launches of several
 * orders per block and chain sweeps always read the stored masks.
 */
bnos_status bnos_table_computed_masks(bnos_table t, int32_t enable);
bnos_status bnos_table_count_tiles(bnos_table t, const int32_t *orders, int32_t B, int64_t *tiles_read,
                                   int64_t *tiles_per_pass);
bnos_status bnos_table_timing_read(bnos_table t, double *total_ms, int64_t *launches,
                                   int64_t *table_passes);

#ifdef __cplusplus
}
#endif

#endif /* BNOS_H */
