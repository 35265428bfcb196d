// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "bnos.h"

namespace bnos {

// Largest contingency table (q_i * r_i cells) a build supports; the counting
// kernel keeps one such histogram per wavefront in LDS.
constexpr int kMaxCells = 16384;
constexpr int kMaxK = 6;

// Order-scoring geometry: 256 threads, 4 entries per thread per step, so a
// block consumes 1024 entries per step; a chunk is 1..16 steps, taken from a
// node's row at a stride of `chunks` steps (chunk c: steps c, c + chunks, ...).
constexpr int kScoreThreads = 256;
constexpr int kEntriesPerStep = 1024;
constexpr int kMaxStepsPerChunk = 16;

// Place of the summaries (tile AND, sub-tile ANDs, tile maximum) of tile w of
// step s of a row inside that row's summary arrays.  The row's steps form C
// chunks of the longest chunk length P (the row padding), chunk c holding steps
// c, c + C, c + 2C, ... as the scoring blocks take them; a chunk's summaries are
// stored together (its i-th step's tile w at (c P + i) 4 + w), so the blocks of
// that launch shape read theirs from one run of memory.  A permutation of the
// row's tiles: only where the summaries sit changes, not what they hold.
__host__ __device__ inline int64_t summary_pos(int64_t s, int w, int64_t C, int P)
{
    return ((s % C) * P + s / C) * 4 + w;
}

// Score bound of the streaming pass: a block first takes, for each of its
// orders, lower bounds on the best and the second-best consistent entry of its
// node from entries it knows the order can use (the empty set, the singletons
// of the predecessors, and kBoundCands listed top entries of the row with two
// or more members), then leaves out for that order every tile whose largest
// score is below both the second-best bound and the best bound minus
// kBoundGap nats.  Such a tile holds neither the argmax nor the second best,
// and each of its terms is below e^-60 of the largest term of the node's sum.
constexpr int kBoundCands = 192;
constexpr int kBoundSlots = 64 + kBoundCands;   // per node: slot s < 63 {slot s}, 63 the empty set, then the list
constexpr float kBoundGap = 60.0f;

// Partial-reduction record written by each scoring block (one per order).
struct Partial {
    float m, s;          // running max and sum of exp(x - m) over consistent entries
    float best, second;  // top-1 score and best score among the others
    uint64_t bmask;      // mask of the top-1 entry
};

struct TableT {
    uint32_t magic = 0;
    int n = 0, K = 0;
    int64_t N = 0, N_pad = 0;
    int64_t S = 0, S_pad = 0;       // entries per node before / after padding
    int chunk_entries = 0;          // entries per scoring block
    int chunks = 0;                 // scoring blocks per node = S_pad / chunk_entries
    int pad_steps = 1;              // rows are padded to a multiple of pad_steps * 1024 entries
    int max_cells = 0;
    int count_mode = 0;             // counting code the build used: 0 joint histograms, 1 per family
    double ess = 1.0, log_gamma = 0.0;
    int device = 0;

    uint8_t *d_data = nullptr;      // column-major [n][N_pad]
    int32_t *d_ar = nullptr;        // [n]
    double *d_prior = nullptr;      // [n][n] prior term in nats (0 where none)
    int64_t *d_nsets = nullptr;     // [64][8] number of masks over `bit` bits with <= k members
    uint64_t *d_masks = nullptr;    // [n][S_pad]
    float *d_scores = nullptr;      // [n][S_pad]
    double *d_nstat = nullptr;      // [n][5]: prior row sum, prior column sum, max, mean, sd of the row
    uint64_t *d_tand = nullptr;     // [n * S_pad / 256]: AND of the masks of each 256-entry tile
    uint64_t *d_tsub = nullptr;     // [n * S_pad / 64]: AND of the masks of each 64-entry sub-tile
    bool tile_skip = true;
    uint64_t *d_anchor = nullptr;   // [n * S_pad / 4]: slot-space mask of every 4th entry
    bool computed_masks = true;     // one-order blocks compute masks from the anchors
    float *d_tmax = nullptr;        // [n * S_pad / 256]: largest score of each tile
    uint64_t *d_cmask = nullptr;    // [n][kBoundSlots]: bound candidates (node-space mask; ~0 for none)
    float *d_cscore = nullptr;      // [n][kBoundSlots]: their scores (-inf for none)
    bool score_bound = true;        // one-order blocks skip tiles by the score bound

    // order-scoring workspace: per (order, node, chunk) partial reductions
    void *d_part = nullptr;
    int64_t part_bytes = 0;         // capacity in bytes

    // kernel timing: a ring of kEventRing event pairs, created when timing is
    // first enabled; launches in flight occupy ev_count slots from ev_head on
    static constexpr size_t kEventRing = 256;
    bool timing = false;
    int timing_every = 1;           // every timing_every-th launch carries events
    int64_t timing_seen = 0;        // scoring launches since timing was enabled
    std::vector<hipEvent_t> ev_start, ev_stop;
    size_t ev_head = 0, ev_count = 0;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
    std::vector<int64_t> ev_passes;     // table passes of the launch in each slot
    int64_t timed_passes = 0;

    // autotuned per batch-size bucket (1, 2-3, 4-7, 8-15, 16+); 0 = default
    int tuned_bt[5] = {0, 0, 0, 0, 0};   // orders per scoring block
    int tuned_cs[5] = {0, 0, 0, 0, 0};   // chunk length in 1024-entry steps
    int tuned_gather[5] = {0, 0, 0, 0, 0};   // 1: score by enumerating the consistent sets (K <= 4)

    int64_t device_bytes() const;
    static int bucket(int B) { return B >= 16 ? 4 : (B >= 8 ? 3 : (B >= 4 ? 2 : (B >= 2 ? 1 : 0))); }
    // Chunk length (entries) and chunks per node used for a launch of B orders:
    // the autotuned length of B's bucket; else for 8+ orders the longest chunk
    // (a block's fixed cost -- tile summaries, predecessor masks, the per-order
    // reductions -- is then spread over the most entries, and the orders
    // already fill the grid); else the length chosen at build time.
    int chunk_entries_for(int B) const
    {
        const int cs = tuned_cs[bucket(B)];
        if (cs > 0) return cs * 1024;
        return B >= 8 ? pad_steps * 1024 : chunk_entries;
    }
    int chunks_for(int B) const { return (int)(S_pad / chunk_entries_for(B)); }
    // Chain sweeps of C chains have their own launch shape (bnos_chains_autotune /
    // bnos_chains_set_launch) per chain-count bucket; 0 = the scoring shape of a
    // batch of C orders, except that the orders per block follow pick_bt.
    int chain_bt[5] = {0, 0, 0, 0, 0};
    int chain_cs[5] = {0, 0, 0, 0, 0};
    int chain_chunk_entries_for(int C) const
    {
        const int cs = chain_cs[bucket(C)];
        return cs > 0 ? cs * 1024 : chunk_entries_for(C);
    }
    int chain_chunks_for(int C) const { return (int)(S_pad / chain_chunk_entries_for(C)); }
    // partials of one launch: [B][chunks][n], with n slots per order in gather mode; a chain
    // sweep of B chains writes [B][chain chunks][n]
    int64_t partial_bytes_for(int B) const
    {
        int c = chunks_for(B) > n ? chunks_for(B) : n;
        if (chain_chunks_for(B) > c) c = chain_chunks_for(B);
        return (int64_t)B * n * c * (int64_t)sizeof(Partial);
    }
    // the partials, then (256-byte aligned) each order's score-bound cut per node
    int64_t cuts_offset_for(int B) const { return (partial_bytes_for(B) + 255) & ~(int64_t)255; }
    int64_t workspace_bytes_for(int B) const { return cuts_offset_for(B) + (int64_t)B * n * (int64_t)sizeof(float); }
    bool gather_for(int B) const { return K <= 4 && tuned_gather[bucket(B)] != 0; }
};

constexpr uint32_t kMagic = 0xB0A5C0DEu;

void set_error(const std::string &msg);
bool handle_live(const TableT *t);
void register_handle(TableT *t);
void unregister_handle(TableT *t);


}  // namespace bnos

#define BNOS_HIP(call)                                                               \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess) {                                                      \
            bnos::set_error(std::string(#call) + ": " + hipGetErrorString(e_));     \
            return BNOS_E_DEVICE;                                                    \
        }                                                                            \
    } while (0)
