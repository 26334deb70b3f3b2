// Host-side launchers of the octree-build kernels (internal to libcstone).
#pragma once

#include "common.hpp"

namespace cs {

// keys.hip
constexpr uint32_t kKeyBlocksMax = 512;  // blocks of the plain key kernel (grid-stride beyond)
constexpr uint32_t kKeyDigitsMax = 3;    // digits the key kernel counts at most (the split sort's top digits)

// First positions of the level-6 nodes, handed from the sort to the loop's start
constexpr uint32_t kLevel6Cells = 1u << 18;
constexpr uint32_t kCellEmpty = 0xffffffffu;
// flags: NULL, or a word into which CSTONE_FLAG_NONFINITE is OR-ed.
// hist_parts: NULL, or kKeyBlocksMax rows of kKeyDigitsMax x 512 words; block b
// stores, for d < hist_digits and every value v, the count of keys with
// ((key >> (hist_shift + d * hist_bits)) & hist_mask) == v at
// [b * kKeyDigitsMax * 512 + d * 512 + v] (hist_mask = 2^hist_bits - 1).
// bad_parts: NULL, or kKeyBlocksMax words; block b stores CSTONE_FLAG_NONFINITE
// or 0. *blocks_used (if not NULL): the rows and words written.
cstone_status launch_keys(const double* x, const double* y, const double* z, size_t n, const cstone_box& box,
                          cstone_curve curve, uint64_t* keys, uint32_t* flags, hipStream_t stream,
                          uint32_t* hist_parts = nullptr, uint32_t hist_mask = 0, uint32_t hist_shift = 0,
                          uint32_t* bad_parts = nullptr, uint32_t* blocks_used = nullptr, uint32_t hist_digits = 1);

// sort.hip — stable radix sort of 64-bit keys (63 or 64 significant bits)
// with an optional uint32 permutation; sig_bits selects how many low bits are
// sorted on. Particle keys with a permutation take the split path (top two
// digits, then every bucket on its own), other sorts plain LSD passes.
size_t sort_workspace_bytes(size_t n, bool with_perm);
// pass_events: NULL, or sort_passes() + 1 events recorded before the first
// pass and after every pass (split path: after the first top pass, after the
// last one, after the bucket sort and after the low passes). prepared: the key
// kernel stored its per-block digit counts (sort_key_parts) and
// sort_setup_from_keys() ran, so no set-up or first histogram is repeated, and
// the split sort's top passes count no digits for the pass after them.
// err_word: NULL, or a caller word (cleared beforehand) into which the sort's
// kernels OR their error bits (a look-back wait that gave up, a bucket-list
// overflow), all above the public CSTONE_FLAG_* bits.
// level6: NULL, or kLevel6Cells words set to kCellEmpty by the set-up; the
// split sort stores there the first position of every non-empty level-6 node.
// variant: the sort shape (sort_variant_count() of them); -1 takes the shape
// of the autotune table for a particle-key sort of n keys (with perm, 63
// bits), else the built-in one. A prepared sort must name the shape its
// set-up used.
cstone_status launch_sort(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n,
                          int sig_bits, void* ws, size_t ws_bytes, hipStream_t stream,
                          hipEvent_t* pass_events = nullptr, bool prepared = false, int variant = -1,
                          uint32_t* err_word = nullptr, uint32_t* level6 = nullptr);
bool sort_uses_split(size_t n, int sig_bits, bool with_perm, int variant);
// clear_word: NULL, or one caller word zeroed by the same launch; variant: the
// sort shape the passes will use
cstone_status sort_prepare(void* ws, size_t n, bool with_perm, hipStream_t stream, uint32_t* clear_word,
                           int variant);
// Per-block digit counts and non-finite flags of the key kernel, in the sort
// workspace: where to store them and which digits to count (the first pass's
// digit, or for the split sort its three top digits: a histogram does not
// depend on the order of the keys, so the unsorted keys give every pass's).
void sort_key_parts(void* ws, size_t n, bool with_perm, int sig_bits, int variant, uint32_t** hist_parts,
                    uint32_t** bad_parts, uint32_t* mask, uint32_t* shift, uint32_t* digits);
// Set-up after the key kernel stored its parts (replaces sort_prepare in a
// build): the counts of the digits sort_key_parts named are the sums of the
// `parts` rows, *flag the OR of the blocks' flags, and everything sort_prepare
// clears is cleared.
cstone_status sort_setup_from_keys(void* ws, size_t n, bool with_perm, int variant, uint32_t parts, uint32_t* flag,
                                   uint32_t* level6, hipStream_t stream);
int sort_passes(size_t n, int sig_bits, bool with_perm, int variant);

// ---- batched builds: many independent sets in one pass of every stage -------

// One particle set of a batch, as the kernels see it (device copy in the
// caller's workspace). Particles of set s occupy [part_off, part_off + n) of
// the concatenated particle arrays; its leaves, counts, nodes and level
// offsets go to its own output regions.
struct BatchSet {
    double lo[3];
    double scale[3];  // 2^21 / (hi - lo), per axis
    uint32_t n;
    uint32_t curve;
    uint32_t n_crit;
    uint32_t part_off;
    uint64_t leaf_off;  // first slot of its leaves (cap + 1 slots) and counts
    uint64_t node_off;  // first slot of its node keys and child offsets
    uint64_t cap;       // leaf capacity
    uint64_t node_cap;  // cap + (cap - 1) / 7
};

// Per-set result, written on the device: leaf and node counts, rebalance
// rounds (including the final check) and a cstone_status.
struct BatchResult {
    uint32_t n_leaves, n_nodes, rounds, status;
};

// keys.hip — tiles[b] = {first particle, count, unused, set}; the lowest
// digit (key & hist_mask) is counted into hist0 + set * hist_stride.
cstone_status launch_keys_batch(const double* x, const double* y, const double* z, const uint4* tiles,
                                uint32_t n_tiles, const BatchSet* sets, uint64_t* keys, uint32_t* set_flags,
                                uint32_t* hist0, uint32_t hist_stride, uint32_t hist_mask, uint32_t hist_shift,
                                hipStream_t stream);

// sort.hip — segmented sort: tiles[b] = {first key, count, first tile of its
// set, set}, never straddling two sets; seg_base[s] = first key of set s.
// Permutation values are relative to the set's first key.
struct SortVariantInfo {
    int bits, block, items, tile, split;
};
cstone_status set_lookback_patience(uint32_t waits);
int sort_variant_count();
SortVariantInfo sort_variant_info(int variant);
int sort_builtin_variant();  // the shape used where the autotune table has no entry

// tune.hip — the autotune table: (kernel, floor(log2 n), device) -> shape
constexpr int kTuneSort = 0;       // particle-key sort of cstone_sort / cstone_build
constexpr int kTuneBatchSort = 1;  // segmented sort of a batch (n: all its keys)
constexpr int kTuneKernels = 2;
int tune_lookup(int kernel, size_t n);  // -1: no entry for the current device
void tune_record(int kernel, size_t n, int variant);
int sort_resolve_variant(size_t n);  // particle-key sort of n keys: the table's shape, else the built-in one
size_t sort_seg_workspace_bytes(size_t n_total, size_t n_tiles, uint32_t n_sets, int variant);
cstone_status sort_seg_prepare(void* ws, size_t n_total, size_t n_tiles, uint32_t n_sets, int variant,
                               hipStream_t stream);
// first-digit counters of the segmented sort (set s at + s * *stride)
uint32_t* sort_seg_first_histogram(void* ws, size_t n_total, size_t n_tiles, uint32_t n_sets, int variant,
                                   uint32_t* stride, uint32_t* mask, uint32_t* shift);
cstone_status launch_sort_segmented(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out,
                                    size_t n_total, const uint4* tiles, uint32_t n_tiles, const uint32_t* seg_base,
                                    uint32_t n_sets, size_t max_set, int sig_bits, int variant, void* ws,
                                    size_t ws_bytes, hipStream_t stream, uint32_t* err_word = nullptr);

// props.hip — particle counts of every node of a linked octree; gather of
// particle arrays by the sort permutation (separate passes, or one fused pass
// over three arrays)
// exclusive prefix sum: out[i] = in[0] + ... + in[i - 1] for i <= n (out[n]
// the total, modulo 2^32), one pass; n < 2^32 - 1
size_t scan_u32_workspace_bytes(size_t n);
cstone_status launch_scan_u32(const uint32_t* in, size_t n, uint32_t* out, void* ws, size_t ws_bytes,
                              hipStream_t stream);
size_t node_props_workspace_bytes(size_t n_leaves);
cstone_status launch_octree_node_counts(const uint64_t* leaves, const uint32_t* counts, size_t n_leaves,
                                        const uint64_t* node_keys, size_t n_nodes, uint32_t* node_counts, void* ws,
                                        size_t ws_bytes, hipStream_t stream);
cstone_status launch_gather(const double* const* src, const uint32_t* perm, size_t n, double* const* dst, int arrays,
                            bool fused, hipStream_t stream);

// global.hip — the replicated tree of sharded particles, its partition
size_t global_rebalance_workspace_bytes(size_t leaf_capacity, uint32_t n_shards);
cstone_status run_global_rebalance(const uint64_t* sorted_keys, const uint64_t* shard_off_dev, uint32_t n_shards,
                                   uint32_t n_crit, uint64_t* leaves, size_t* n_leaves, size_t leaf_capacity,
                                   uint32_t* counts, uint32_t max_iters, uint32_t* iters_done, void* ws,
                                   size_t ws_bytes, hipStream_t stream);
size_t sfc_partition_workspace_bytes(size_t n_leaves);
cstone_status launch_sfc_partition(const uint32_t* counts, size_t n_leaves, uint32_t n_ranks, uint32_t* bounds,
                                   void* ws, size_t ws_bytes, hipStream_t stream);

// radix.hip — binary radix tree (after Karras) and the octrees built on it
cstone_status launch_radix_tree(const uint64_t* keys, size_t m, uint32_t* first, uint32_t* last, uint32_t* split,
                                uint32_t* prefix_len, hipStream_t stream);
size_t radix_link_workspace_bytes(size_t n_leaves);
cstone_status launch_link_radix(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys, uint32_t* child,
                                uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream);
size_t compact_octree_workspace_bytes(size_t n_leaves);
cstone_status launch_compact_octree(const uint64_t* leaves, const uint32_t* counts, size_t n_leaves,
                                    uint64_t* node_keys, uint32_t* parent, uint32_t* level_offsets, size_t* n_nodes,
                                    void* ws, size_t ws_bytes, hipStream_t stream);

// rebalance.hip
cstone_status launch_node_counts(const uint64_t* sorted_keys, size_t n, const uint64_t* leaves, size_t n_leaves,
                                 uint32_t* counts, hipStream_t stream);
size_t rebalance_workspace_bytes(size_t n, uint32_t n_crit, size_t leaf_capacity);

constexpr int kMaxRounds = 64;
// Tiles of a round are taken in order from one counter per round (each in a
// 128-byte line of its own), so that every tile a block waits for in the
// round's look-back is held by a running block.
constexpr int kCounterWords = 32;

// Device-side loop state: the part the host reads after a batch of rounds ...
struct LoopHeader {
    uint64_t nl[kMaxRounds + 1];    // leaves entering round r (batched: entries, closing keys included)
    uint32_t changed[kMaxRounds];   // some O_i != 1 in round r
    uint32_t merged[kMaxRounds];    // some O_i == 0 in round r
    uint32_t over[kMaxRounds];      // a child of a leaf split in round r holds more than n_crit (and can split)
    uint32_t nsplit[kMaxRounds];    // split leaves listed in round r
    uint32_t err;
    uint32_t input_flags;  // copy of the caller's key-stage flag word
    uint64_t final_nl;     // set by the finalize kernel: leaves (entries) of the result array
    uint32_t final_last;   // rounds behind it
    uint32_t final_code;   // 0 running, 1 converged, 2 capacity exceeded
    uint32_t start_level;  // from the root: rounds skipped by starting at the uniform grid of this level
    uint32_t start_fine;   // the start-level search went finer than level 3
    uint32_t mins[kL + 1]; // least node count of every level (start-level search)
};

// ... and, after it and never copied to the host, the tile counters of every round.
struct LoopState : LoopHeader {
    alignas(128) uint32_t counters[kMaxRounds][kCounterWords];
};

// The rebalance loop, driven from the device: rounds are enqueued ahead of
// the host's convergence check, and after every batch a finalize kernel picks
// the array of the last complete round, leaves it in `leaves` with its counts
// and publishes its leaf count in device memory, so later stages (the link)
// can be enqueued before the host has looked at anything.
class RebalanceLoop {
public:
    cstone_status begin(const uint64_t* sorted_keys, size_t n, uint32_t n_crit, uint64_t* leaves, size_t n_leaves,
                        size_t leaf_capacity, uint32_t* counts, uint32_t max_iters, void* ws, size_t ws_bytes,
                        hipStream_t stream, const uint32_t* input_flags,
                        const uint32_t* level6 = nullptr);
    // enqueue the next batch of rounds (0: the expected number) and the finalize step
    cstone_status enqueue(uint32_t rounds = 0);
    // device word holding the leaf count of the array left in `leaves`
    const uint64_t* device_leaf_count() const;
    // copy the loop state to the host (synchronises the stream); *finished is
    // false if the loop neither converged nor failed and rounds remain
    cstone_status wait(bool* finished);

    // results after wait()
    size_t n_leaves = 0;  // leaves in `leaves` (CAPACITY: the count the failing round needed)
    uint32_t rounds = 0;  // complete rounds
    uint32_t input_flags = 0;
    cstone_status status = CSTONE_OK;

private:
    const uint64_t* P_ = nullptr;
    size_t n_ = 0;
    uint32_t n_crit_ = 0;
    uint64_t* leaves_ = nullptr;
    size_t nl0_ = 0, cap_ = 0;
    uint32_t* counts_ = nullptr;
    uint32_t max_iters_ = 0, enqueued_ = 0;
    hipStream_t stream_ = nullptr;
    void* ws_ = nullptr;
    LoopState* st_ = nullptr;
    bool root_ = false;
    int start_top_ = 0;  // > 0: the loop may start at a uniform level up to this one
};

cstone_status run_rebalance(const uint64_t* sorted_keys, size_t n, uint32_t n_crit, uint64_t* leaves,
                            size_t* n_leaves, size_t leaf_capacity, uint32_t* counts, uint32_t max_iters,
                            uint32_t* iters_done, void* ws, size_t ws_bytes, hipStream_t stream);

// Batched rebalance from the root of every set, all rounds enqueued at once
// (a round after global convergence exits at once), then per-set leaves,
// counts and results. Sets' arrays are kept back to back on the device.
size_t batch_rebalance_workspace_bytes(uint32_t n_sets, size_t entry_capacity, size_t split_capacity);
cstone_status launch_batch_rebalance(const uint64_t* P, size_t n_total, const BatchSet* sets, uint32_t n_sets,
                                     size_t entry_capacity, size_t split_capacity, uint32_t rounds,
                                     const uint32_t* set_flags, uint64_t* leaves, uint32_t* counts,
                                     BatchResult* results, void* ws, size_t ws_bytes, const uint32_t* sort_err,
                                     hipStream_t stream);
// The final back-to-back arrays, for the batched link.
struct BatchTreeView {
    const uint64_t* K[2];
    const uint32_t* sid[2];
    const uint32_t* starts[2];
    const LoopState* st;
};
BatchTreeView batch_rebalance_view(void* ws, uint32_t n_sets, size_t entry_capacity, size_t split_capacity);

// link.hip — n_leaves_dev, if not NULL, holds the leaf count on the device
// (then n_leaves is only an upper bound used to size grids and workspace).
size_t link_workspace_bytes(size_t n_leaves);
cstone_status launch_link(const uint64_t* leaves, size_t n_leaves, const uint64_t* n_leaves_dev,
                          uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets, void* ws, size_t ws_bytes,
                          hipStream_t stream);
size_t link_batch_workspace_bytes(uint32_t n_sets, size_t entry_capacity);
cstone_status launch_link_batch(const BatchTreeView& tree, const BatchSet* sets, uint32_t n_sets,
                                size_t entry_capacity, uint64_t* node_keys, uint32_t* child,
                                uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream);
// steps 3-5 of Sec. 5 from unsorted node keys: sort (keys only, 64 bits), LO
// by search, and CO (skipped if child is NULL)
cstone_status launch_link_finish(const uint64_t* unsorted, size_t n, uint64_t* node_keys, uint32_t* child,
                                 uint32_t* level_offsets, void* sort_ws, size_t sort_ws_bytes, hipStream_t stream);
cstone_status launch_link_by_sort(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys, uint32_t* child,
                                  uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream);

}  // namespace cs
