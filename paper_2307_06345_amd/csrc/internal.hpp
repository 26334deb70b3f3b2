// Host-side launchers of the octree-build kernels (internal to libcstone).
#pragma once

#include "common.hpp"

namespace cs {

// keys.hip
// hist0: NULL, or hist_mask + 1 (<= 512) counters to which the count of
// every key's value of (key & hist_mask) is added
cstone_status launch_keys(const double* x, const double* y, const double* z, size_t n, const cstone_box& box,
                          cstone_curve curve, uint64_t* keys, uint32_t* flags, hipStream_t stream,
                          uint32_t* hist0 = nullptr, uint32_t hist_mask = 0);

// sort.hip — stable LSD radix sort of 64-bit keys (63 or 64 significant bits)
// with an optional uint32 permutation; sig_bits selects how many low bits are
// sorted on.
size_t sort_workspace_bytes(size_t n, bool with_perm);
// pass_events: NULL, or passes + 1 events recorded before the first digit pass
// and after every pass. prepared: sort_prepare() already ran on this
// workspace and the producer of the keys counted their lowest digit into
// sort_first_histogram() (*mask + 1 counters), so neither step is repeated.
cstone_status launch_sort(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n,
                          int sig_bits, void* ws, size_t ws_bytes, hipStream_t stream,
                          hipEvent_t* pass_events = nullptr, bool prepared = false);
cstone_status sort_prepare(void* ws, size_t n, bool with_perm, hipStream_t stream);
uint32_t* sort_first_histogram(void* ws, size_t n, bool with_perm, uint32_t* mask);
int sort_passes(int sig_bits);

// rebalance.hip
cstone_status launch_node_counts(const uint64_t* sorted_keys, size_t n, const uint64_t* leaves, size_t n_leaves,
                                 uint32_t* counts, hipStream_t stream);
size_t rebalance_workspace_bytes(size_t n, uint32_t n_crit, size_t leaf_capacity);

struct LoopState;

// The rebalance loop, driven from the device: rounds are enqueued ahead of
// the host's convergence check, and after every batch a finalize kernel picks
// the array of the last complete round, leaves it in `leaves` with its counts
// and publishes its leaf count in device memory, so later stages (the link)
// can be enqueued before the host has looked at anything.
class RebalanceLoop {
public:
    cstone_status begin(const uint64_t* sorted_keys, size_t n, uint32_t n_crit, uint64_t* leaves, size_t n_leaves,
                        size_t leaf_capacity, uint32_t* counts, uint32_t max_iters, void* ws, size_t ws_bytes,
                        hipStream_t stream, const uint32_t* input_flags);
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
};

cstone_status run_rebalance(const uint64_t* sorted_keys, size_t n, uint32_t n_crit, uint64_t* leaves,
                            size_t* n_leaves, size_t leaf_capacity, uint32_t* counts, uint32_t max_iters,
                            uint32_t* iters_done, void* ws, size_t ws_bytes, hipStream_t stream);

// link.hip — n_leaves_dev, if not NULL, holds the leaf count on the device
// (then n_leaves is only an upper bound used to size grids and workspace).
size_t link_workspace_bytes(size_t n_leaves);
cstone_status launch_link(const uint64_t* leaves, size_t n_leaves, const uint64_t* n_leaves_dev,
                          uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets, void* ws, size_t ws_bytes,
                          hipStream_t stream);
cstone_status launch_link_by_sort(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys, uint32_t* child,
                                  uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream);

}  // namespace cs
