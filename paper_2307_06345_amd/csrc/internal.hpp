// Host-side launchers of the octree-build kernels (internal to libcstone).
#pragma once

#include "common.hpp"

namespace cs {

// keys.hip
cstone_status launch_keys(const double* x, const double* y, const double* z, size_t n, const cstone_box& box,
                          cstone_curve curve, uint64_t* keys, uint32_t* flags, hipStream_t stream);

// sort.hip — stable LSD radix sort of 64-bit keys (63 or 64 significant bits)
// with an optional uint32 permutation; sig_bits selects how many low bits are
// sorted on.
size_t sort_workspace_bytes(size_t n, bool with_perm);
cstone_status launch_sort(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n,
                          int sig_bits, void* ws, size_t ws_bytes, hipStream_t stream);

// rebalance.hip
cstone_status launch_node_counts(const uint64_t* sorted_keys, size_t n, const uint64_t* leaves, size_t n_leaves,
                                 uint32_t* counts, hipStream_t stream);
size_t rebalance_workspace_bytes(size_t leaf_capacity);
cstone_status run_rebalance(const uint64_t* sorted_keys, size_t n, uint32_t n_crit, uint64_t* leaves,
                            size_t* n_leaves, size_t leaf_capacity, uint32_t* counts, uint32_t max_iters,
                            uint32_t* iters_done, void* ws, size_t ws_bytes, hipStream_t stream,
                            const uint32_t* input_flags = nullptr, uint32_t* input_flags_out = nullptr);

// link.hip
size_t link_workspace_bytes(size_t n_leaves);
cstone_status launch_link(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys, uint32_t* child,
                          uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream);

}  // namespace cs
