// C ABI entry points of libcstone (declared and documented in cstone.h):
// argument checks, workspace layout and the order of the stages on a stream.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

using namespace cs;

namespace {

bool box_ok(const cstone_box* b) {
    if (!b) return false;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(b->lo[d]) || !std::isfinite(b->hi[d]) || !(b->lo[d] < b->hi[d])) return false;
    return true;
}

constexpr size_t kMaxN = 0xffffffffull;  // counts, perm, CO and LO are uint32

size_t nodes_of(size_t nl) { return nl + (nl ? (nl - 1) / 7 : 0); }

__global__ void clear_word_kernel(uint32_t* w) { *w = 0; }

}  // namespace

extern "C" {

const char* cstone_status_string(cstone_status s) {
    switch (s) {
        case CSTONE_OK: return "ok";
        case CSTONE_ERR_INVALID_ARG: return "invalid argument";
        case CSTONE_ERR_NONFINITE: return "non-finite coordinate";
        case CSTONE_ERR_CAPACITY: return "leaf capacity exceeded";
        case CSTONE_ERR_NOT_CONVERGED: return "rebalance did not converge within max_iters";
        case CSTONE_ERR_DEVICE: return "device error";
    }
    return "unknown status";
}

cstone_status cstone_compute_keys(const double* x, const double* y, const double* z, size_t n, const cstone_box* box,
                                  cstone_curve curve, uint64_t* keys, uint32_t* flags, hipStream_t stream) {
    if (n > kMaxN || !box_ok(box) || (curve != CSTONE_MORTON && curve != CSTONE_HILBERT)) return CSTONE_ERR_INVALID_ARG;
    if (n && (!x || !y || !z || !keys)) return CSTONE_ERR_INVALID_ARG;
    return launch_keys(x, y, z, n, *box, curve, keys, flags, stream);
}

size_t cstone_sort_workspace_bytes(size_t n) { return sort_workspace_bytes(n, true); }

cstone_status cstone_sort(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n, void* ws,
                          size_t ws_bytes, hipStream_t stream) {
    if (n > kMaxN) return CSTONE_ERR_INVALID_ARG;
    if (n && (!keys_in || !keys_out || !perm_out || !ws)) return CSTONE_ERR_INVALID_ARG;
    return launch_sort(keys_in, keys_out, perm_out, n, 63, ws, ws_bytes, stream);
}

cstone_status cstone_node_counts(const uint64_t* sorted_keys, size_t n, const uint64_t* leaves, size_t n_leaves,
                                 uint32_t* counts, hipStream_t stream) {
    if (n > kMaxN || n_leaves < 1 || !leaves || !counts || (n && !sorted_keys)) return CSTONE_ERR_INVALID_ARG;
    return launch_node_counts(sorted_keys, n, leaves, n_leaves, counts, stream);
}

size_t cstone_rebalance_workspace_bytes(size_t n, uint32_t n_crit, size_t leaf_capacity) {
    return rebalance_workspace_bytes(n, n_crit, leaf_capacity);
}

size_t cstone_leaf_capacity_bound(size_t n, uint32_t n_crit, size_t n_leaves_start) {
    const size_t full = n / (static_cast<size_t>(n_crit) + 1);
    size_t bound = 7 * static_cast<size_t>(kL) * full + 1;
    if (n_leaves_start > 1) bound = std::max(bound, n_leaves_start + 7 * full);
    return bound;
}

cstone_status cstone_rebalance(const uint64_t* sorted_keys, size_t n, uint32_t n_crit, uint64_t* leaves,
                               size_t* n_leaves, size_t leaf_capacity, uint32_t* counts, uint32_t max_iters,
                               uint32_t* iters_done, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n > kMaxN || n_crit == 0 || !leaves || !n_leaves || !ws || (n && !sorted_keys)) return CSTONE_ERR_INVALID_ARG;
    if (*n_leaves < 1 || *n_leaves > leaf_capacity) return CSTONE_ERR_INVALID_ARG;
    return run_rebalance(sorted_keys, n, n_crit, leaves, n_leaves, leaf_capacity, counts, max_iters, iters_done, ws,
                         ws_bytes, stream);
}

size_t cstone_node_count(size_t n_leaves) { return nodes_of(n_leaves); }

size_t cstone_link_workspace_bytes(size_t n_leaves) { return link_workspace_bytes(n_leaves); }

cstone_status cstone_link_octree(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys, uint32_t* child,
                                 uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n_leaves < 1 || n_leaves > kMaxN || (n_leaves - 1) % 7 != 0) return CSTONE_ERR_INVALID_ARG;
    if (!leaves || !node_keys || !child || !level_offsets || !ws) return CSTONE_ERR_INVALID_ARG;
    return launch_link(leaves, n_leaves, nullptr, node_keys, child, level_offsets, ws, ws_bytes, stream);
}

cstone_status cstone_link_octree_by_sort(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys, uint32_t* child,
                                         uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n_leaves < 1 || n_leaves > kMaxN || (n_leaves - 1) % 7 != 0) return CSTONE_ERR_INVALID_ARG;
    if (!leaves || !node_keys || !child || !level_offsets || !ws) return CSTONE_ERR_INVALID_ARG;
    return launch_link_by_sort(leaves, n_leaves, node_keys, child, level_offsets, ws, ws_bytes, stream);
}

cstone_status cstone_radix_tree(const uint64_t* keys, size_t m, uint32_t* first, uint32_t* last, uint32_t* split,
                                uint32_t* prefix_len, hipStream_t stream) {
    if (m > kMaxN || (m >= 2 && (!keys || !prefix_len))) return CSTONE_ERR_INVALID_ARG;
    return launch_radix_tree(keys, m, first, last, split, prefix_len, stream);
}

size_t cstone_link_octree_radix_workspace_bytes(size_t n_leaves) { return radix_link_workspace_bytes(n_leaves); }

cstone_status cstone_link_octree_radix(const uint64_t* leaves, size_t n_leaves, uint64_t* node_keys, uint32_t* child,
                                       uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n_leaves < 1 || n_leaves > kMaxN || (n_leaves - 1) % 7 != 0) return CSTONE_ERR_INVALID_ARG;
    if (!leaves || !node_keys || !child || !level_offsets || !ws) return CSTONE_ERR_INVALID_ARG;
    return launch_link_radix(leaves, n_leaves, node_keys, child, level_offsets, ws, ws_bytes, stream);
}

size_t cstone_compact_octree_workspace_bytes(size_t n_leaves) { return compact_octree_workspace_bytes(n_leaves); }

cstone_status cstone_compact_octree(const uint64_t* leaves, const uint32_t* counts, size_t n_leaves,
                                    uint64_t* node_keys, uint32_t* parent, uint32_t* level_offsets, size_t* n_nodes,
                                    void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n_leaves < 1 || n_leaves >= kMaxN / 2) return CSTONE_ERR_INVALID_ARG;
    if (!leaves || !counts || !node_keys || !parent || !level_offsets || !n_nodes || !ws) return CSTONE_ERR_INVALID_ARG;
    return launch_compact_octree(leaves, counts, n_leaves, node_keys, parent, level_offsets, n_nodes, ws, ws_bytes,
                                 stream);
}

size_t cstone_octree_node_counts_workspace_bytes(size_t n_leaves) { return node_props_workspace_bytes(n_leaves); }

cstone_status cstone_octree_node_counts(const uint64_t* leaves, const uint32_t* counts, size_t n_leaves,
                                        const uint64_t* node_keys, size_t n_nodes, uint32_t* node_counts, void* ws,
                                        size_t ws_bytes, hipStream_t stream) {
    if (n_leaves < 1 || n_leaves > kMaxN || n_nodes > kMaxN) return CSTONE_ERR_INVALID_ARG;
    if (!leaves || !counts || !ws || (n_nodes && (!node_keys || !node_counts))) return CSTONE_ERR_INVALID_ARG;
    return launch_octree_node_counts(leaves, counts, n_leaves, node_keys, n_nodes, node_counts, ws, ws_bytes, stream);
}

cstone_status cstone_gather(const double* src, const uint32_t* perm, size_t n, double* dst, hipStream_t stream) {
    if (n > kMaxN || (n && (!src || !perm || !dst))) return CSTONE_ERR_INVALID_ARG;
    return launch_gather(&src, perm, n, &dst, 1, false, stream);
}

cstone_status cstone_gather_xyz(const double* x, const double* y, const double* z, const uint32_t* perm, size_t n,
                                double* ox, double* oy, double* oz, int fused, hipStream_t stream) {
    if (n > kMaxN || (n && (!x || !y || !z || !perm || !ox || !oy || !oz))) return CSTONE_ERR_INVALID_ARG;
    const double* src[3] = {x, y, z};
    double* dst[3] = {ox, oy, oz};
    return launch_gather(src, perm, n, dst, 3, fused != 0, stream);
}

size_t cstone_build_workspace_bytes(size_t n, size_t leaf_capacity) {
    Carve c(nullptr);
    c.take<uint64_t>(n);  // unsorted keys
    c.take<uint32_t>(1);  // non-finite flag
    c.take<uint32_t>(kLevel6Cells);  // first positions of the level-6 nodes (sort to loop)
    // the sort runs before the loop; the loop and the link share the stream
    // without a host check in between, so they get separate parts (the split
    // list of the loop is largest for n_crit = 1)
    size_t stage = std::max(sort_workspace_bytes(n, true),
                            rebalance_workspace_bytes(n, 1, leaf_capacity) + link_workspace_bytes(leaf_capacity));
    return c.off + stage;
}

cstone_status cstone_build(const double* x, const double* y, const double* z, size_t n, const cstone_box* box,
                           cstone_curve curve, uint32_t n_crit, uint64_t* sorted_keys, uint32_t* perm,
                           uint64_t* leaves, size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                           uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets, uint32_t max_iters,
                           uint32_t* iters_done, void* ws, size_t ws_bytes, cstone_timings* timings,
                           hipStream_t stream) {
    if (n > kMaxN || n_crit == 0 || !box_ok(box) || !leaves || !n_leaves || !ws) return CSTONE_ERR_INVALID_ARG;
    if (curve != CSTONE_MORTON && curve != CSTONE_HILBERT) return CSTONE_ERR_INVALID_ARG;
    if (n && (!x || !y || !z || !sorted_keys || !perm)) return CSTONE_ERR_INVALID_ARG;
    if ((node_keys == nullptr) != (child == nullptr) || (node_keys && !level_offsets)) return CSTONE_ERR_INVALID_ARG;
    if (leaf_capacity < 1 || *n_leaves > leaf_capacity) return CSTONE_ERR_INVALID_ARG;
    if (ws_bytes < cstone_build_workspace_bytes(n, leaf_capacity)) return CSTONE_ERR_INVALID_ARG;

    Carve c(ws);
    uint64_t* keys = c.take<uint64_t>(n);
    uint32_t* flag = c.take<uint32_t>(1);
    uint32_t* level6_table = c.take<uint32_t>(kLevel6Cells);
    // the sort shape is looked up once: the key kernel's digit counts, the
    // sort's set-up and its passes must all use the same one
    const int variant = sort_resolve_variant(n);
    uint32_t* level6 = n && sort_uses_split(n, 63, true, variant) ? level6_table : nullptr;
    void* stage_ws = static_cast<char*>(ws) + c.off;
    const size_t stage_bytes = ws_bytes - c.off;

    hipEvent_t ev[5] = {};
    hipEvent_t pass_ev[9] = {};
    const int passes = sort_passes(n, 63, true, variant);
    const bool timed = timings != nullptr;
    auto cleanup = [&]() {
        for (auto& e : ev)
            if (e) (void)hipEventDestroy(e);
        for (auto& e : pass_ev)
            if (e) (void)hipEventDestroy(e);
    };
    if (timed) {
        for (auto& e : ev)
            if (hipEventCreate(&e) != hipSuccess) { cleanup(); return CSTONE_ERR_DEVICE; }
        for (int i = 0; i <= passes; ++i)
            if (hipEventCreate(&pass_ev[i]) != hipSuccess) { cleanup(); return CSTONE_ERR_DEVICE; }
    }
    auto mark = [&](int i) -> hipError_t { return timed ? hipEventRecord(ev[i], stream) : hipSuccess; };
    cstone_status s = CSTONE_OK;
    uint32_t host_flag = 0;
    size_t nl = *n_leaves;
    do {
        if (mark(0) != hipSuccess) { s = CSTONE_ERR_DEVICE; break; }
        // The key kernel goes first (a long launch, so the host's later
        // launches overlap it) and stores per-block counts of the sort's first
        // digit (of all three top digits for the split sort) and per-block
        // non-finite flags; the sort's set-up launch sums them, writes the
        // flag word and clears what the passes need cleared.
        if (n) {
            uint32_t *hist_parts = nullptr, *bad_parts = nullptr, hist_mask = 0, hist_shift = 0, parts = 0,
                     hist_digits = 1;
            sort_key_parts(stage_ws, n, true, 63, variant, &hist_parts, &bad_parts, &hist_mask, &hist_shift,
                           &hist_digits);
            s = launch_keys(x, y, z, n, *box, curve, keys, nullptr, stream, hist_parts, hist_mask, hist_shift,
                            bad_parts, &parts, hist_digits);
            if (s != CSTONE_OK) break;
            if (mark(1) != hipSuccess) { s = CSTONE_ERR_DEVICE; break; }
            if ((s = sort_setup_from_keys(stage_ws, n, true, variant, parts, flag, level6, stream)) != CSTONE_OK) break;
        } else {
            hipLaunchKernelGGL(clear_word_kernel, dim3(1), dim3(1), 0, stream, flag);
            if (mark(1) != hipSuccess) { s = CSTONE_ERR_DEVICE; break; }
        }
        // the sort reports a failed device-side wait into the same flag word,
        // and (split sort) hands the level-6 node positions to the loop's start
        s = launch_sort(keys, sorted_keys, perm, n, 63, stage_ws, stage_bytes, stream,
                        timed && n ? pass_ev : nullptr, /*prepared=*/true, variant, flag, level6);
        if (s != CSTONE_OK) break;
        if (mark(2) != hipSuccess) { s = CSTONE_ERR_DEVICE; break; }
        if (nl == 0) nl = 1;  // start from the root leaf {0, 8^L}
        // the loop and the link are enqueued together; the host looks once,
        // after the link, and only goes round again if the loop needs more rounds
        const size_t reb_bytes = rebalance_workspace_bytes(n, n_crit, leaf_capacity);
        void* link_ws = static_cast<char*>(stage_ws) + reb_bytes;
        const size_t link_bytes = stage_bytes - reb_bytes;
        RebalanceLoop loop;
        s = loop.begin(sorted_keys, n, n_crit, leaves, nl, leaf_capacity, counts, max_iters, stage_ws, reb_bytes,
                       stream, flag, level6);
        if (s != CSTONE_OK) break;
        // The link is enqueued behind the first batch of rounds (usually the
        // last one), so one synchronisation serves both; if more rounds are
        // needed, it runs again once, after the last batch.
        bool finished = false, linked = false;
        for (uint32_t batch = 0; !finished; batch = 4) {
            if ((s = loop.enqueue(batch)) != CSTONE_OK) break;
            if (mark(3) != hipSuccess) { s = CSTONE_ERR_DEVICE; break; }
            if (node_keys && batch == 0) {
                s = launch_link(leaves, leaf_capacity, loop.device_leaf_count(), node_keys, child, level_offsets,
                                link_ws, link_bytes, stream);
                if (s != CSTONE_OK) break;
                linked = true;
            }
            if (mark(4) != hipSuccess) { s = CSTONE_ERR_DEVICE; break; }
            loop.wait(&finished);
            if (!finished) linked = false;
        }
        if (s != CSTONE_OK) break;
        if (node_keys && !linked && loop.status == CSTONE_OK) {  // the tree the first link saw was not the last
            if (mark(3) != hipSuccess) { s = CSTONE_ERR_DEVICE; break; }
            s = launch_link(leaves, leaf_capacity, loop.device_leaf_count(), node_keys, child, level_offsets, link_ws,
                            link_bytes, stream);
            if (s != CSTONE_OK) break;
            if (mark(4) != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) { s = CSTONE_ERR_DEVICE; break; }
        }
        *n_leaves = loop.n_leaves;
        if (iters_done) *iters_done = loop.rounds;
        host_flag = loop.input_flags;
        if (host_flag & ~CSTONE_FLAG_NONFINITE) { s = CSTONE_ERR_DEVICE; break; }  // the sort gave up a wait
        if (host_flag & CSTONE_FLAG_NONFINITE) { s = CSTONE_ERR_NONFINITE; break; }
        if ((s = loop.status) != CSTONE_OK) break;
        if (timed) {
            for (int i = 0; i < 4; ++i)
                if (hipEventElapsedTime(&timings->stage_ms[i], ev[i], ev[i + 1]) != hipSuccess) s = CSTONE_ERR_DEVICE;
            timings->sort_passes = n ? static_cast<uint32_t>(passes) : 0u;
            for (int p = 0; p < 8; ++p) timings->sort_pass_ms[p] = 0.f;
            for (int p = 0; n && p < passes; ++p)
                if (hipEventElapsedTime(&timings->sort_pass_ms[p], pass_ev[p], pass_ev[p + 1]) != hipSuccess)
                    s = CSTONE_ERR_DEVICE;
        }
    } while (false);
    cleanup();
    return s;
}

}  // extern "C"
