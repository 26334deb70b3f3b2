// Batched builds (many independent particle sets in one launch sequence) and
// the sort-shape autotuner.
//
// A plan fixes, on the host, where every set's particles, leaves and nodes
// live, each set's leaf capacity, and the tile table shared by the key kernel
// and the segmented sort (tiles never straddle two sets). The tables are
// copied once into the caller's workspace; the build itself is a fixed
// sequence of kernels on one stream:
//   clear   per-set flags, sort histograms and look-back words;
//   keys    one tile of one set per block, with that set's box and curve,
//           counting the set's first radix digit;
//   sort    one launch per digit pass over all tiles; each set has its own
//           digit counts and look-back chain;
//   rebalance  all sets' cornerstone arrays back to back, one decision +
//           scan + write launch and one split-search launch per round, for
//           L + 1 rounds (rounds after every set has converged exit at once);
//           per-set convergence flags; per-set leaves and counts at the end;
//   link    one count, scan, per-set base and write pass over all entries.
// With no host synchronisation and no allocation inside, the sequence is
// captured into one hipGraph and replayed.
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

using cs::BatchResult;
using cs::BatchSet;

struct cstone_batch {
    std::vector<cstone_set> in;
    std::vector<BatchSet> sets;
    std::vector<uint4> tiles;
    std::vector<uint32_t> seg_base;
    std::vector<uint64_t> part_off, leaf_off, node_off;
    uint64_t n_total = 0, leaf_slots = 0, node_slots = 0;
    uint64_t entries = 0;  // capacity of the back-to-back arrays
    uint64_t split_capacity = 0;
    uint64_t max_set = 0;
    uint64_t max_tiles = 0;  // over all sort shapes
    int variant = 0;
    uint32_t rounds = cs::kL + 1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace cs {
namespace {

struct BatchWs {
    BatchSet* sets;
    uint4* tiles;
    uint32_t* seg_base;
    uint32_t* flags;
    uint64_t* keys;
    void* stage;  // the sort's workspace, then the rebalance's and the link's
    size_t stage_bytes;
    size_t bytes;
    size_t off_tiles, off_seg_base, tables_end;  // byte offsets of the plan tables (sets start at 0)
};

size_t stage_bytes_for(const cstone_batch& p) {
    const uint32_t ns = static_cast<uint32_t>(p.sets.size());
    size_t sort_max = 0;
    for (int v = 0; v < sort_variant_count(); ++v)
        sort_max = std::max(sort_max, sort_seg_workspace_bytes(p.n_total, p.max_tiles, ns, v));
    Carve c(nullptr);
    c.take<uint8_t>(batch_rebalance_workspace_bytes(ns, p.entries, p.split_capacity));
    c.take<uint8_t>(link_batch_workspace_bytes(ns, p.entries));
    return std::max(sort_max, c.off);
}

BatchWs carve_batch(const cstone_batch& p, void* ws) {
    Carve c(ws);
    BatchWs w{};
    w.sets = c.take<BatchSet>(p.sets.size());
    w.off_tiles = c.off;
    w.tiles = c.take<uint4>(p.max_tiles);
    w.off_seg_base = c.off;
    w.seg_base = c.take<uint32_t>(p.sets.size());
    w.tables_end = w.off_seg_base + p.sets.size() * sizeof(uint32_t);
    w.flags = c.take<uint32_t>(p.sets.size() + 1);  // per set, then the sort's device-wait error word
    w.keys = c.take<uint64_t>(p.n_total);
    w.stage_bytes = stage_bytes_for(p);
    w.stage = c.take<uint8_t>(w.stage_bytes);
    w.bytes = c.off;
    return w;
}

// the rebalance workspace and, after it, the link's, inside the stage region
void* rebalance_ws(const BatchWs& w) { return w.stage; }
void* link_ws(const cstone_batch& p, const BatchWs& w) {
    return static_cast<char*>(w.stage) +
           align_up(batch_rebalance_workspace_bytes(static_cast<uint32_t>(p.sets.size()), p.entries,
                                                    p.split_capacity),
                    256);
}

uint64_t tiles_for(const cstone_batch& p, int variant) {
    const uint64_t t = sort_variant_info(variant).tile;
    uint64_t n = 0;
    for (const BatchSet& s : p.sets) n += (s.n + t - 1) / t;
    return n;
}

void make_tiles(cstone_batch& p) {
    const uint32_t t = static_cast<uint32_t>(sort_variant_info(p.variant).tile);
    p.tiles.clear();
    for (uint32_t s = 0; s < p.sets.size(); ++s) {
        const BatchSet& S = p.sets[s];
        const uint32_t first = static_cast<uint32_t>(p.tiles.size());
        for (uint32_t b = 0; b < S.n; b += t) p.tiles.push_back(make_uint4(S.part_off + b, std::min(t, S.n - b), first, s));
    }
}

__global__ void fill_u32_kernel(uint32_t* p, size_t n, uint32_t v) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) p[i] = v;
}

bool box_ok(const cstone_box& b) {
    for (int d = 0; d < 3; ++d)
        if (!(b.lo[d] < b.hi[d]) || !__builtin_isfinite(b.lo[d]) || !__builtin_isfinite(b.hi[d])) return false;
    return true;
}

cstone_status enqueue_build(const cstone_batch& p, const double* x, const double* y, const double* z,
                            uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves, uint32_t* counts,
                            uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets,
                            cstone_set_result* results, void* ws, size_t ws_bytes, hipStream_t stream) {
    const BatchWs w = carve_batch(p, ws);
    if (!ws || ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    if (!leaves || !counts || !node_keys || !child || !level_offsets || !results) return CSTONE_ERR_INVALID_ARG;
    if (p.n_total && (!x || !y || !z || !sorted_keys || !perm)) return CSTONE_ERR_INVALID_ARG;
    const uint32_t ns = static_cast<uint32_t>(p.sets.size());
    if (ns == 0) return CSTONE_OK;
    const uint32_t nt = static_cast<uint32_t>(p.tiles.size());
    cstone_status st;
    uint32_t* sort_err = w.flags + ns;
    hipLaunchKernelGGL(fill_u32_kernel, dim3((ns + 256) / 256), dim3(256), 0, stream, w.flags,
                       static_cast<size_t>(ns) + 1, 0u);
    if (p.n_total) {
        if ((st = sort_seg_prepare(w.stage, p.n_total, nt, ns, p.variant, stream)) != CSTONE_OK) return st;
        uint32_t stride = 0, mask = 0, shift = 0;
        uint32_t* hist0 = sort_seg_first_histogram(w.stage, p.n_total, nt, ns, p.variant, &stride, &mask, &shift);
        if ((st = launch_keys_batch(x, y, z, w.tiles, nt, w.sets, w.keys, w.flags, hist0, stride, mask, shift,
                                    stream)) != CSTONE_OK)
            return st;
        if ((st = launch_sort_segmented(w.keys, sorted_keys, perm, p.n_total, w.tiles, nt, w.seg_base, ns,
                                        p.max_set, 63, p.variant, w.stage, w.stage_bytes, stream, sort_err)) !=
            CSTONE_OK)
            return st;
    }
    const size_t rb = batch_rebalance_workspace_bytes(ns, p.entries, p.split_capacity);
    if ((st = launch_batch_rebalance(sorted_keys, p.n_total, w.sets, ns, p.entries, p.split_capacity, p.rounds, w.flags,
                                     leaves, counts, reinterpret_cast<BatchResult*>(results), rebalance_ws(w), rb,
                                     sort_err, stream)) != CSTONE_OK)
        return st;
    const BatchTreeView view = batch_rebalance_view(rebalance_ws(w), ns, p.entries, p.split_capacity);
    return launch_link_batch(view, w.sets, ns, p.entries, node_keys, child, level_offsets, link_ws(p, w),
                             link_batch_workspace_bytes(ns, p.entries), stream);
}

void drop_graph(cstone_batch* p) {
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->exec = nullptr;
    p->graph = nullptr;
}

}  // namespace
}  // namespace cs

extern "C" {

CSTONE_API cstone_status cstone_batch_create(const cstone_set* sets, uint32_t n_sets, cstone_batch** plan) {
    if (!plan || (n_sets && !sets)) return CSTONE_ERR_INVALID_ARG;
    *plan = nullptr;
    cstone_batch* p = new (std::nothrow) cstone_batch();
    if (!p) return CSTONE_ERR_INVALID_ARG;
    p->in.assign(sets, sets + n_sets);
    uint64_t part = 0, leaf = 0, node = 0, entries = 0, splits = 0;
    for (uint32_t s = 0; s < n_sets; ++s) {
        const cstone_set& in = sets[s];
        if (in.n_crit == 0 || !cs::box_ok(in.box) || (in.curve != CSTONE_MORTON && in.curve != CSTONE_HILBERT)) {
            delete p;
            return CSTONE_ERR_INVALID_ARG;
        }
        const uint64_t cap = in.leaf_capacity ? in.leaf_capacity : cstone_leaf_capacity_bound(in.n, in.n_crit, 1);
        cs::BatchSet b{};
        for (int d = 0; d < 3; ++d) {
            b.lo[d] = in.box.lo[d];
            b.scale[d] = 2097152.0 / (in.box.hi[d] - in.box.lo[d]);
        }
        b.n = static_cast<uint32_t>(in.n);
        b.curve = static_cast<uint32_t>(in.curve);
        b.n_crit = in.n_crit;
        b.part_off = static_cast<uint32_t>(part);
        b.leaf_off = leaf;
        b.node_off = node;
        b.cap = cap;
        b.node_cap = cap + (cap - 1) / 7;
        p->part_off.push_back(part);
        p->leaf_off.push_back(leaf);
        p->node_off.push_back(node);
        part += in.n;
        leaf += cap + 1;
        node += b.node_cap;
        entries += cap + 1;
        splits += std::min<uint64_t>(cap, in.n / (static_cast<uint64_t>(in.n_crit) + 1)) + 1;
        p->max_set = std::max<uint64_t>(p->max_set, in.n);
        p->sets.push_back(b);
        p->seg_base.push_back(b.part_off);
        if (in.n >= (1ull << 32) || cap < 1 || part >= (1ull << 32) || entries >= (1ull << 32) - 1) {
            delete p;
            return CSTONE_ERR_INVALID_ARG;
        }
    }
    p->part_off.push_back(part);
    p->leaf_off.push_back(leaf);
    p->node_off.push_back(node);
    p->n_total = part;
    p->leaf_slots = leaf;
    p->node_slots = node;
    p->entries = std::max<uint64_t>(entries, 2ull * n_sets);
    p->split_capacity = splits + 1;
    for (int v = 0; v < cs::sort_variant_count(); ++v)
        p->max_tiles = std::max<uint64_t>(p->max_tiles, cs::tiles_for(*p, v));
    {  // the autotune table's shape for a batch of this many keys, else the built-in one
        const int tuned = cs::tune_lookup(cs::kTuneBatchSort, p->n_total);
        p->variant = tuned >= 0 ? tuned : cs::sort_builtin_variant();
    }
    cs::make_tiles(*p);
    *plan = p;
    return CSTONE_OK;
}

CSTONE_API void cstone_batch_destroy(cstone_batch* plan) {
    if (!plan) return;
    cs::drop_graph(plan);
    delete plan;
}

CSTONE_API cstone_status cstone_batch_get_layout(const cstone_batch* p, cstone_batch_layout* layout,
                                                 uint64_t* particle_offsets, uint64_t* leaf_offsets,
                                                 uint64_t* node_offsets) {
    if (!p) return CSTONE_ERR_INVALID_ARG;
    if (layout) {
        layout->n_sets = p->sets.size();
        layout->n_particles = p->n_total;
        layout->leaf_slots = p->leaf_slots;
        layout->node_slots = p->node_slots;
        layout->workspace_bytes = cs::carve_batch(*p, nullptr).bytes;
        layout->n_tiles = p->tiles.size();
        layout->sort_variant = p->variant;
        layout->rounds = p->rounds;
    }
    const size_t m = p->part_off.size() * sizeof(uint64_t);
    if (particle_offsets) std::memcpy(particle_offsets, p->part_off.data(), m);
    if (leaf_offsets) std::memcpy(leaf_offsets, p->leaf_off.data(), m);
    if (node_offsets) std::memcpy(node_offsets, p->node_off.data(), m);
    return CSTONE_OK;
}

CSTONE_API cstone_status cstone_batch_set_variant(cstone_batch* p, int variant) {
    if (!p || variant < 0 || variant >= cs::sort_variant_count()) return CSTONE_ERR_INVALID_ARG;
    if (variant == p->variant) return CSTONE_OK;
    cs::drop_graph(p);
    p->variant = variant;
    cs::make_tiles(*p);
    return CSTONE_OK;
}

CSTONE_API cstone_status cstone_batch_set_rounds(cstone_batch* p, uint32_t rounds) {
    if (!p || rounds < 1 || rounds > static_cast<uint32_t>(cs::kL + 1)) return CSTONE_ERR_INVALID_ARG;
    if (rounds != p->rounds) cs::drop_graph(p);
    p->rounds = rounds;
    return CSTONE_OK;
}

CSTONE_API cstone_status cstone_batch_upload(const cstone_batch* p, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (!p) return CSTONE_ERR_INVALID_ARG;
    const cs::BatchWs w = cs::carve_batch(*p, ws);
    if (!ws || ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    if (!p->sets.empty()) {
        CS_HIP(hipMemcpyAsync(w.sets, p->sets.data(), p->sets.size() * sizeof(BatchSet), hipMemcpyHostToDevice,
                              stream));
        CS_HIP(hipMemcpyAsync(w.seg_base, p->seg_base.data(), p->seg_base.size() * sizeof(uint32_t),
                              hipMemcpyHostToDevice, stream));
    }
    if (!p->tiles.empty())
        CS_HIP(hipMemcpyAsync(w.tiles, p->tiles.data(), p->tiles.size() * sizeof(uint4), hipMemcpyHostToDevice,
                              stream));
    CS_HIP(hipStreamSynchronize(stream));
    return CSTONE_OK;
}

CSTONE_API size_t cstone_batch_table_bytes(const cstone_batch* p) {
    return p ? cs::carve_batch(*p, nullptr).tables_end : 0;
}

CSTONE_API cstone_status cstone_batch_upload_staged(const cstone_batch* p, void* ws, size_t ws_bytes, void* host_stage,
                                                    size_t stage_bytes, hipStream_t stream) {
    if (!p) return CSTONE_ERR_INVALID_ARG;
    const cs::BatchWs w = cs::carve_batch(*p, ws);
    if (!ws || ws_bytes < w.bytes || !host_stage || stage_bytes < w.tables_end) return CSTONE_ERR_INVALID_ARG;
    // the tables in their device layout, so one copy moves them all (the
    // gaps between them are copied too and never read)
    char* h = static_cast<char*>(host_stage);
    if (!p->sets.empty()) {
        std::memcpy(h, p->sets.data(), p->sets.size() * sizeof(BatchSet));
        std::memcpy(h + w.off_seg_base, p->seg_base.data(), p->seg_base.size() * sizeof(uint32_t));
    }
    if (!p->tiles.empty()) std::memcpy(h + w.off_tiles, p->tiles.data(), p->tiles.size() * sizeof(uint4));
    if (w.tables_end) CS_HIP(hipMemcpyAsync(ws, host_stage, w.tables_end, hipMemcpyHostToDevice, stream));
    return CSTONE_OK;
}

CSTONE_API cstone_status cstone_batch_build(const cstone_batch* p, const double* x, const double* y, const double* z,
                                            uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves, uint32_t* counts,
                                            uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets,
                                            cstone_set_result* results, void* ws, size_t ws_bytes,
                                            hipStream_t stream) {
    if (!p) return CSTONE_ERR_INVALID_ARG;
    return cs::enqueue_build(*p, x, y, z, sorted_keys, perm, leaves, counts, node_keys, child, level_offsets, results,
                             ws, ws_bytes, stream);
}

CSTONE_API cstone_status cstone_batch_capture(cstone_batch* p, const double* x, const double* y, const double* z,
                                              uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves,
                                              uint32_t* counts, uint64_t* node_keys, uint32_t* child,
                                              uint32_t* level_offsets, cstone_set_result* results, void* ws,
                                              size_t ws_bytes, hipStream_t stream) {
    if (!p || !stream) return CSTONE_ERR_INVALID_ARG;
    cs::drop_graph(p);
    CS_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    const cstone_status st = cs::enqueue_build(*p, x, y, z, sorted_keys, perm, leaves, counts, node_keys, child,
                                               level_offsets, results, ws, ws_bytes, stream);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(stream, &g);
    if (st != CSTONE_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess || !g) return CSTONE_ERR_DEVICE;
    hipGraphExec_t x_exec = nullptr;
    if (hipGraphInstantiate(&x_exec, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGraphDestroy(g);
        return CSTONE_ERR_DEVICE;
    }
    p->graph = g;
    p->exec = x_exec;
    return CSTONE_OK;
}

CSTONE_API cstone_status cstone_batch_launch(cstone_batch* p, hipStream_t stream) {
    if (!p || !p->exec) return CSTONE_ERR_INVALID_ARG;
    CS_HIP(hipGraphLaunch(p->exec, stream));
    return CSTONE_OK;
}

CSTONE_API cstone_status cstone_batch_autotune(cstone_batch* p, const double* x, const double* y, const double* z,
                                               uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves,
                                               uint32_t* counts, uint64_t* node_keys, uint32_t* child,
                                               uint32_t* level_offsets, cstone_set_result* results, void* ws,
                                               size_t ws_bytes, int reps, float* ms_per_variant, hipStream_t stream) {
    if (!p || reps < 1) return CSTONE_ERR_INVALID_ARG;
    cs::drop_graph(p);
    hipEvent_t e0, e1;
    CS_HIP(hipEventCreate(&e0));
    CS_HIP(hipEventCreate(&e1));
    int best = p->variant;
    float best_ms = 0.f;
    cstone_status st = CSTONE_OK;
    for (int v = 0; v < cs::sort_variant_count() && st == CSTONE_OK; ++v) {
        if ((st = cstone_batch_set_variant(p, v)) != CSTONE_OK) break;
        if ((st = cstone_batch_upload(p, ws, ws_bytes, stream)) != CSTONE_OK) break;
        float ms = 0.f;
        for (int r = -1; r < reps && st == CSTONE_OK; ++r) {  // r = -1: warm-up
            if (hipEventRecord(e0, stream) != hipSuccess) st = CSTONE_ERR_DEVICE;
            if (st == CSTONE_OK)
                st = cs::enqueue_build(*p, x, y, z, sorted_keys, perm, leaves, counts, node_keys, child,
                                       level_offsets, results, ws, ws_bytes, stream);
            if (st == CSTONE_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                st = CSTONE_ERR_DEVICE;
            float t = 0.f;
            if (st == CSTONE_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = CSTONE_ERR_DEVICE;
            if (r >= 0) ms += t;
        }
        ms /= static_cast<float>(reps);
        if (ms_per_variant) ms_per_variant[v] = ms;
        if (st == CSTONE_OK && (v == 0 || ms < best_ms)) {
            best = v;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != CSTONE_OK) return st;
    if ((st = cstone_batch_set_variant(p, best)) != CSTONE_OK) return st;
    cs::tune_record(cs::kTuneBatchSort, p->n_total, best);  // later plans of this size class start from it
    return cstone_batch_upload(p, ws, ws_bytes, stream);
}

CSTONE_API int cstone_sort_variant_count(void) { return cs::sort_variant_count(); }

CSTONE_API cstone_status cstone_sort_variant_info(int variant, int* digit_bits, int* block, int* items) {
    if (variant < 0 || variant >= cs::sort_variant_count()) return CSTONE_ERR_INVALID_ARG;
    const cs::SortVariantInfo v = cs::sort_variant_info(variant);
    if (digit_bits) *digit_bits = v.bits;
    if (block) *block = v.block;
    if (items) *items = v.items;
    return CSTONE_OK;
}

CSTONE_API cstone_status cstone_set_lookback_patience(uint32_t waits) { return cs::set_lookback_patience(waits); }

CSTONE_API cstone_status cstone_sort_variant_split(int variant, int* split) {
    if (variant < 0 || variant >= cs::sort_variant_count()) return CSTONE_ERR_INVALID_ARG;
    const cs::SortVariantInfo v = cs::sort_variant_info(variant);
    if (split) *split = v.split;
    return CSTONE_OK;
}

CSTONE_API cstone_status cstone_sort_autotune(const uint64_t* keys_in, size_t n, uint64_t* keys_out,
                                              uint32_t* perm_out, void* ws, size_t ws_bytes, int reps,
                                              float* ms_per_variant, int* chosen, hipStream_t stream) {
    if (!keys_in || !keys_out || !ws || reps < 1 || n == 0) return CSTONE_ERR_INVALID_ARG;
    if (ws_bytes < cs::sort_workspace_bytes(n, perm_out != nullptr)) return CSTONE_ERR_INVALID_ARG;
    hipEvent_t e0, e1;
    CS_HIP(hipEventCreate(&e0));
    CS_HIP(hipEventCreate(&e1));
    int best = 0;
    float best_ms = 0.f;
    cstone_status st = CSTONE_OK;
    for (int v = 0; v < cs::sort_variant_count() && st == CSTONE_OK; ++v) {
        float ms = 0.f;
        for (int r = -1; r < reps && st == CSTONE_OK; ++r) {
            if (hipEventRecord(e0, stream) != hipSuccess) st = CSTONE_ERR_DEVICE;
            if (st == CSTONE_OK)
                st = cs::launch_sort(keys_in, keys_out, perm_out, n, 63, ws, ws_bytes, stream, nullptr, false, v);
            if (st == CSTONE_OK && (hipEventRecord(e1, stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess))
                st = CSTONE_ERR_DEVICE;
            float t = 0.f;
            if (st == CSTONE_OK && hipEventElapsedTime(&t, e0, e1) != hipSuccess) st = CSTONE_ERR_DEVICE;
            if (r >= 0) ms += t;
        }
        ms /= static_cast<float>(reps);
        if (ms_per_variant) ms_per_variant[v] = ms;
        if (st == CSTONE_OK && (v == 0 || ms < best_ms)) {
            best = v;
            best_ms = ms;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != CSTONE_OK) return st;
    cs::tune_record(cs::kTuneSort, n, best);
    if (chosen) *chosen = best;
    return CSTONE_OK;
}

}  // extern "C"
