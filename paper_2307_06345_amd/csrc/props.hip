// Node properties of the linked octree and particles in curve order.
//
// Node counts (Sec. 5: properties of all n nodes in separate arrays, here the
// particle count an upward pass gives every node). The count of a node is the
// sum of its leaves' counts, and a node's leaves are a contiguous run of K:
// with S the exclusive prefix sum of the leaf counts, a node covering the key
// range [a, b) holds S[lb(K, b)] - S[lb(K, a)] particles. So one scan of the
// leaf counts and one pass over the nodes (two searches of K each, adjacent
// threads searching adjacent keys, so their paths share cache lines) replace
// the level-by-level pass, with the same exact integers.
//
// Gather (Sec. 4, the permutation that sorts the keys applied to the particle
// arrays): dst[i] = src[perm[i]]. The writes and the reads of perm stream; the
// source reads follow the curve, scattered for unsorted input. One array per
// pass keeps the array being gathered (8 B per particle) resident in the
// 256 MB last-level cache for inputs up to 2^25 particles.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr uint32_t kScanTile = kScanBlock * kScanItems;
constexpr int kNodeBlock = 256;
constexpr int kGatherBlock = 256;
constexpr int kGatherItems = 8;

// Clears the scan's look-back words, its tile counter and its error word.
__global__ __launch_bounds__(256) void props_setup_kernel(uint64_t* words, size_t n_words, uint32_t* counter,
                                                          uint32_t* err) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n_words; i += stride) words[i] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *counter = 0;
        *err = 0;
    }
}

// S[i] = counts[0] + ... + counts[i - 1] for i <= nl (S[nl] the total): one
// pass, tiles taken in order from a counter, decoupled look-back across tiles.
__global__ __launch_bounds__(kScanBlock) void exclusive_scan_kernel(const uint32_t* __restrict__ counts, uint32_t nl,
                                                                    uint32_t* __restrict__ S, uint64_t* words,
                                                                    uint32_t* counter, uint32_t* err) {
    __shared__ uint32_t slot;
    __shared__ uint64_t scan_tmp[kScanBlock / kWave];
    __shared__ uint64_t tile_prefix;
    const uint32_t tile = take_tile(counter, &slot);
    const uint32_t base = tile * kScanTile + threadIdx.x * kScanItems;  // blocked: each thread a run of items
    uint32_t v[kScanItems];
    uint64_t mine = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < nl ? counts[base + i] : 0u;
        mine += v[i];
    }
    uint64_t total;
    const uint64_t excl = block_exclusive_sum<uint64_t, kScanBlock>(mine, scan_tmp, &total);
    if (threadIdx.x < kWave) {  // the first wave publishes the aggregate and resolves the prefix
        const uint32_t lane = lane_id();
        if (lane == 0) st_agent(words + tile, lb_word(tile == 0 ? kFlagInc : kFlagAgg, 1, total));
        uint64_t prefix = 0;
        if (tile > 0) {
            prefix = lookback_wave<4>(words, tile, 1, err);
            if (lane == 0) st_agent(words + tile, lb_word(kFlagInc, 1, prefix + total));
        }
        if (lane == 0) tile_prefix = prefix;
    }
    __syncthreads();
    uint64_t run = tile_prefix + excl;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i <= nl) S[base + i] = static_cast<uint32_t>(run);  // the entry at nl is the total
        run += v[i];
    }
}

// Particle count of every node: the leaf run of its key range, by two
// searches of K. A node that does not start at a leaf boundary (node keys of
// another tree) gets 0xffffffff.
__global__ __launch_bounds__(kNodeBlock) void node_counts_tree_kernel(const uint64_t* __restrict__ K, uint32_t nl,
                                                                      const uint32_t* __restrict__ S,
                                                                      const uint64_t* __restrict__ NK, uint32_t n,
                                                                      uint32_t* __restrict__ out) {
    const uint32_t p = blockIdx.x * kNodeBlock + threadIdx.x;
    if (p >= n) return;
    const uint64_t key = NK[p];
    const int level = (63 - clz64(key)) / 3;  // the placeholder bit sits at 3 * level
    const int shift = 3 * (kL - level);
    const uint64_t start = (key ^ (1ull << (3 * level))) << shift;
    const uint64_t end = start + (1ull << shift);
    const uint32_t i0 = static_cast<uint32_t>(lower_bound_u64(K, 0, nl, start));
    if (i0 >= nl || K[i0] != start) {  // never for a node of this tree: it starts at a leaf boundary
        out[p] = 0xffffffffu;
        return;
    }
    // the run's end: the next leaf (a leaf node), else a galloping search forward
    uint32_t i1 = i0 + 1;
    if (K[i1] < end) {
        uint32_t step = 1, lo = i1;
        while (true) {
            const uint32_t probe = static_cast<uint32_t>(std::min<uint64_t>(static_cast<uint64_t>(lo) + step, nl));
            if (K[probe] >= end) {
                i1 = static_cast<uint32_t>(lower_bound_u64(K, lo + 1, probe, end));
                break;
            }
            lo = probe;
            step <<= 1;
        }
    }
    out[p] = S[i1] - S[i0];
}

template <int ARRAYS>
__global__ __launch_bounds__(kGatherBlock) void gather_kernel(const double* __restrict__ a0,
                                                              const double* __restrict__ a1,
                                                              const double* __restrict__ a2,
                                                              const uint32_t* __restrict__ perm, uint32_t n,
                                                              double* __restrict__ o0, double* __restrict__ o1,
                                                              double* __restrict__ o2) {
    const size_t base = static_cast<size_t>(blockIdx.x) * (kGatherBlock * kGatherItems) + threadIdx.x;
    uint32_t src[kGatherItems];
#pragma unroll
    for (int i = 0; i < kGatherItems; ++i) {
        const size_t j = base + i * kGatherBlock;
        src[i] = j < n ? perm[j] : 0u;
    }
    double v[kGatherItems];
#pragma unroll
    for (int i = 0; i < kGatherItems; ++i) v[i] = base + i * kGatherBlock < n ? a0[src[i]] : 0.0;
#pragma unroll
    for (int i = 0; i < kGatherItems; ++i)
        if (base + i * kGatherBlock < n) o0[base + i * kGatherBlock] = v[i];
    if constexpr (ARRAYS > 1) {
#pragma unroll
        for (int i = 0; i < kGatherItems; ++i) v[i] = base + i * kGatherBlock < n ? a1[src[i]] : 0.0;
#pragma unroll
        for (int i = 0; i < kGatherItems; ++i)
            if (base + i * kGatherBlock < n) o1[base + i * kGatherBlock] = v[i];
    }
    if constexpr (ARRAYS > 2) {
#pragma unroll
        for (int i = 0; i < kGatherItems; ++i) v[i] = base + i * kGatherBlock < n ? a2[src[i]] : 0.0;
#pragma unroll
        for (int i = 0; i < kGatherItems; ++i)
            if (base + i * kGatherBlock < n) o2[base + i * kGatherBlock] = v[i];
    }
}

struct ScanWs {
    uint64_t* words;
    uint32_t* counter;
    uint32_t* err;
    size_t tiles, bytes;
};

ScanWs carve_scan(void* ws, size_t n) {
    Carve c(ws);
    ScanWs w{};
    w.tiles = (n + 1 + kScanTile - 1) / kScanTile;
    w.words = c.take<uint64_t>(w.tiles);
    w.counter = c.take<uint32_t>(1);
    w.err = c.take<uint32_t>(1);
    w.bytes = c.off;
    return w;
}

}  // namespace

size_t scan_u32_workspace_bytes(size_t n) { return carve_scan(nullptr, n).bytes; }

cstone_status launch_scan_u32(const uint32_t* in, size_t n, uint32_t* out, void* ws, size_t ws_bytes,
                              hipStream_t stream) {
    ScanWs w = carve_scan(ws, n);
    if (ws_bytes < w.bytes || n >= 0xffffffffull) return CSTONE_ERR_INVALID_ARG;
    hipLaunchKernelGGL(props_setup_kernel, dim3(static_cast<uint32_t>(std::min<size_t>((w.tiles + 255) / 256, 256))),
                       dim3(256), 0, stream, w.words, w.tiles, w.counter, w.err);
    hipLaunchKernelGGL(exclusive_scan_kernel, dim3(static_cast<uint32_t>(w.tiles)), dim3(kScanBlock), 0, stream, in,
                       static_cast<uint32_t>(n), out, w.words, w.counter, w.err);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

size_t node_props_workspace_bytes(size_t n_leaves) {
    Carve c(nullptr);
    c.take<uint32_t>(n_leaves + 1);
    return c.off + scan_u32_workspace_bytes(n_leaves);
}

cstone_status launch_octree_node_counts(const uint64_t* leaves, const uint32_t* counts, size_t nl,
                                        const uint64_t* node_keys, size_t n_nodes, uint32_t* node_counts, void* ws,
                                        size_t ws_bytes, hipStream_t stream) {
    if (ws_bytes < node_props_workspace_bytes(nl)) return CSTONE_ERR_INVALID_ARG;
    Carve c(ws);
    uint32_t* S = c.take<uint32_t>(nl + 1);
    cstone_status st = launch_scan_u32(counts, nl, S, static_cast<char*>(ws) + c.off, ws_bytes - c.off, stream);
    if (st != CSTONE_OK) return st;
    if (n_nodes)
        hipLaunchKernelGGL(node_counts_tree_kernel, dim3(static_cast<uint32_t>((n_nodes + kNodeBlock - 1) / kNodeBlock)),
                           dim3(kNodeBlock), 0, stream, leaves, static_cast<uint32_t>(nl), S, node_keys,
                           static_cast<uint32_t>(n_nodes), node_counts);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

cstone_status launch_gather(const double* const* src, const uint32_t* perm, size_t n, double* const* dst, int arrays,
                            bool fused, hipStream_t stream) {
    if (n == 0) return CSTONE_OK;
    const uint32_t un = static_cast<uint32_t>(n);
    const dim3 grid(static_cast<uint32_t>((n + kGatherBlock * kGatherItems - 1) / (kGatherBlock * kGatherItems)));
    if (fused && arrays == 3) {
        hipLaunchKernelGGL(gather_kernel<3>, grid, dim3(kGatherBlock), 0, stream, src[0], src[1], src[2], perm, un,
                           dst[0], dst[1], dst[2]);
    } else {
        for (int a = 0; a < arrays; ++a)
            hipLaunchKernelGGL(gather_kernel<1>, grid, dim3(kGatherBlock), 0, stream, src[a],
                               static_cast<const double*>(nullptr), static_cast<const double*>(nullptr), perm, un,
                               dst[a], static_cast<double*>(nullptr), static_cast<double*>(nullptr));
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace cs
