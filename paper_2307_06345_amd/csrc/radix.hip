// Octrees by way of a binary radix tree (Sec. 5, after Karras).
//
// The binary radix tree over m sorted unique 63-bit keys has m - 1 internal
// nodes, each built independently: node i's key range has i at one end, runs
// towards the neighbour sharing the longer prefix with key i, and extends as
// far as keys share more than the prefix key i shares with its other
// neighbour (an exponential then a binary search); its split is where the
// range's common prefix grows (another binary search).
//
// Two octree paths use it:
//  * linked octree over the cornerstone array K (every internal node has 8
//    children): the radix nodes whose prefix length is a multiple of 3 are
//    the internal octree nodes; a flag per node, an exclusive scan and one
//    extraction pass place them (and the leaves) in the node array, then the
//    node keys are sorted and linked as in the paper's steps 3-5. The result
//    equals cstone_link_octree's. This is the route the paper's closed-form
//    slot formula (Eq. digitweight) replaces.
//  * compact octree: the leaves that hold particles (empty buckets removed),
//    the radix nodes over their keys with whole-digit prefixes, and the root;
//    sorted breadth-first, each node linked to its nearest ancestor present.
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr int kRBlock = 256;

uint32_t grid_for(size_t items) { return static_cast<uint32_t>(std::max<size_t>(1, (items + kRBlock - 1) / kRBlock)); }

// Common prefix length of keys i and j (leading zeros of their XOR, the
// unused top bit included), -1 if j lies outside [0, m).
__device__ __forceinline__ int delta_at(const uint64_t* __restrict__ k, int64_t m, int64_t i, int64_t j) {
    return (j < 0 || j >= m) ? -1 : clz64(k[i] ^ k[j]);
}

// Internal node i < m - 1: its key range [first, last], the split (the last
// key of its left child) and its prefix length inside the 63-bit key; with
// whole != NULL, whole[i] = 1 if the prefix length is a multiple of 3.
__global__ __launch_bounds__(kRBlock) void radix_tree_kernel(const uint64_t* __restrict__ k, uint32_t m,
                                                             uint32_t* __restrict__ first, uint32_t* __restrict__ last,
                                                             uint32_t* __restrict__ split,
                                                             uint32_t* __restrict__ plen, uint32_t* __restrict__ whole) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * kRBlock + threadIdx.x;
    if (i + 1 >= static_cast<int64_t>(m)) return;
    const int64_t mm = m;
    const int d = delta_at(k, mm, i, i + 1) > delta_at(k, mm, i, i - 1) ? 1 : -1;
    const int dmin = delta_at(k, mm, i, i - d);
    int64_t lmax = 2;
    while (delta_at(k, mm, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
        if (delta_at(k, mm, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = delta_at(k, mm, i, j);
    int64_t s = 0, t = l;
    do {
        t = (t + 1) >> 1;
        if (delta_at(k, mm, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    const uint32_t p = static_cast<uint32_t>(dnode - 1);
    if (first) first[i] = static_cast<uint32_t>(min(i, j));
    if (last) last[i] = static_cast<uint32_t>(max(i, j));
    if (split) split[i] = static_cast<uint32_t>(gamma);
    plen[i] = p;
    if (whole) whole[i] = p % 3 == 0 ? 1u : 0u;
}

__device__ __forceinline__ int span_level(uint64_t delta) { return kL - (63 - clz64(delta)) / 3; }

__device__ __forceinline__ uint64_t prefix_node(uint64_t key, uint32_t plen) {
    return (1ull << plen) | (plen ? key >> (63 - plen) : 0ull);
}

// Linked path: internal node keys at their scan slots, leaf keys after the
// n_int internal ones (n_int = slot[m - 1], the flags' total).
__global__ __launch_bounds__(kRBlock) void radix_extract_kernel(const uint64_t* __restrict__ K, uint32_t m,
                                                                const uint32_t* __restrict__ plen,
                                                                const uint32_t* __restrict__ whole,
                                                                const uint32_t* __restrict__ slot,
                                                                uint64_t* __restrict__ nk) {
    const uint32_t i = blockIdx.x * kRBlock + threadIdx.x;
    if (i >= m) return;
    const uint64_t ki = K[i];
    const uint32_t n_int = m > 1 ? slot[m - 1] : 0u;
    if (i + 1 < m && whole[i]) nk[slot[i]] = prefix_node(ki, plen[i]);
    const int lv = span_level(K[i + 1] - ki);
    nk[n_int + i] = (1ull << (3 * lv)) | (ki >> (3 * (kL - lv)));
}

// Compact path, step 1: flags of the leaves that hold particles.
__global__ __launch_bounds__(kRBlock) void nonempty_kernel(const uint32_t* __restrict__ counts, uint32_t nl,
                                                           uint32_t* __restrict__ flag) {
    const uint32_t i = blockIdx.x * kRBlock + threadIdx.x;
    if (i < nl) flag[i] = counts[i] ? 1u : 0u;
}

// Step 2: their keys and leaf node keys, packed in order.
__global__ __launch_bounds__(kRBlock) void compact_leaves_kernel(const uint64_t* __restrict__ K, uint32_t nl,
                                                                 const uint32_t* __restrict__ flag,
                                                                 const uint32_t* __restrict__ pos,
                                                                 uint64_t* __restrict__ ck,
                                                                 uint64_t* __restrict__ cleaf) {
    const uint32_t i = blockIdx.x * kRBlock + threadIdx.x;
    if (i >= nl || !flag[i]) return;
    const uint64_t ki = K[i];
    const int lv = span_level(K[i + 1] - ki);
    ck[pos[i]] = ki;
    cleaf[pos[i]] = (1ull << (3 * lv)) | (ki >> (3 * (kL - lv)));
}

// Step 4: node keys of the compact tree (internal ones at their slots, then
// the leaves, then the root if no node is the root yet).
__global__ __launch_bounds__(kRBlock) void compact_extract_kernel(const uint64_t* __restrict__ ck, uint32_t m,
                                                                  const uint64_t* __restrict__ cleaf,
                                                                  const uint32_t* __restrict__ plen,
                                                                  const uint32_t* __restrict__ whole,
                                                                  const uint32_t* __restrict__ slot, uint32_t n_int,
                                                                  uint32_t add_root, uint64_t* __restrict__ nk) {
    const uint32_t i = blockIdx.x * kRBlock + threadIdx.x;
    if (i == 0 && add_root) nk[n_int + m] = 1ull;
    if (i >= m) return;
    if (i + 1 < m && whole[i]) nk[slot[i]] = prefix_node(ck[i], plen[i]);
    nk[n_int + i] = cleaf[i];
}

// Step 6: the nearest ancestor present, searched level by level upwards.
__global__ __launch_bounds__(kRBlock) void compact_parent_kernel(const uint64_t* __restrict__ nk, uint32_t n,
                                                                 const uint32_t* __restrict__ lo,
                                                                 uint32_t* __restrict__ parent) {
    const uint32_t p = blockIdx.x * kRBlock + threadIdx.x;
    if (p >= n) return;
    const uint64_t key = nk[p];
    const int lv = (63 - clz64(key)) / 3;
    uint32_t par = 0xffffffffu;
    for (int up = lv - 1; up >= 0; --up) {
        const uint64_t a = key >> (3 * (lv - up));
        const uint64_t b = lo[up], e = lo[up + 1];
        const uint64_t at = lower_bound_u64(nk, b, e, a);
        if (at < e && nk[at] == a) {
            par = static_cast<uint32_t>(at);
            break;
        }
    }
    parent[p] = par;
}

struct RadixLinkWs {
    uint32_t *plen, *whole, *slot;
    uint64_t* unsorted;
    void* scan;
    size_t scan_bytes;
    void* sort;
    size_t sort_bytes, bytes;
};

RadixLinkWs carve_radix_link(void* ws, size_t m) {
    const size_t n = m + (m ? (m - 1) / 7 : 0);
    Carve c(ws);
    RadixLinkWs w{};
    w.plen = c.take<uint32_t>(m);
    w.whole = c.take<uint32_t>(m);
    w.slot = c.take<uint32_t>(m + 1);
    w.unsorted = c.take<uint64_t>(n);
    w.scan_bytes = scan_u32_workspace_bytes(m);
    w.scan = c.take<char>(w.scan_bytes);
    w.sort_bytes = sort_workspace_bytes(n, false);
    w.sort = c.take<char>(w.sort_bytes);
    w.bytes = c.off;
    return w;
}

struct CompactWs {
    uint32_t *flag, *pos, *plen, *whole, *slot;
    uint64_t *ck, *cleaf, *unsorted;
    void* scan;
    size_t scan_bytes;
    void* sort;
    size_t sort_bytes, bytes;
};

CompactWs carve_compact(void* ws, size_t nl) {
    const size_t cap = 2 * nl + 1;  // leaves, internal nodes, the root
    Carve c(ws);
    CompactWs w{};
    w.flag = c.take<uint32_t>(nl + 1);
    w.pos = c.take<uint32_t>(nl + 1);
    w.plen = c.take<uint32_t>(nl);
    w.whole = c.take<uint32_t>(nl);
    w.slot = c.take<uint32_t>(nl + 1);
    w.ck = c.take<uint64_t>(nl);
    w.cleaf = c.take<uint64_t>(nl);
    w.unsorted = c.take<uint64_t>(cap);
    w.scan_bytes = scan_u32_workspace_bytes(nl + 1);
    w.scan = c.take<char>(w.scan_bytes);
    w.sort_bytes = sort_workspace_bytes(cap, false);
    w.sort = c.take<char>(w.sort_bytes);
    w.bytes = c.off;
    return w;
}

}  // namespace

cstone_status launch_radix_tree(const uint64_t* keys, size_t m, uint32_t* first, uint32_t* last, uint32_t* split,
                                uint32_t* prefix_len, hipStream_t stream) {
    if (m >= 2)
        hipLaunchKernelGGL(radix_tree_kernel, dim3(grid_for(m - 1)), dim3(kRBlock), 0, stream, keys,
                           static_cast<uint32_t>(m), first, last, split, prefix_len, static_cast<uint32_t*>(nullptr));
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

size_t radix_link_workspace_bytes(size_t n_leaves) { return carve_radix_link(nullptr, n_leaves).bytes; }

cstone_status launch_link_radix(const uint64_t* leaves, size_t m, uint64_t* node_keys, uint32_t* child,
                                uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream) {
    RadixLinkWs w = carve_radix_link(ws, m);
    if (ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    const size_t n = m + (m - 1) / 7;
    const uint32_t um = static_cast<uint32_t>(m);
    if (m >= 2)
        hipLaunchKernelGGL(radix_tree_kernel, dim3(grid_for(m - 1)), dim3(kRBlock), 0, stream, leaves, um,
                           static_cast<uint32_t*>(nullptr), static_cast<uint32_t*>(nullptr),
                           static_cast<uint32_t*>(nullptr), w.plen, w.whole);
    // slots of the whole-digit nodes; slot[m - 1] is their number (n_i for a cornerstone array)
    if (m >= 2) {
        cstone_status st = launch_scan_u32(w.whole, m - 1, w.slot, w.scan, w.scan_bytes, stream);
        if (st != CSTONE_OK) return st;
    }
    hipLaunchKernelGGL(radix_extract_kernel, dim3(grid_for(m)), dim3(kRBlock), 0, stream, leaves, um, w.plen, w.whole,
                       w.slot, w.unsorted);
    CS_HIP(hipGetLastError());
    return launch_link_finish(w.unsorted, n, node_keys, child, level_offsets, w.sort, w.sort_bytes, stream);
}

size_t compact_octree_workspace_bytes(size_t n_leaves) { return carve_compact(nullptr, n_leaves).bytes; }

cstone_status launch_compact_octree(const uint64_t* leaves, const uint32_t* counts, size_t nl, uint64_t* node_keys,
                                    uint32_t* parent, uint32_t* level_offsets, size_t* n_nodes, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
    CompactWs w = carve_compact(ws, nl);
    if (ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    const uint32_t unl = static_cast<uint32_t>(nl);
    hipLaunchKernelGGL(nonempty_kernel, dim3(grid_for(nl)), dim3(kRBlock), 0, stream, counts, unl, w.flag);
    cstone_status st = launch_scan_u32(w.flag, nl, w.pos, w.scan, w.scan_bytes, stream);
    if (st != CSTONE_OK) return st;
    hipLaunchKernelGGL(compact_leaves_kernel, dim3(grid_for(nl)), dim3(kRBlock), 0, stream, leaves, unl, w.flag, w.pos,
                       w.ck, w.cleaf);
    uint32_t mh = 0;
    CS_HIP(hipMemcpyAsync(&mh, w.pos + nl, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    CS_HIP(hipStreamSynchronize(stream));
    const size_t m = mh;  // leaves that hold particles
    uint32_t n_int = 0, root_plen = 0xffffffffu;
    if (m >= 2) {
        hipLaunchKernelGGL(radix_tree_kernel, dim3(grid_for(m - 1)), dim3(kRBlock), 0, stream, w.ck, mh,
                           static_cast<uint32_t*>(nullptr), static_cast<uint32_t*>(nullptr),
                           static_cast<uint32_t*>(nullptr), w.plen, w.whole);
        if ((st = launch_scan_u32(w.whole, m - 1, w.slot, w.scan, w.scan_bytes, stream)) != CSTONE_OK) return st;
        CS_HIP(hipMemcpyAsync(&n_int, w.slot + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        CS_HIP(hipMemcpyAsync(&root_plen, w.plen, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));  // node 0: the root
        CS_HIP(hipStreamSynchronize(stream));
    }
    // the root is a node already if the radix root's prefix is empty, or if the
    // only leaf holding particles is the root leaf
    const bool root_present = m >= 2 ? root_plen == 0 : (m == 1 && nl == 1);
    const uint32_t add_root = root_present ? 0u : 1u;
    const size_t n = m + n_int + add_root;
    hipLaunchKernelGGL(compact_extract_kernel, dim3(grid_for(std::max<size_t>(m, 1))), dim3(kRBlock), 0, stream,
                       w.ck, mh, w.cleaf, w.plen, w.whole, w.slot, n_int, add_root, w.unsorted);
    CS_HIP(hipGetLastError());
    if ((st = launch_link_finish(w.unsorted, n, node_keys, nullptr, level_offsets, w.sort, w.sort_bytes, stream)) !=
        CSTONE_OK)
        return st;
    hipLaunchKernelGGL(compact_parent_kernel, dim3(grid_for(n)), dim3(kRBlock), 0, stream, node_keys,
                       static_cast<uint32_t>(n), level_offsets, parent);
    CS_HIP(hipGetLastError());
    CS_HIP(hipStreamSynchronize(stream));
    *n_nodes = n;
    return CSTONE_OK;
}

}  // namespace cs
