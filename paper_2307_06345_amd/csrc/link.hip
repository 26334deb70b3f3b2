// Fully linked octree (Sec. 5): node keys NK in placeholder-bit form,
// breadth-first order, child offsets CO and level offsets LO.
//
//   step 1+2  one thread per leaf i writes the leaf's node key at n_i + i and,
//             if the common prefix d of K_i and K_{i+1} is a whole number of
//             octal digits, the internal node with that prefix (the boundary
//             between its 4th and 5th child) at its rank among such boundaries;
//   step 3    radix sort of NK (keys only) gives the breadth-first order;
//   step 4    LO[l] by binary search for the first key of level l;
//   step 5    CO[p] by binary search for NK[p] << 3 within level l + 1.
//
// Internal-node slot (Eq. digitweight, with the sign of the digit weights
// reversed): if K_i's first d/3 octal digits are k_1..k_l, the boundary i is
// preceded by (i - 3 + sum_m mu(k_m)) / 7 boundaries of the same kind, with
// mu = {0,-1,-2,-3,3,2,1,0}. Counting the leaves left of the boundary: they
// fill k_m complete sibling subtrees at every level m plus 4 children of the
// node itself (7 t + 1 leaves for a subtree with t internal nodes), and every
// ancestor whose path digit is >= 4 has its own 4|5 boundary further left.
// Writing mu(k) = -k for k < 4 and 7 - k for k >= 4, sum mu equals
// 7 #{k_m >= 4} - sum k_m, which popcounts of the prefix give directly.
#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr int kLinkBlock = 256;

__device__ __forceinline__ int span_level(uint64_t delta) {
    // delta = 8^(L - level): level = L - log2(delta) / 3
    return kL - (63 - clz64(delta)) / 3;
}

__global__ __launch_bounds__(kLinkBlock) void link_nodes_kernel(const uint64_t* __restrict__ K, size_t nl,
                                                                 uint64_t* __restrict__ nk) {
    const size_t i = static_cast<size_t>(blockIdx.x) * kLinkBlock + threadIdx.x;
    if (i >= nl) return;
    const size_t ni = (nl - 1) / 7;
    const uint64_t ki = K[i];
    const uint64_t kn = K[i + 1];
    const int lv = span_level(kn - ki);
    nk[ni + i] = (1ull << (3 * lv)) | (ki >> (3 * (kL - lv)));
    const int d = clz64(ki ^ kn) - 1;  // prefix length inside the 63-bit key; -1 at the closing 8^L
    if (d >= 0 && d % 3 == 0) {
        const int l = d / 3;
        const uint64_t prefix = l ? (ki >> (63 - d)) : 0ull;
        const int p0 = __popcll(prefix & 0x1249249249249249ull);  // 1s bits of the digits
        const int p1 = __popcll(prefix & 0x2492492492492492ull);  // 2s bits
        const int p2 = __popcll(prefix & 0x4924924924924924ull);  // 4s bits
        const int64_t mu_sum = 7 * p2 - (p0 + 2 * p1 + 4 * p2);
        const int64_t slot = (static_cast<int64_t>(i) - 3 + mu_sum) / 7;
        if (slot >= 0 && slot < static_cast<int64_t>(ni)) nk[slot] = (1ull << d) | prefix;
    }
}

__global__ void level_offsets_kernel(const uint64_t* __restrict__ nk, size_t n, uint32_t* __restrict__ lo) {
    const int l = threadIdx.x;
    if (l <= kL) lo[l] = static_cast<uint32_t>(lower_bound_u64(nk, 0, n, 1ull << (3 * l)));
    if (l == kL + 1) lo[l] = static_cast<uint32_t>(n);
}

__global__ __launch_bounds__(kLinkBlock) void child_offsets_kernel(const uint64_t* __restrict__ nk, size_t n,
                                                                    const uint32_t* __restrict__ lo,
                                                                    uint32_t* __restrict__ co) {
    const size_t p = static_cast<size_t>(blockIdx.x) * kLinkBlock + threadIdx.x;
    if (p >= n) return;
    const uint64_t key = nk[p];
    const int lv = (63 - clz64(key)) / 3;
    uint32_t c = 0;
    if (lv < kL) {
        const uint64_t child = key << 3;
        const uint64_t b = lo[lv + 1], e = lo[lv + 2];
        const uint64_t at = lower_bound_u64(nk, b, e, child);
        if (at < e && nk[at] == child) c = static_cast<uint32_t>(at);
    }
    co[p] = c;
}

}  // namespace

size_t link_workspace_bytes(size_t n_leaves) {
    const size_t n = n_leaves + (n_leaves ? (n_leaves - 1) / 7 : 0);
    Carve c(nullptr);
    c.take<uint64_t>(n);
    return c.off + sort_workspace_bytes(n, false);
}

cstone_status launch_link(const uint64_t* leaves, size_t nl, uint64_t* node_keys, uint32_t* child,
                          uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (ws_bytes < link_workspace_bytes(nl)) return CSTONE_ERR_INVALID_ARG;
    const size_t n = nl + (nl - 1) / 7;
    Carve c(ws);
    uint64_t* unsorted = c.take<uint64_t>(n);
    void* sort_ws = static_cast<char*>(ws) + c.off;
    hipLaunchKernelGGL(link_nodes_kernel, dim3((nl + kLinkBlock - 1) / kLinkBlock), dim3(kLinkBlock), 0, stream,
                       leaves, nl, unsorted);
    CS_HIP(hipGetLastError());
    // placeholder keys use up to 64 bits (level 21 sets bit 63)
    cstone_status s = launch_sort(unsorted, node_keys, nullptr, n, 64, sort_ws, ws_bytes - c.off, stream);
    if (s != CSTONE_OK) return s;
    hipLaunchKernelGGL(level_offsets_kernel, dim3(1), dim3(64), 0, stream, node_keys, n, level_offsets);
    hipLaunchKernelGGL(child_offsets_kernel, dim3((n + kLinkBlock - 1) / kLinkBlock), dim3(kLinkBlock), 0, stream,
                       node_keys, n, level_offsets, child);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace cs
