// The replicated tree of particles spread over several ranks (Sec. 6),
// emulated on one GPU, and the partition of its leaves into rank domains.
//
// The particles are split into G shards (contiguous ranges of the input), as
// ranks would hold them; each shard's keys are sorted on their own. A round
// then applies f to every shard (Eq. histogram against the shard's own sorted
// keys), sums the G count arrays element by element (f_r, the reduction that
// a collective over the ranks performs; here one kernel), and applies
// g = g3 . g2 . g1 to the summed counts, which every rank would do
// identically. Rounds repeat until no leaf changes. Since the counts of the
// union are the sums of the shards' counts, the result is the tree of all
// particles, bit for bit.
//
// The same rounds build the tree focused on a range F of the curve (Sec. 7):
// with one shard, and g1 replaced by g^LE_1, which splits a leaf over N_crit
// only if it fails the minimum-distance MAC against F and also merges a group
// of 8 sibling leaves whose parent passes it. The MAC of a node is evaluated
// against F cut into maximal aligned key blocks (at most 2 x 7 per level),
// whose grid boxes the host computes once and the kernel holds in LDS.
//
// The partition (Sec. 6) groups the leaves into n_ranks bins of consecutive
// leaves with about N / n_ranks particles each: bin r starts at the first
// leaf boundary whose particle prefix reaches r N / n_ranks.
#include <algorithm>
#include <cmath>

#include "common.hpp"
#include "hilbert.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr int kGBlock = 256;

// f on every shard: Ng[g * nl + i] = particles of shard g in leaf i.
__global__ __launch_bounds__(kGBlock) void shard_counts_kernel(const uint64_t* __restrict__ P,
                                                               const uint64_t* __restrict__ shard_off, uint32_t G,
                                                               const uint64_t* __restrict__ K, uint32_t nl,
                                                               uint32_t* __restrict__ Ng) {
    const size_t t = static_cast<size_t>(blockIdx.x) * kGBlock + threadIdx.x;
    if (t >= static_cast<size_t>(G) * nl) return;
    const uint32_t g = static_cast<uint32_t>(t / nl), i = static_cast<uint32_t>(t % nl);
    const uint64_t a = shard_off[g], b = shard_off[g + 1];
    const uint64_t lo = lower_bound_u64(P, a, b, K[i]);
    const uint64_t hi = lower_bound_u64(P, lo, b, K[i + 1]);
    Ng[t] = static_cast<uint32_t>(hi - lo);
}

// f_r: N[i] = sum over the shards of Ng[g * nl + i].
__global__ __launch_bounds__(kGBlock) void shard_reduce_kernel(const uint32_t* __restrict__ Ng, uint32_t G,
                                                               uint32_t nl, uint32_t* __restrict__ N) {
    const uint32_t i = blockIdx.x * kGBlock + threadIdx.x;
    if (i >= nl) return;
    uint32_t sum = 0;
    for (uint32_t g = 0; g < G; ++g) sum += Ng[static_cast<size_t>(g) * nl + i];
    N[i] = sum;
}

// Minimum-distance MAC of the node (corner, edge) against the focus blocks:
// fails iff some block lies within l / theta, tested as r^2 theta^2 <= l^2
// with r^2 exact (integer grid) and one rounding in the product.
__device__ __forceinline__ bool mac_fails_dev(const uint32_t c[3], uint32_t edge, const uint4* blocks,
                                              uint32_t nblocks, double theta2) {
    const double l2 = static_cast<double>(edge) * static_cast<double>(edge);
    for (uint32_t b = 0; b < nblocks; ++b) {
        const uint4 f = blocks[b];
        const uint32_t fl[3] = {f.x, f.y, f.z};
        uint64_t r2 = 0;
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int64_t a0 = c[d], a1 = static_cast<int64_t>(c[d]) + edge;
            const int64_t b0 = fl[d], b1 = static_cast<int64_t>(fl[d]) + f.w;
            const int64_t gap = b0 > a1 ? b0 - a1 : (a0 > b1 ? a0 - b1 : 0);
            r2 += static_cast<uint64_t>(gap * gap);
        }
        if (!(static_cast<double>(r2) * theta2 > l2)) return true;
    }
    return false;
}

struct FocusSpec {
    const uint4* blocks;  // {corner x, y, z, edge} of the focus blocks
    uint32_t nblocks;
    int curve;
    double theta2;
};

constexpr uint32_t kMaxFocusBlocks = 320;  // 2 x 7 x 21 = 294 at most

__device__ __forceinline__ int level_of_delta(uint64_t delta) {  // delta = 8^(L - level)
    return kL - (63 - clz64(delta)) / 3;
}

// g1 (Eq. g1 with a leaf of span 1 never split, the root never merged and a
// merge iff the 8 siblings' counts sum to at most n_crit), or with FOCUS
// g^LE_1: a split also needs the leaf to fail the MAC, and a complete sibling
// group also merges if its parent passes it. O[i] in {8, 0, 1}, O[nl] = 0;
// *changed set if some O[i] != 1.
template <bool FOCUS>
__global__ __launch_bounds__(kGBlock) void global_decide_kernel(const uint64_t* __restrict__ K,
                                                                const uint32_t* __restrict__ N, uint32_t nl,
                                                                uint32_t n_crit, uint32_t* __restrict__ O,
                                                                uint32_t* changed, FocusSpec focus) {
    __shared__ uint4 fb[FOCUS ? kMaxFocusBlocks : 1];
    __shared__ uint16_t dec[FOCUS ? kStates * 8 : 1];
    if constexpr (FOCUS) {
        for (uint32_t b = threadIdx.x; b < focus.nblocks; b += kGBlock) fb[b] = focus.blocks[b];
        for (uint32_t e = threadIdx.x; e < kStates * 8; e += kGBlock) dec[e] = kHilbertDecode.dec[e];
        __syncthreads();
    }
    const uint32_t i = blockIdx.x * kGBlock + threadIdx.x;
    if (i > nl) return;
    if (i == nl) {
        O[nl] = 0;
        return;
    }
    const uint64_t k = K[i], delta = K[i + 1] - k;
    uint32_t op = 1;
    bool split = N[i] > n_crit && delta > 1;
    if constexpr (FOCUS) {
        if (split) {
            uint32_t c[3];
            const int level = level_of_delta(delta);
            node_corner(k, level, focus.curve, dec, c);
            split = mac_fails_dev(c, 1u << (kL - level), fb, focus.nblocks, focus.theta2);
        }
    }
    if (split) {
        op = 8;
    } else if (delta < kKeyEnd) {
        const uint64_t j = (k % (8 * delta)) / delta;  // place among the siblings
        if (j >= 1 && i >= j && i - j + 8 <= nl && K[i - j] + 8 * delta == K[i - j + 8]) {
            uint64_t group = 0;
            for (uint32_t m = 0; m < 8; ++m) group += N[i - j + m];
            bool merge = group <= n_crit;
            if constexpr (FOCUS) {
                if (!merge) {  // the parent passes the MAC
                    uint32_t c[3];
                    const int plevel = level_of_delta(delta) - 1;
                    node_corner(K[i - j], plevel, focus.curve, dec, c);
                    merge = !mac_fails_dev(c, 1u << (kL - plevel), fb, focus.nblocks, focus.theta2);
                }
            }
            if (merge) op = 0;
        }
    }
    O[i] = op;
    if (__ballot(op != 1) && lane_id() == 0) atomicOr(changed, 1u);
}

// f^LE_2: the MAC of every node of a linked octree (placeholder keys), 1 if
// it fails against the focus range.
__global__ __launch_bounds__(kGBlock) void focus_mac_kernel(const uint64_t* __restrict__ NK, uint32_t n,
                                                            FocusSpec focus, uint8_t* __restrict__ fails) {
    __shared__ uint4 fb[kMaxFocusBlocks];
    __shared__ uint16_t dec[kStates * 8];
    for (uint32_t b = threadIdx.x; b < focus.nblocks; b += kGBlock) fb[b] = focus.blocks[b];
    for (uint32_t e = threadIdx.x; e < kStates * 8; e += kGBlock) dec[e] = kHilbertDecode.dec[e];
    __syncthreads();
    const uint32_t p = blockIdx.x * kGBlock + threadIdx.x;
    if (p >= n) return;
    const uint64_t key = NK[p];
    const int level = (63 - clz64(key)) / 3;
    const uint64_t start = (key ^ (1ull << (3 * level))) << (3 * (kL - level));
    uint32_t c[3];
    node_corner(start, level, focus.curve, dec, c);
    fails[p] = mac_fails_dev(c, 1u << (kL - level), fb, focus.nblocks, focus.theta2) ? 1 : 0;
}

// g3 (Eqs. rebalancecopy, rebalancesplit) into K_out, unless the new array
// (Op[nl] + 1 keys) exceeds the capacity.
__global__ __launch_bounds__(kGBlock) void global_write_kernel(const uint64_t* __restrict__ K,
                                                               const uint32_t* __restrict__ O,
                                                               const uint32_t* __restrict__ Op, uint32_t nl,
                                                               uint64_t cap, uint64_t* __restrict__ K_out) {
    const uint32_t i = blockIdx.x * kGBlock + threadIdx.x;
    if (i > nl || Op[nl] > cap) return;
    if (i == nl) {
        K_out[Op[nl]] = kKeyEnd;
        return;
    }
    const uint64_t k = K[i];
    if (O[i] == 1) {
        K_out[Op[i]] = k;
    } else if (O[i] == 8) {
        const uint64_t step = (K[i + 1] - k) / 8;
        for (uint32_t j = 0; j < 8; ++j) K_out[Op[i] + j] = k + j * step;
    }
}

// bounds[r] = min { i <= nl : S[i] * R >= r * S[nl] } for r < R, bounds[R] = nl.
__global__ __launch_bounds__(kGBlock) void partition_kernel(const uint32_t* __restrict__ S, uint32_t nl, uint32_t R,
                                                            uint32_t* __restrict__ bounds) {
    const uint32_t r = blockIdx.x * kGBlock + threadIdx.x;
    if (r > R) return;
    if (r == R) {
        bounds[R] = nl;
        return;
    }
    const uint64_t target = static_cast<uint64_t>(r) * S[nl];
    uint32_t lo = 0, hi = nl;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo) / 2;
        if (static_cast<uint64_t>(S[mid]) * R >= target)
            hi = mid;
        else
            lo = mid + 1;
    }
    bounds[r] = lo;
}

struct GlobalWs {
    uint64_t* K_alt;
    uint32_t *Ng, *N, *O, *Op, *flags;
    void* scan;
    size_t scan_bytes, bytes;
};

GlobalWs carve_global(void* ws, size_t cap, uint32_t G) {
    Carve c(ws);
    GlobalWs w{};
    w.K_alt = c.take<uint64_t>(cap + 1);
    w.Ng = c.take<uint32_t>(static_cast<size_t>(G) * cap);
    w.N = c.take<uint32_t>(cap);
    w.O = c.take<uint32_t>(cap + 1);
    w.Op = c.take<uint32_t>(cap + 1);
    w.flags = c.take<uint32_t>(2);
    w.scan_bytes = scan_u32_workspace_bytes(cap + 1);
    w.scan = c.take<char>(w.scan_bytes);
    w.bytes = c.off;
    return w;
}

uint32_t grid_of(size_t items) { return static_cast<uint32_t>(std::max<size_t>(1, (items + kGBlock - 1) / kGBlock)); }

}  // namespace

__global__ void clear_flags_kernel(uint32_t* f) { f[0] = 0; }

size_t global_rebalance_workspace_bytes(size_t leaf_capacity, uint32_t G) {
    return carve_global(nullptr, leaf_capacity, G).bytes;
}

namespace {

cstone_status run_rounds(const uint64_t* P, const uint64_t* shard_off_dev, uint32_t G, uint32_t n_crit,
                         uint64_t* leaves, size_t* n_leaves, size_t cap, uint32_t* counts, uint32_t max_iters,
                         uint32_t* iters_done, void* ws, size_t ws_bytes, const FocusSpec* focus,
                         hipStream_t stream) {
    GlobalWs w = carve_global(ws, cap, G);
    if (ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    if (max_iters == 0) max_iters = kL + 1;
    uint64_t* buf[2] = {leaves, w.K_alt};
    int cur = 0;
    size_t nl = *n_leaves;
    uint32_t rounds = 0;
    cstone_status status = CSTONE_ERR_NOT_CONVERGED;
    while (rounds < max_iters) {
        const uint32_t unl = static_cast<uint32_t>(nl);
        hipLaunchKernelGGL(clear_flags_kernel, dim3(1), dim3(1), 0, stream, w.flags);
        hipLaunchKernelGGL(shard_counts_kernel, dim3(grid_of(static_cast<size_t>(G) * nl)), dim3(kGBlock), 0, stream,
                           P, shard_off_dev, G, buf[cur], unl, w.Ng);
        hipLaunchKernelGGL(shard_reduce_kernel, dim3(grid_of(nl)), dim3(kGBlock), 0, stream, w.Ng, G, unl, w.N);
        if (focus)
            hipLaunchKernelGGL(global_decide_kernel<true>, dim3(grid_of(nl + 1)), dim3(kGBlock), 0, stream, buf[cur],
                               w.N, unl, n_crit, w.O, w.flags, *focus);
        else
            hipLaunchKernelGGL(global_decide_kernel<false>, dim3(grid_of(nl + 1)), dim3(kGBlock), 0, stream, buf[cur],
                               w.N, unl, n_crit, w.O, w.flags, FocusSpec{});
        cstone_status st = launch_scan_u32(w.O, nl, w.Op, w.scan, w.scan_bytes, stream);
        if (st != CSTONE_OK) return st;
        hipLaunchKernelGGL(global_write_kernel, dim3(grid_of(nl + 1)), dim3(kGBlock), 0, stream, buf[cur], w.O, w.Op,
                           unl, static_cast<uint64_t>(cap), buf[cur ^ 1]);
        CS_HIP(hipGetLastError());
        uint32_t host[2] = {0, 0};  // changed, new leaf count
        CS_HIP(hipMemcpyAsync(&host[0], w.flags, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        CS_HIP(hipMemcpyAsync(&host[1], w.Op + nl, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
        CS_HIP(hipStreamSynchronize(stream));
        ++rounds;
        if (!host[0]) {  // converged: the summed counts belong to the final array
            status = CSTONE_OK;
            break;
        }
        if (host[1] > cap) {
            status = CSTONE_ERR_CAPACITY;
            *n_leaves = host[1];
            break;
        }
        cur ^= 1;
        nl = host[1];
    }
    if (status == CSTONE_ERR_NOT_CONVERGED) {  // counts of the last array
        const uint32_t unl = static_cast<uint32_t>(nl);
        hipLaunchKernelGGL(shard_counts_kernel, dim3(grid_of(static_cast<size_t>(G) * nl)), dim3(kGBlock), 0, stream,
                           P, shard_off_dev, G, buf[cur], unl, w.Ng);
        hipLaunchKernelGGL(shard_reduce_kernel, dim3(grid_of(nl)), dim3(kGBlock), 0, stream, w.Ng, G, unl, w.N);
    }
    if (status != CSTONE_ERR_CAPACITY) {
        if (cur == 1) CS_HIP(hipMemcpyAsync(leaves, w.K_alt, (nl + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, stream));
        if (counts) CS_HIP(hipMemcpyAsync(counts, w.N, nl * sizeof(uint32_t), hipMemcpyDeviceToDevice, stream));
        CS_HIP(hipStreamSynchronize(stream));
        *n_leaves = nl;
    } else if (cur == 1) {  // leave the last valid array in `leaves`
        CS_HIP(hipMemcpyAsync(leaves, w.K_alt, (nl + 1) * sizeof(uint64_t), hipMemcpyDeviceToDevice, stream));
        CS_HIP(hipStreamSynchronize(stream));
    }
    if (iters_done) *iters_done = rounds;
    return status;
}

// The focus range [fa, fb) as maximal aligned key blocks, each as its grid
// box {corner x, y, z, edge}.
uint32_t focus_blocks(uint64_t fa, uint64_t fb, int curve, uint4* out) {
    uint32_t nb = 0;
    uint64_t k = fa;
    while (k < fb) {
        int e = kL;  // the block 8^e: aligned at k and ending by fb
        while (e > 0 && ((k & ((1ull << (3 * e)) - 1)) != 0 || fb - k < (1ull << (3 * e)))) --e;
        uint32_t c[3];
        node_corner(k, kL - e, curve, kHilbertDecode.dec, c);
        out[nb++] = make_uint4(c[0], c[1], c[2], 1u << e);
        k += 1ull << (3 * e);
    }
    return nb;
}

}  // namespace

cstone_status run_global_rebalance(const uint64_t* P, const uint64_t* shard_off_dev, uint32_t G, uint32_t n_crit,
                                   uint64_t* leaves, size_t* n_leaves, size_t cap, uint32_t* counts,
                                   uint32_t max_iters, uint32_t* iters_done, void* ws, size_t ws_bytes,
                                   hipStream_t stream) {
    return run_rounds(P, shard_off_dev, G, n_crit, leaves, n_leaves, cap, counts, max_iters, iters_done, ws, ws_bytes,
                      nullptr, stream);
}

size_t focus_workspace_bytes(size_t leaf_capacity) {
    Carve c(nullptr);
    c.take<uint64_t>(2);
    c.take<uint4>(kMaxFocusBlocks);
    return c.off + global_rebalance_workspace_bytes(leaf_capacity, 1);
}

cstone_status run_focus_rebalance(const uint64_t* P, size_t n, uint32_t n_crit, int curve, uint64_t fa, uint64_t fb,
                                  double theta, uint64_t* leaves, size_t* n_leaves, size_t cap, uint32_t* counts,
                                  uint32_t max_iters, uint32_t* iters_done, void* ws, size_t ws_bytes,
                                  hipStream_t stream) {
    if (ws_bytes < focus_workspace_bytes(cap)) return CSTONE_ERR_INVALID_ARG;
    Carve c(ws);
    uint64_t* off = c.take<uint64_t>(2);
    uint4* blocks = c.take<uint4>(kMaxFocusBlocks);
    const uint64_t host_off[2] = {0, n};
    uint4 host_blocks[kMaxFocusBlocks];
    FocusSpec f{};
    f.blocks = blocks;
    f.nblocks = focus_blocks(fa, fb, curve, host_blocks);
    f.curve = curve;
    f.theta2 = theta * theta;
    CS_HIP(hipMemcpyAsync(off, host_off, sizeof host_off, hipMemcpyHostToDevice, stream));
    if (f.nblocks)
        CS_HIP(hipMemcpyAsync(blocks, host_blocks, f.nblocks * sizeof(uint4), hipMemcpyHostToDevice, stream));
    return run_rounds(P, off, 1, n_crit, leaves, n_leaves, cap, counts, max_iters, iters_done,
                      static_cast<char*>(ws) + c.off, ws_bytes - c.off, &f, stream);
}

size_t focus_mac_workspace_bytes() {
    Carve c(nullptr);
    c.take<uint4>(kMaxFocusBlocks);
    return c.off;
}

cstone_status launch_focus_mac(const uint64_t* node_keys, size_t n_nodes, int curve, uint64_t fa, uint64_t fb,
                               double theta, uint8_t* fails, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (ws_bytes < focus_mac_workspace_bytes()) return CSTONE_ERR_INVALID_ARG;
    uint4 host_blocks[kMaxFocusBlocks];
    FocusSpec f{};
    f.blocks = static_cast<uint4*>(ws);
    f.nblocks = focus_blocks(fa, fb, curve, host_blocks);
    f.curve = curve;
    f.theta2 = theta * theta;
    if (f.nblocks)
        CS_HIP(hipMemcpyAsync(static_cast<uint4*>(ws), host_blocks, f.nblocks * sizeof(uint4), hipMemcpyHostToDevice,
                              stream));
    if (n_nodes)
        hipLaunchKernelGGL(focus_mac_kernel, dim3(grid_of(n_nodes)), dim3(kGBlock), 0, stream, node_keys,
                           static_cast<uint32_t>(n_nodes), f, fails);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

size_t sfc_partition_workspace_bytes(size_t n_leaves) {
    Carve c(nullptr);
    c.take<uint32_t>(n_leaves + 1);
    return c.off + scan_u32_workspace_bytes(n_leaves);
}

cstone_status launch_sfc_partition(const uint32_t* counts, size_t nl, uint32_t n_ranks, uint32_t* bounds, void* ws,
                                   size_t ws_bytes, hipStream_t stream) {
    if (ws_bytes < sfc_partition_workspace_bytes(nl)) return CSTONE_ERR_INVALID_ARG;
    Carve c(ws);
    uint32_t* S = c.take<uint32_t>(nl + 1);
    cstone_status st = launch_scan_u32(counts, nl, S, static_cast<char*>(ws) + c.off, ws_bytes - c.off, stream);
    if (st != CSTONE_OK) return st;
    hipLaunchKernelGGL(partition_kernel, dim3(grid_of(static_cast<size_t>(n_ranks) + 1)), dim3(kGBlock), 0, stream, S,
                       static_cast<uint32_t>(nl), n_ranks, bounds);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}


namespace {

// Workspace of the sharded build: unsorted keys, the shard offsets on the
// device, then the sorts (one shard at a time) or the rounds.
struct ShardedWs {
    uint64_t* keys;
    uint64_t* off;
    void* stage;
    size_t stage_bytes, bytes;
};

ShardedWs carve_sharded(void* ws, size_t n, size_t max_shard, size_t cap, uint32_t G) {
    Carve c(ws);
    ShardedWs w{};
    w.keys = c.take<uint64_t>(n);
    w.off = c.take<uint64_t>(G + 1);
    w.stage_bytes = std::max(sort_workspace_bytes(max_shard, true), cs::global_rebalance_workspace_bytes(cap, G));
    w.stage = c.take<char>(w.stage_bytes);
    w.bytes = c.off;
    return w;
}

bool offsets_ok(const uint64_t* off, uint32_t G, size_t n, size_t* max_shard) {
    if (!off || G == 0 || off[0] != 0 || off[G] != n) return false;
    size_t mx = 0;
    for (uint32_t g = 0; g < G; ++g) {
        if (off[g + 1] < off[g]) return false;
        mx = std::max<size_t>(mx, off[g + 1] - off[g]);
    }
    if (max_shard) *max_shard = mx;
    return true;
}

constexpr size_t kMaxN = 0xffffffffull;

}  // namespace
}  // namespace cs

extern "C" {

CSTONE_API size_t cstone_global_rebalance_workspace_bytes(size_t leaf_capacity, uint32_t n_shards) {
    cs::Carve c(nullptr);
    c.take<uint64_t>(static_cast<size_t>(n_shards) + 1);
    return c.off + cs::global_rebalance_workspace_bytes(leaf_capacity, n_shards);
}

CSTONE_API cstone_status cstone_global_rebalance(const uint64_t* sorted_keys, const uint64_t* shard_offsets,
                                                 uint32_t n_shards, uint32_t n_crit, uint64_t* leaves,
                                                 size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                                                 uint32_t max_iters, uint32_t* iters_done, void* ws, size_t ws_bytes,
                                                 hipStream_t stream) {
    if (n_crit == 0 || !leaves || !n_leaves || !ws || n_shards == 0 || !shard_offsets) return CSTONE_ERR_INVALID_ARG;
    const size_t n = shard_offsets[n_shards];
    if (n > cs::kMaxN || !cs::offsets_ok(shard_offsets, n_shards, n, nullptr) || (n && !sorted_keys))
        return CSTONE_ERR_INVALID_ARG;
    if (*n_leaves < 1 || *n_leaves > leaf_capacity || leaf_capacity >= cs::kMaxN) return CSTONE_ERR_INVALID_ARG;
    if (ws_bytes < cstone_global_rebalance_workspace_bytes(leaf_capacity, n_shards)) return CSTONE_ERR_INVALID_ARG;
    cs::Carve c(ws);
    uint64_t* off = c.take<uint64_t>(static_cast<size_t>(n_shards) + 1);
    CS_HIP(hipMemcpyAsync(off, shard_offsets, (static_cast<size_t>(n_shards) + 1) * sizeof(uint64_t),
                          hipMemcpyHostToDevice, stream));
    return cs::run_global_rebalance(sorted_keys, off, n_shards, n_crit, leaves, n_leaves, leaf_capacity, counts,
                                    max_iters, iters_done, static_cast<char*>(ws) + c.off, ws_bytes - c.off, stream);
}

CSTONE_API size_t cstone_build_sharded_workspace_bytes(const uint64_t* shard_offsets, uint32_t n_shards,
                                                       size_t leaf_capacity) {
    size_t mx = 0;
    if (!shard_offsets || !cs::offsets_ok(shard_offsets, n_shards, shard_offsets[n_shards], &mx)) return 0;
    return cs::carve_sharded(nullptr, shard_offsets[n_shards], mx, leaf_capacity, n_shards).bytes;
}

CSTONE_API cstone_status cstone_build_sharded(const double* x, const double* y, const double* z,
                                              const uint64_t* shard_offsets, uint32_t n_shards,
                                              const cstone_box* box, cstone_curve curve, uint32_t n_crit,
                                              uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves,
                                              size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                                              uint32_t max_iters, uint32_t* iters_done, void* ws, size_t ws_bytes,
                                              hipStream_t stream) {
    size_t mx = 0;
    if (!shard_offsets || n_shards == 0) return CSTONE_ERR_INVALID_ARG;
    const size_t n = shard_offsets[n_shards];
    if (n > cs::kMaxN || !cs::offsets_ok(shard_offsets, n_shards, n, &mx) || n_crit == 0 || !box || !leaves ||
        !n_leaves || !ws)
        return CSTONE_ERR_INVALID_ARG;
    if (n && (!x || !y || !z || !sorted_keys || !perm)) return CSTONE_ERR_INVALID_ARG;
    if (curve != CSTONE_MORTON && curve != CSTONE_HILBERT) return CSTONE_ERR_INVALID_ARG;
    if (*n_leaves < 1 || *n_leaves > leaf_capacity || leaf_capacity >= cs::kMaxN) return CSTONE_ERR_INVALID_ARG;
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(box->lo[d]) || !std::isfinite(box->hi[d]) || !(box->lo[d] < box->hi[d]))
            return CSTONE_ERR_INVALID_ARG;
    cs::ShardedWs w = cs::carve_sharded(ws, n, mx, leaf_capacity, n_shards);
    if (ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    // keys of every particle (a rank's keys depend only on its own particles),
    // with the non-finite flag in the first word of the offsets' slot, read
    // back before the offsets are copied in
    uint32_t* flag = reinterpret_cast<uint32_t*>(w.off);
    hipLaunchKernelGGL(cs::clear_flags_kernel, dim3(1), dim3(1), 0, stream, flag);
    cstone_status st = cs::launch_keys(x, y, z, n, *box, curve, w.keys, flag, stream);
    if (st != CSTONE_OK) return st;
    uint32_t host_flag = 0;
    CS_HIP(hipMemcpyAsync(&host_flag, flag, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    CS_HIP(hipStreamSynchronize(stream));
    if (host_flag & CSTONE_FLAG_NONFINITE) return CSTONE_ERR_NONFINITE;
    // every shard's keys sorted on their own (perm relative to the shard's first particle)
    for (uint32_t g = 0; g < n_shards; ++g) {
        const size_t a = shard_offsets[g], m = shard_offsets[g + 1] - a;
        if (m == 0) continue;
        st = cs::launch_sort(w.keys + a, sorted_keys + a, perm + a, m, 63, w.stage, w.stage_bytes, stream);
        if (st != CSTONE_OK) return st;
    }
    CS_HIP(hipMemcpyAsync(w.off, shard_offsets, (static_cast<size_t>(n_shards) + 1) * sizeof(uint64_t),
                          hipMemcpyHostToDevice, stream));
    return cs::run_global_rebalance(sorted_keys, w.off, n_shards, n_crit, leaves, n_leaves, leaf_capacity, counts,
                                    max_iters, iters_done, w.stage, w.stage_bytes, stream);
}

CSTONE_API size_t cstone_focus_rebalance_workspace_bytes(size_t leaf_capacity) {
    return cs::focus_workspace_bytes(leaf_capacity);
}

CSTONE_API cstone_status cstone_focus_rebalance(const uint64_t* sorted_keys, size_t n, uint32_t n_crit,
                                                cstone_curve curve, uint64_t focus_start, uint64_t focus_end,
                                                double theta, uint64_t* leaves, size_t* n_leaves,
                                                size_t leaf_capacity, uint32_t* counts, uint32_t max_iters,
                                                uint32_t* iters_done, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n > cs::kMaxN || n_crit == 0 || !leaves || !n_leaves || !ws || (n && !sorted_keys)) return CSTONE_ERR_INVALID_ARG;
    if (curve != CSTONE_MORTON && curve != CSTONE_HILBERT) return CSTONE_ERR_INVALID_ARG;
    if (!(focus_start <= focus_end && focus_end <= cs::kKeyEnd) || !(theta >= 0.0) || !std::isfinite(theta))
        return CSTONE_ERR_INVALID_ARG;
    if (*n_leaves < 1 || *n_leaves > leaf_capacity || leaf_capacity >= cs::kMaxN) return CSTONE_ERR_INVALID_ARG;
    return cs::run_focus_rebalance(sorted_keys, n, n_crit, curve, focus_start, focus_end, theta, leaves, n_leaves,
                                   leaf_capacity, counts, max_iters, iters_done, ws, ws_bytes, stream);
}

CSTONE_API size_t cstone_focus_mac_workspace_bytes(void) { return cs::focus_mac_workspace_bytes(); }

CSTONE_API cstone_status cstone_focus_mac(const uint64_t* node_keys, size_t n_nodes, cstone_curve curve,
                                          uint64_t focus_start, uint64_t focus_end, double theta, uint8_t* fails,
                                          void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n_nodes > cs::kMaxN || (n_nodes && (!node_keys || !fails)) || !ws) return CSTONE_ERR_INVALID_ARG;
    if (curve != CSTONE_MORTON && curve != CSTONE_HILBERT) return CSTONE_ERR_INVALID_ARG;
    if (!(focus_start <= focus_end && focus_end <= cs::kKeyEnd) || !(theta >= 0.0) || !std::isfinite(theta))
        return CSTONE_ERR_INVALID_ARG;
    return cs::launch_focus_mac(node_keys, n_nodes, curve, focus_start, focus_end, theta, fails, ws, ws_bytes, stream);
}

CSTONE_API size_t cstone_sfc_partition_workspace_bytes(size_t n_leaves) {
    return cs::sfc_partition_workspace_bytes(n_leaves);
}

CSTONE_API cstone_status cstone_sfc_partition(const uint32_t* counts, size_t n_leaves, uint32_t n_ranks,
                                              uint32_t* bounds, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (n_leaves < 1 || n_leaves >= cs::kMaxN || n_ranks == 0 || !counts || !bounds || !ws)
        return CSTONE_ERR_INVALID_ARG;
    return cs::launch_sfc_partition(counts, n_leaves, n_ranks, bounds, ws, ws_bytes, stream);
}

}  // extern "C"
