// Fully linked octree (Sec. 5): node keys NK in placeholder-bit form,
// breadth-first order, child offsets CO and level offsets LO.
//
// Two paths with identical outputs. launch_link places every node at its
// breadth-first index directly (see "breadth-first placement" below).
// launch_link_by_sort follows the five steps of Sec. 5:
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
#include <algorithm>

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

// ---- breadth-first placement without sorting ---------------------------------
//
// Every node starts at exactly one leaf: its first one. Leaf j starts the
// nodes of levels a_j + 1 .. lambda_j, where lambda_j is its own level and a_j
// the level of its deepest common ancestor with leaf j - 1 (a_0 = -1), and in
// breadth-first order the nodes of one level are in leaf order. So node (l, j)
// sits at LO[l] + #{j' < j : a_j' < l <= lambda_j'}, and its first child is
// node (l + 1, j), started by the same leaf. One counting pass, a scan per
// level over the tiles, and one writing pass replace steps 3-5.

constexpr int kLevels = kL + 1;
constexpr int kBfBlock = 256;
constexpr int kBfItems = 4;
constexpr int kBfTile = kBfBlock * kBfItems;
constexpr int kBfWaves = kBfBlock / kWave;

struct LeafLevels {
    int a[kBfItems];
    int lam[kBfItems];
    uint64_t k[kBfItems];  // the keys themselves
};

__device__ __forceinline__ LeafLevels leaf_levels(const uint64_t* __restrict__ K, size_t nl, size_t first) {
    // K[first - 1 .. first + kBfItems] (K holds nl + 1 keys), every load in flight at once; an
    // index outside 0 .. nl reads a key that is not used
    uint64_t kv[kBfItems + 2];
#pragma unroll
    for (int t = 0; t < kBfItems + 2; ++t) {
        const size_t raw = first + t;  // key raw - 1
        kv[t] = K[raw == 0 ? 0 : min(raw - 1, nl)];
    }
    LeafLevels r;
#pragma unroll
    for (int it = 0; it < kBfItems; ++it) {
        const size_t j = first + it;
        r.a[it] = 0;
        r.lam[it] = -1;  // no levels for padding items
        r.k[it] = kv[it + 1];
        if (j < nl) {
            const uint64_t kj = kv[it + 1];
            r.lam[it] = span_level(kv[it + 2] - kj);
            r.a[it] = j ? (clz64(kv[it] ^ kj) - 1) / 3 : -1;
        }
    }
    return r;
}

// Wave total of a per-lane count v < 8, and this lane's exclusive prefix of
// it, from its three bit planes: three ballots and bit counts instead of a
// chain of cross-lane shuffles.
static_assert(kBfItems < 8, "a lane's count of one level fits in three bits");
__device__ __forceinline__ uint32_t wave_count_total(uint32_t v) {
    return static_cast<uint32_t>(__popcll(__ballot(v & 1u))) + 2u * static_cast<uint32_t>(__popcll(__ballot(v & 2u))) +
           4u * static_cast<uint32_t>(__popcll(__ballot(v & 4u)));
}
__device__ __forceinline__ uint32_t wave_count_prefix(uint32_t v, uint32_t* total) {
    const uint64_t b0 = __ballot(v & 1u), b1 = __ballot(v & 2u), b2 = __ballot(v & 4u);
    *total = static_cast<uint32_t>(__popcll(b0)) + 2u * static_cast<uint32_t>(__popcll(b1)) +
             4u * static_cast<uint32_t>(__popcll(b2));
    return lanes_below(b0) + 2u * lanes_below(b1) + 4u * lanes_below(b2);
}

__device__ __forceinline__ uint32_t level_count(const LeafLevels& r, int l) {
    uint32_t c = 0;
#pragma unroll
    for (int it = 0; it < kBfItems; ++it) c += (r.a[it] < l && l <= r.lam[it]) ? 1u : 0u;
    return c;
}

// Per tile and level: number of nodes the tile's leaves start (level-major,
// row stride `stride` tiles). The leaf count comes from nl_dev if set.
__global__ __launch_bounds__(kBfBlock) void bf_count_kernel(const uint64_t* __restrict__ K, const uint64_t* nl_dev,
                                                            size_t nl_host, uint32_t* __restrict__ tile_counts,
                                                            uint32_t stride) {
    __shared__ uint32_t wtot[kLevels][kBfWaves];
    const size_t nl = nl_dev ? *nl_dev : nl_host;
    const uint32_t tiles = static_cast<uint32_t>((nl + kBfTile - 1) / kBfTile);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    for (uint32_t tile = blockIdx.x; tile < tiles && tile < stride; tile += gridDim.x) {
        const LeafLevels r = leaf_levels(K, nl, static_cast<size_t>(tile) * kBfTile + threadIdx.x * kBfItems);
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            const uint32_t s = wave_count_total(level_count(r, l));
            if (lane_id() == 0) wtot[l][wave] = s;
        }
        __syncthreads();
        if (threadIdx.x < kLevels) {
            uint32_t s = 0;
#pragma unroll
            for (int w = 0; w < kBfWaves; ++w) s += wtot[threadIdx.x][w];
            tile_counts[static_cast<size_t>(threadIdx.x) * stride + tile] = s;
        }
        __syncthreads();
    }
}

// One block per level: exclusive scan over the tiles, in place; level totals.
__global__ __launch_bounds__(kBfBlock) void bf_scan_kernel(uint32_t* __restrict__ tile_counts, const uint64_t* nl_dev,
                                                           size_t nl_host, uint32_t stride,
                                                           uint32_t* __restrict__ totals) {
    __shared__ uint32_t tmp[kBfWaves];
    const size_t nl = nl_dev ? *nl_dev : nl_host;
    const uint32_t tiles = min(static_cast<uint32_t>((nl + kBfTile - 1) / kBfTile), stride);
    uint32_t* row = tile_counts + static_cast<size_t>(blockIdx.x) * stride;
    uint32_t carry = 0;
    for (uint32_t base = 0; base < tiles; base += kBfBlock) {
        const uint32_t t = base + threadIdx.x;
        const uint32_t v = t < tiles ? row[t] : 0u;
        uint32_t sum;
        const uint32_t ex = block_exclusive_sum<uint32_t, kBfBlock>(v, tmp, &sum);
        if (t < tiles) row[t] = carry + ex;
        carry += sum;
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = carry;
}

__global__ __launch_bounds__(kBfBlock, 5) void bf_write_kernel(const uint64_t* __restrict__ K, const uint64_t* nl_dev,
                                                            size_t nl_host, const uint32_t* __restrict__ tile_offsets,
                                                            uint32_t stride, const uint32_t* __restrict__ totals,
                                                            uint64_t* __restrict__ nk, uint32_t* __restrict__ co,
                                                            uint32_t* __restrict__ lo_out) {
    __shared__ uint32_t lo[kLevels + 1];
    __shared__ uint32_t wtot[kLevels][kBfWaves];
    __shared__ uint32_t run[kLevels][kBfBlock];  // next index per level for each thread
    const size_t nl = nl_dev ? *nl_dev : nl_host;
    const size_t n = nl + (nl - 1) / 7;
    const uint32_t tiles = static_cast<uint32_t>((nl + kBfTile - 1) / kBfTile);
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform
    if (tid < kWave) {  // LO: exclusive scan of the level totals
        const uint32_t v = tid < kLevels ? totals[tid] : 0u;
        const uint32_t inc = wave_inclusive_sum(v);
        if (tid <= kLevels) lo[tid] = inc - v;
        if (blockIdx.x == 0 && tid <= kLevels) lo_out[tid] = tid < kLevels ? inc - v : static_cast<uint32_t>(n);
    }
    for (uint32_t tile = blockIdx.x; tile < tiles && tile < stride; tile += gridDim.x) {
        const size_t first = static_cast<size_t>(tile) * kBfTile + tid * kBfItems;
        const LeafLevels r = leaf_levels(K, nl, first);
        uint32_t ex[kLevels];  // this lane's exclusive prefix in its wave, per level
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            uint32_t total;
            ex[l] = wave_count_prefix(level_count(r, l), &total);
            if (lane_id() == 0) wtot[l][wave] = total;
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            uint32_t before = 0;
#pragma unroll
            for (int w = 0; w < kBfWaves; ++w) before += w < static_cast<int>(wave) ? wtot[l][w] : 0u;
            run[l][tid] = lo[l] + tile_offsets[static_cast<size_t>(l) * stride + tile] + before + ex[l];
        }
        // each thread only touches its own column of run[][]
#pragma unroll
        for (int it = 0; it < kBfItems; ++it) {
            const size_t j = first + it;
            if (j >= nl) continue;
            const uint64_t kj = r.k[it];
            for (int l = r.a[it] + 1; l <= r.lam[it]; ++l) {
                const uint32_t p = run[l][tid]++;
                if (p >= n) continue;  // always in range for a cornerstone array; guards memory
                nk[p] = (1ull << (3 * l)) | (kj >> (3 * (kL - l)));
                co[p] = l < r.lam[it] ? run[l + 1][tid] : 0u;
            }
        }
        __syncthreads();
    }
}

// ---- batched link: the back-to-back arrays of many sets ------------------------
//
// The same placement per set: node (l, j) of set s sits at
// LO_s[l] + #{leaves j' < j of set s starting a node of level l}. The counts
// and the per-level scan run over all entries at once (a closing entry starts
// no node, the first leaf of a set has a = -1); subtracting the running count
// at the set's first entry makes them relative to the set.

__device__ __forceinline__ LeafLevels entry_levels(const uint64_t* __restrict__ K, size_t M, size_t first) {
    // K[first - 1 .. first + kBfItems], every load in flight at once; an index outside
    // 0 .. M - 1 reads a key that is not used (M >= 1 whenever a thread has an entry)
    uint64_t kv[kBfItems + 2];
#pragma unroll
    for (int t = 0; t < kBfItems + 2; ++t) {
        const size_t raw = first + t;  // entry raw - 1
        kv[t] = M ? K[raw == 0 ? 0 : min(raw - 1, M - 1)] : 0ull;
    }
    LeafLevels r;
#pragma unroll
    for (int it = 0; it < kBfItems; ++it) {
        const size_t j = first + it;
        r.a[it] = 0;
        r.lam[it] = -1;
        r.k[it] = kv[it + 1];
        if (j < M) {
            const uint64_t kj = kv[it + 1];
            if (kj != kKeyEnd) {
                r.lam[it] = span_level(kv[it + 2] - kj);
                r.a[it] = kj == 0 ? -1 : (clz64(kv[it] ^ kj) - 1) / 3;
            }
        }
    }
    return r;
}

struct BatchSrc {
    const uint64_t* K;
    const uint32_t* sid;
    const uint32_t* starts;
    size_t M;
};

__device__ __forceinline__ BatchSrc batch_src(const BatchTreeView& v) {
    const int b = v.st->final_last & 1u;
    return {v.K[b], v.sid[b], v.starts[b], v.st->final_nl};
}

__global__ __launch_bounds__(kBfBlock) void batch_bf_count_kernel(BatchTreeView view,
                                                                  uint32_t* __restrict__ tile_counts,
                                                                  uint32_t stride) {
    __shared__ uint32_t wtot[kLevels][kBfWaves];
    const BatchSrc src = batch_src(view);
    const uint32_t tiles = static_cast<uint32_t>((src.M + kBfTile - 1) / kBfTile);
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    for (uint32_t tile = blockIdx.x; tile < tiles && tile < stride; tile += gridDim.x) {
        const LeafLevels r =
            entry_levels(src.K, src.M, static_cast<size_t>(tile) * kBfTile + threadIdx.x * kBfItems);
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            const uint32_t sum = wave_count_total(level_count(r, l));
            if (lane_id() == 0) wtot[l][wave] = sum;
        }
        __syncthreads();
        if (threadIdx.x < kLevels) {
            uint32_t sum = 0;
#pragma unroll
            for (int w = 0; w < kBfWaves; ++w) sum += wtot[threadIdx.x][w];
            tile_counts[static_cast<size_t>(threadIdx.x) * stride + tile] = sum;
        }
        __syncthreads();
    }
}

// Running count of level-l node starts before entry b (the scan gives it per
// tile; the entries of b's tile before b are counted here). One wave per call.
__device__ __forceinline__ void running_counts(const BatchSrc& src, const uint32_t* __restrict__ tile_offsets,
                                               uint32_t stride, const uint32_t* __restrict__ totals, size_t b,
                                               uint32_t* g) {
    const uint32_t lane = lane_id();
    uint32_t c[kLevels];
#pragma unroll
    for (int l = 0; l < kLevels; ++l) c[l] = 0;
    const size_t tile = b / kBfTile;
    if (b < src.M) {
        for (size_t e = tile * kBfTile + lane; e < b; e += kWave) {
            const uint64_t ke = src.K[e];
            if (ke == kKeyEnd) continue;
            const int lam = span_level(src.K[e + 1] - ke);
            const int a = ke == 0 ? -1 : (clz64(src.K[e - 1] ^ ke) - 1) / 3;
#pragma unroll
            for (int l = 0; l < kLevels; ++l) c[l] += (a < l && l <= lam) ? 1u : 0u;
        }
    }
#pragma unroll
    for (int l = 0; l < kLevels; ++l) {
        const uint32_t part = wave_sum<uint32_t>(c[l]);
        g[l] = b < src.M ? tile_offsets[static_cast<size_t>(l) * stride + tile] + part : totals[l];
    }
}

// Per set: level offsets LO_s and rel[s][l] = LO_s[l] - (running count at the set's first entry).
__global__ __launch_bounds__(kBfBlock) void batch_bf_base_kernel(BatchTreeView view, uint32_t n_sets,
                                                                 const uint32_t* __restrict__ tile_offsets,
                                                                 uint32_t stride, const uint32_t* __restrict__ totals,
                                                                 uint32_t* __restrict__ rel,
                                                                 uint32_t* __restrict__ level_offsets) {
    const BatchSrc src = batch_src(view);
    const uint32_t s = blockIdx.x * kBfWaves + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (s >= n_sets || src.M == 0) return;
    uint32_t g0[kLevels], g1[kLevels];
    running_counts(src, tile_offsets, stride, totals, src.starts[s], g0);
    running_counts(src, tile_offsets, stride, totals, src.starts[s + 1], g1);
    if (lane_id() == 0) {
        uint32_t lo = 0;
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            level_offsets[static_cast<size_t>(s) * (kLevels + 1) + l] = lo;
            rel[static_cast<size_t>(s) * kLevels + l] = lo - g0[l];
            lo += g1[l] - g0[l];
        }
        level_offsets[static_cast<size_t>(s) * (kLevels + 1) + kLevels] = lo;
    }
}

__global__ __launch_bounds__(kBfBlock) void batch_bf_write_kernel(BatchTreeView view,
                                                                  const BatchSet* __restrict__ sets,
                                                                  const uint32_t* __restrict__ tile_offsets,
                                                                  uint32_t stride, const uint32_t* __restrict__ rel,
                                                                  uint64_t* __restrict__ nk,
                                                                  uint32_t* __restrict__ co) {
    __shared__ uint32_t wtot[kLevels][kBfWaves];
    __shared__ uint32_t run[kLevels][kBfBlock];
    const BatchSrc src = batch_src(view);
    const uint32_t tiles = static_cast<uint32_t>((src.M + kBfTile - 1) / kBfTile);
    const uint32_t tid = threadIdx.x;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform
    for (uint32_t tile = blockIdx.x; tile < tiles && tile < stride; tile += gridDim.x) {
        const size_t first = static_cast<size_t>(tile) * kBfTile + tid * kBfItems;
        const LeafLevels r = entry_levels(src.K, src.M, first);
        uint32_t ex[kLevels];  // this lane's exclusive prefix in its wave, per level
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            uint32_t total;
            ex[l] = wave_count_prefix(level_count(r, l), &total);
            if (lane_id() == 0) wtot[l][wave] = total;
        }
        __syncthreads();
#pragma unroll
        for (int l = 0; l < kLevels; ++l) {
            uint32_t before = 0;
#pragma unroll
            for (int w = 0; w < kBfWaves; ++w) before += w < static_cast<int>(wave) ? wtot[l][w] : 0u;
            run[l][tid] = tile_offsets[static_cast<size_t>(l) * stride + tile] + before + ex[l];
        }
        // a thread's entries nearly always share one set: its node region is
        // read once per set, not per entry
        uint32_t cur = 0xffffffffu;
        uint64_t node_off = 0, node_cap = 0;
        const uint32_t* rs = rel;
#pragma unroll
        for (int it = 0; it < kBfItems; ++it) {
            const size_t j = first + it;
            if (j >= src.M || r.lam[it] < 0) continue;
            const uint64_t kj = r.k[it];
            const uint32_t s = src.sid[j];
            if (s != cur) {
                cur = s;
                node_off = sets[s].node_off;
                node_cap = sets[s].node_cap;
                rs = rel + static_cast<size_t>(s) * kLevels;
            }
            for (int l = r.a[it] + 1; l <= r.lam[it]; ++l) {
                const uint32_t p = rs[l] + run[l][tid]++;  // index within the set's node array
                if (p >= node_cap) continue;              // never for a cornerstone array; guards memory
                nk[node_off + p] = (1ull << (3 * l)) | (kj >> (3 * (kL - l)));
                co[node_off + p] = l < r.lam[it] ? rs[l + 1] + run[l + 1][tid] : 0u;
            }
        }
        __syncthreads();
    }
}

}  // namespace

size_t link_batch_workspace_bytes(uint32_t n_sets, size_t C) {
    Carve b(nullptr);
    b.take<uint32_t>(static_cast<size_t>(kLevels) * ((C + 1 + kBfTile - 1) / kBfTile));
    b.take<uint32_t>(kLevels);
    b.take<uint32_t>(static_cast<size_t>(n_sets) * kLevels);
    return b.off;
}

cstone_status launch_link_batch(const BatchTreeView& view, const BatchSet* sets, uint32_t n_sets, size_t C,
                                uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets, void* ws,
                                size_t ws_bytes, hipStream_t stream) {
    if (ws_bytes < link_batch_workspace_bytes(n_sets, C)) return CSTONE_ERR_INVALID_ARG;
    if (n_sets == 0) return CSTONE_OK;
    const uint32_t stride = static_cast<uint32_t>((C + 1 + kBfTile - 1) / kBfTile);
    Carve c(ws);
    uint32_t* tile_counts = c.take<uint32_t>(static_cast<size_t>(kLevels) * stride);
    uint32_t* totals = c.take<uint32_t>(kLevels);
    uint32_t* rel = c.take<uint32_t>(static_cast<size_t>(n_sets) * kLevels);
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(stride, 2048));
    hipLaunchKernelGGL(batch_bf_count_kernel, dim3(grid), dim3(kBfBlock), 0, stream, view, tile_counts, stride);
    hipLaunchKernelGGL(bf_scan_kernel, dim3(kLevels), dim3(kBfBlock), 0, stream, tile_counts, &view.st->final_nl,
                       static_cast<size_t>(0), stride, totals);
    hipLaunchKernelGGL(batch_bf_base_kernel, dim3((n_sets + kBfWaves - 1) / kBfWaves), dim3(kBfBlock), 0, stream,
                       view, n_sets, tile_counts, stride, totals, rel, level_offsets);
    hipLaunchKernelGGL(batch_bf_write_kernel, dim3(grid), dim3(kBfBlock), 0, stream, view, sets, tile_counts,
                       stride, rel, node_keys, child);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

size_t link_workspace_bytes(size_t n_leaves) {
    const size_t n = n_leaves + (n_leaves ? (n_leaves - 1) / 7 : 0);
    Carve c(nullptr);
    c.take<uint64_t>(n);
    const size_t by_sort = c.off + sort_workspace_bytes(n, false);
    Carve b(nullptr);
    b.take<uint32_t>(static_cast<size_t>(kLevels) * ((n_leaves + kBfTile - 1) / kBfTile));
    b.take<uint32_t>(kLevels);
    return std::max(by_sort, b.off);
}

cstone_status launch_link(const uint64_t* leaves, size_t nl, const uint64_t* nl_dev, uint64_t* node_keys,
                          uint32_t* child, uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (ws_bytes < link_workspace_bytes(nl)) return CSTONE_ERR_INVALID_ARG;
    const uint32_t stride = static_cast<uint32_t>((nl + kBfTile - 1) / kBfTile);  // tiles of the largest array
    Carve c(ws);
    uint32_t* tile_counts = c.take<uint32_t>(static_cast<size_t>(kLevels) * stride);
    uint32_t* totals = c.take<uint32_t>(kLevels);
    const uint32_t grid = std::max<uint32_t>(1, std::min<uint32_t>(stride, 2048));
    hipLaunchKernelGGL(bf_count_kernel, dim3(grid), dim3(kBfBlock), 0, stream, leaves, nl_dev, nl, tile_counts,
                       stride);
    hipLaunchKernelGGL(bf_scan_kernel, dim3(kLevels), dim3(kBfBlock), 0, stream, tile_counts, nl_dev, nl, stride,
                       totals);
    hipLaunchKernelGGL(bf_write_kernel, dim3(grid), dim3(kBfBlock), 0, stream, leaves, nl_dev, nl, tile_counts, stride,
                       totals, node_keys, child, level_offsets);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

cstone_status launch_link_finish(const uint64_t* unsorted, size_t n, uint64_t* node_keys, uint32_t* child,
                                 uint32_t* level_offsets, void* sort_ws, size_t sort_ws_bytes, hipStream_t stream) {
    // placeholder keys use up to 64 bits (level 21 sets bit 63)
    cstone_status s = launch_sort(unsorted, node_keys, nullptr, n, 64, sort_ws, sort_ws_bytes, stream);
    if (s != CSTONE_OK) return s;
    hipLaunchKernelGGL(level_offsets_kernel, dim3(1), dim3(64), 0, stream, node_keys, n, level_offsets);
    if (child)
        hipLaunchKernelGGL(child_offsets_kernel, dim3((n + kLinkBlock - 1) / kLinkBlock), dim3(kLinkBlock), 0, stream,
                           node_keys, n, level_offsets, child);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

cstone_status launch_link_by_sort(const uint64_t* leaves, size_t nl, uint64_t* node_keys, uint32_t* child,
                                  uint32_t* level_offsets, void* ws, size_t ws_bytes, hipStream_t stream) {
    if (ws_bytes < link_workspace_bytes(nl)) return CSTONE_ERR_INVALID_ARG;
    const size_t n = nl + (nl - 1) / 7;
    Carve c(ws);
    uint64_t* unsorted = c.take<uint64_t>(n);
    void* sort_ws = static_cast<char*>(ws) + c.off;
    hipLaunchKernelGGL(link_nodes_kernel, dim3((nl + kLinkBlock - 1) / kLinkBlock), dim3(kLinkBlock), 0, stream,
                       leaves, nl, unsorted);
    CS_HIP(hipGetLastError());
    return launch_link_finish(unsorted, n, node_keys, child, level_offsets, sort_ws, ws_bytes - c.off, stream);
}

}  // namespace cs
