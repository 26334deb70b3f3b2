// Leaf counts f (Eq. histogram) and the rebalance loop g = g3.g2.g1 (Sec. 4).
//
// The loop keeps, next to the cornerstone array K, the position of every key
// of K in the sorted particle keys P (the lower bound that f computes). A
// leaf's count is the difference of two adjacent positions, and the combined
// count of 8 sibling leaves is the difference of the positions around them.
// Each round is two kernels:
//   round_kernel   g1 (decision), g2 (exclusive scan of O in one pass with a
//                  wave-wide decoupled look-back) and g3 (writing K'); copied
//                  leaves and the first child of a split keep their position,
//                  and every split leaf is appended to a list;
//   split_search   f for the next round: the 7 inner boundaries of every split
//                  leaf, searched inside that leaf's own range of P, spread
//                  over the whole GPU (one lane per search, or one wave with
//                  63 probes per step when the range is long).
// Rounds are enqueued ahead of the host's convergence check; a round that
// starts after convergence (or after a capacity overflow) exits at once, and a
// finalize kernel leaves the last complete round's array in place with its
// counts and its leaf count in device memory.
#include <algorithm>
#include <cstddef>
#include <cstring>
#include <memory>

#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr int kCountBlock = 256;
constexpr int kRBlock = 256;
constexpr int kRItems = 8;
constexpr int kRTile = kRBlock * kRItems;
constexpr uint32_t kMaxGrid = 2048;
constexpr uint32_t kSearchBlock = 256;


// ---- f as a standalone operation -----------------------------------------

__global__ __launch_bounds__(kCountBlock) void node_counts_kernel(const uint64_t* __restrict__ P, size_t n,
                                                                   const uint64_t* __restrict__ K, size_t nl,
                                                                   uint32_t* __restrict__ counts) {
    __shared__ uint32_t pos[kCountBlock + 1];
    const size_t base = static_cast<size_t>(blockIdx.x) * kCountBlock;
    const size_t i = base + threadIdx.x;
    if (i <= nl) pos[threadIdx.x] = static_cast<uint32_t>(lower_bound_u64(P, 0, n, K[i]));
    if (threadIdx.x == 0) {
        const size_t e = base + kCountBlock;
        if (e <= nl) pos[kCountBlock] = static_cast<uint32_t>(lower_bound_u64(P, 0, n, K[e]));
    }
    __syncthreads();
    if (i < nl) counts[i] = pos[threadIdx.x + 1] - pos[threadIdx.x];
}

// Positions of every key of K in P (start of the loop from a given array).
__global__ __launch_bounds__(kCountBlock) void positions_kernel(const uint64_t* __restrict__ P, size_t n,
                                                                 const uint64_t* __restrict__ K, size_t nl,
                                                                 uint32_t* __restrict__ pos) {
    const size_t i = static_cast<size_t>(blockIdx.x) * kCountBlock + threadIdx.x;
    if (i <= nl) pos[i] = static_cast<uint32_t>(lower_bound_u64(P, 0, n, K[i]));
}

// The loop's set-up, as thread t of `stride` threads.
__device__ __forceinline__ void loop_init_part(size_t t, size_t stride, LoopState* st, uint64_t nl0, uint64_t* lb,
                                               size_t lb_words, uint32_t* pos, uint32_t n, int root, uint64_t* K,
                                               const uint32_t* input_flags) {
    for (size_t i = t; i < lb_words; i += stride) lb[i] = 0;
    if (t < kMaxRounds) {
        st->changed[t] = 0;
        st->merged[t] = 0;
        st->over[t] = 0;
        st->counters[t][0] = 0;
        st->nsplit[t] = 0;
    }
    if (t <= kMaxRounds) st->nl[t] = t == 0 ? nl0 : 0;
    if (t <= kL) st->mins[t] = 0xffffffffu;
    if (t == 0) {
        st->err = 0;
        st->start_level = 0;
        st->input_flags = input_flags ? *input_flags : 0u;
        if (root) {  // the only one-leaf cornerstone array
            K[0] = 0;
            K[1] = kKeyEnd;
            pos[0] = 0;
            pos[1] = n;
        }
    }
}

__global__ __launch_bounds__(256) void loop_init_kernel(LoopState* st, uint64_t nl0, uint64_t* lb, size_t lb_words,
                                                        uint32_t* pos, uint32_t n, int root, uint64_t* K,
                                                        const uint32_t* input_flags) {
    loop_init_part(static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x,
                   static_cast<size_t>(gridDim.x) * blockDim.x, st, nl0, lb, lb_words, pos, n, root, K, input_flags);
}

// ---- an exact start from a uniform level ---------------------------------------
//
// From the root, a round splits every leaf holding more than n_crit particles
// and merges nothing (8 children hold more than n_crit together). So if every
// node of level l - 1 holds more than n_crit particles, the array after l
// rounds is the uniform grid of level l, and the loop may start there, with
// the l rounds counted. The node positions of level 3 come first (one wave per
// boundary); only if every level-2 node is over n_crit are those of a finer
// level (at most kStartFine) searched inside them, and only if every level-3
// node is over n_crit. Per-level least counts then give the deepest such l.

constexpr int kStartCoarse = 3;
constexpr int kStartFine = 6;
constexpr uint32_t kCoarseNodes = 1u << (3 * kStartCoarse);  // 512

__global__ __launch_bounds__(256) void start_coarse_kernel(const uint64_t* __restrict__ P, uint32_t n,
                                                           uint32_t* __restrict__ posc) {
    const uint32_t w = blockIdx.x * (256 / kWave) + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (w > kCoarseNodes) return;  // whole waves
    const uint64_t key = static_cast<uint64_t>(w) << (3 * (kL - kStartCoarse));  // w = 512: 8^21
    const uint32_t at = wave_lower_bound(P, 0, n, key);
    if (lane_id() == 0) posc[w] = at;
}

// One block of 512: least counts of levels 0..3 from the level-3 positions,
// and whether a start finer than level 3 is possible (every level-3 node over
// n_crit), so whether the finer positions are worth searching.
__global__ __launch_bounds__(kCoarseNodes) void start_check_kernel(const uint32_t* __restrict__ posc, uint32_t n_crit,
                                                                   int lf, LoopState* st) {
    __shared__ uint32_t red[kCoarseNodes / kWave];
    const uint32_t t = threadIdx.x;
    uint32_t lvl_min[kStartCoarse + 1];
#pragma unroll
    for (int k = 0; k <= kStartCoarse; ++k) {
        const int span = 1 << (3 * (kStartCoarse - k));  // level-3 nodes per level-k node
        uint32_t c = 0xffffffffu;
        if ((t & (span - 1)) == 0) c = posc[t + span] - posc[t];
        for (int d = 1; d < kWave; d <<= 1) c = min(c, static_cast<uint32_t>(__shfl_xor(static_cast<int>(c), d, kWave)));
        if (lane_id() == 0) red[t / kWave] = c;
        __syncthreads();
        uint32_t m = 0xffffffffu;
        for (uint32_t w = 0; w < kCoarseNodes / kWave; ++w) m = min(m, red[w]);
        lvl_min[k] = m;
        __syncthreads();
    }
    if (t == 0) {
        for (int k = 0; k <= kStartCoarse; ++k) st->mins[k] = lvl_min[k];
        st->start_fine = (lf > kStartCoarse && lvl_min[kStartCoarse] > n_crit) ? 1u : 0u;
    }
}

// Level-3 and level-lf positions from the sort's level-6 table: the first
// position at or after node j's start is that of the first non-empty level-6
// node at or after it; up to 64 entries are scanned, then P is searched.
__device__ __forceinline__ void start_table_part(uint32_t t, uint32_t stride, const uint64_t* __restrict__ P,
                                                 uint32_t n, const uint32_t* __restrict__ level6, int lf,
                                                 uint32_t* __restrict__ posc, uint32_t* __restrict__ posf) {
    const uint32_t nodes = 1u << (3 * lf);
    const int sh = 3 * (kStartFine - lf);   // level-6 nodes per level-lf node: 2^sh
    const int up = 3 * (lf - kStartCoarse);  // level-lf nodes per level-3 node: 2^up
    for (uint32_t j = t; j <= nodes; j += stride) {
        const uint32_t c0 = j << sh;
        uint32_t at = n;
        if (c0 < kLevel6Cells) {
            const uint32_t c1 = min(c0 + 64u, kLevel6Cells);
            uint32_t c = c0;
            while (c < c1 && level6[c] == kCellEmpty) ++c;
            if (c < c1)
                at = level6[c];
            else if (c < kLevel6Cells)  // a long empty run: search
                at = static_cast<uint32_t>(lower_bound_u64(P, 0, n, static_cast<uint64_t>(c0) << (3 * (kL - kStartFine))));
        }
        posf[j] = at;
        if ((j & ((1u << up) - 1)) == 0) posc[j >> up] = at;
    }
}

// The loop's set-up and the table positions in one launch (independent work).
__global__ __launch_bounds__(256) void loop_init_table_kernel(LoopState* st, uint64_t nl0, uint64_t* lb,
                                                              size_t lb_words, uint32_t* pos, uint32_t n,
                                                              const uint32_t* input_flags,
                                                              const uint64_t* __restrict__ P,
                                                              const uint32_t* __restrict__ level6, int lf,
                                                              uint32_t* __restrict__ posc,
                                                              uint32_t* __restrict__ posf) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    loop_init_part(t, stride, st, nl0, lb, lb_words, pos, n, 0, nullptr, input_flags);
    start_table_part(t, stride, P, n, level6, lf, posc, posf);
}

// Positions of the level-lf nodes: block c searches the nodes inside coarse
// node c. It first reads kFineSamples evenly spaced keys of the coarse node's
// range into LDS; each search then runs in LDS and ends with a binary search of
// P only between the two samples that bracket its key.
constexpr int kFineBlock = 256;
constexpr uint32_t kFineSamples = 1024;

__global__ __launch_bounds__(kFineBlock) void start_fine_kernel(const uint64_t* __restrict__ P,
                                                                const uint32_t* __restrict__ posc, int lf,
                                                                const LoopState* st, uint32_t* __restrict__ posf) {
    __shared__ uint64_t samp[kFineSamples];
    if (!st->start_fine) return;
    const uint32_t per = 1u << (3 * (lf - kStartCoarse));  // fine nodes per coarse node
    const uint32_t c = blockIdx.x;
    const uint32_t a = posc[c], b = posc[c + 1];
    const uint64_t len = b - a;
    const uint32_t S = static_cast<uint32_t>(min<uint64_t>(len, kFineSamples));
    // sample i sits at a + floor(len * i / S): strictly increasing, since S <= len
    for (uint32_t i = threadIdx.x; i < S; i += kFineBlock) samp[i] = P[a + len * i / S];
    __syncthreads();
    for (uint32_t t = threadIdx.x; t < per; t += kFineBlock) {
        const uint32_t j = c * per + t;
        uint32_t at = a;
        if (t != 0 && S != 0) {
            const uint64_t key = static_cast<uint64_t>(j) << (3 * (kL - lf));
            uint32_t lo = 0, hi = S;  // first sample >= key
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (samp[mid] < key)
                    lo = mid + 1;
                else
                    hi = mid;
            }
            // the answer lies after the sample below the key and at or before the one above it
            const uint64_t from = lo == 0 ? a : a + len * (lo - 1) / S + 1;
            const uint64_t to = lo == S ? b : a + len * lo / S;
            at = static_cast<uint32_t>(lower_bound_u64(P, from, to, key));
        }
        posf[j] = at;
    }
    if (c == kCoarseNodes - 1 && threadIdx.x == 0) posf[kCoarseNodes * per] = posc[kCoarseNodes];
}

// least counts of levels k0 .. lf - 1 from the finer positions (block minima,
// then one atomic per block and level). With `all` (positions from the sort's
// level-6 table, complete at every level up to lf) it covers levels 0 .. lf - 1
// and marks the start search fine; otherwise levels 4 .. lf - 1, once the
// coarse check found every level-3 node over n_crit.
__global__ __launch_bounds__(256) void start_mins_kernel(const uint32_t* __restrict__ posf, int lf, LoopState* st,
                                                         int all) {
    __shared__ uint32_t red[kStartFine][256 / kWave];
    if (!all && !st->start_fine) return;
    if (all && blockIdx.x == 0 && threadIdx.x == 0) st->start_fine = 1;
    const int k0 = all ? 0 : kStartCoarse + 1;
    const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x, stride = gridDim.x * blockDim.x;
    uint32_t c[kStartFine];
    // this thread's first node of every level, all loads in flight at once (a
    // level outside k0 .. lf - 1, or a node past the level, reads entry 0 and
    // is not counted); lf <= kStartFine
#pragma unroll
    for (int k = 0; k < kStartFine; ++k) {
        const bool lv = k >= k0 && k < lf;
        const uint32_t nodes = lv ? 1u << (3 * k) : 0u;
        const uint32_t span = lv ? 1u << (3 * (lf - k)) : 0u;
        const uint32_t u = gtid < nodes ? gtid : 0u;
        const uint32_t hi = posf[(u + 1) * span], lo = posf[u * span];
        c[k] = gtid < nodes ? hi - lo : 0xffffffffu;
    }
    // further nodes, when the grid is smaller than a level
#pragma unroll
    for (int k = 0; k < kStartFine; ++k) {
        if (k < k0 || k >= lf) continue;
        const uint32_t nodes = 1u << (3 * k), span = 1u << (3 * (lf - k));
        for (uint32_t u = gtid + stride; u < nodes; u += stride) c[k] = min(c[k], posf[(u + 1) * span] - posf[u * span]);
    }
    // wave minima of all levels together, then one barrier and one atomic per level and block
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1)
#pragma unroll
        for (int k = 0; k < kStartFine; ++k) c[k] = min(c[k], static_cast<uint32_t>(__shfl_xor(static_cast<int>(c[k]), d, kWave)));
    if (lane_id() == 0)
#pragma unroll
        for (int k = 0; k < kStartFine; ++k) red[k][threadIdx.x / kWave] = c[k];
    __syncthreads();
    if (threadIdx.x < static_cast<uint32_t>(kStartFine)) {
        const int k = static_cast<int>(threadIdx.x);
        uint32_t m = 0xffffffffu;
        for (int w = 0; w < 256 / kWave; ++w) m = min(m, red[k][w]);
        if (k >= k0 && k < lf && m != 0xffffffffu) atomicMin(&st->mins[k], m);
    }
}

__global__ __launch_bounds__(256) void start_write_kernel(const uint32_t* __restrict__ posc,
                                                          const uint32_t* __restrict__ posf, int lf, uint32_t n_crit,
                                                          LoopState* st, uint64_t* __restrict__ K,
                                                          uint32_t* __restrict__ pos_out) {
    const bool fine = st->start_fine != 0;
    const int e = fine ? lf : kStartCoarse;
    const uint32_t* pos = fine ? posf : posc;
    int l = 0;  // deepest level whose nodes' parents all hold more than n_crit
    while (l < e && st->mins[l] > n_crit) ++l;
    const uint32_t nodes = 1u << (3 * l);
    const int step = 3 * (e - l);
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j <= nodes; j += stride) {
        K[j] = j == nodes ? kKeyEnd : static_cast<uint64_t>(j) << (3 * (kL - l));
        pos_out[j] = pos[static_cast<size_t>(j) << step];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->nl[0] = nodes;
        st->start_level = static_cast<uint32_t>(l);
    }
}

// ---- one round: g1 + g2 + g3 -------------------------------------------------
//
// A tile is kRTile consecutive leaves. Their keys and positions, with kRHalo
// entries on either side (K_{i+1} and the 8-sibling checks reach up to 8
// entries away), are first read into LDS with coalesced loads; each thread
// then decides its kRItems consecutive leaves from LDS. When the tile's new
// entries fit in the same LDS (no split-heavy tile), they are assembled there
// and stored with coalesced writes; otherwise every thread writes its own.

constexpr int kRHalo = 8;
constexpr int kRSpan = kRTile + 2 * kRHalo;

__global__ __launch_bounds__(kRBlock, 4) void round_kernel(uint32_t n, uint32_t n_crit, const uint64_t* __restrict__ K,
                                                         const uint32_t* __restrict__ pos,
                                                         uint64_t* __restrict__ K_out, uint32_t* __restrict__ pos_out,
                                                         uint64_t* __restrict__ splits, uint32_t split_capacity,
                                                         LoopState* st, int round, uint64_t capacity, uint64_t* lb) {
    __shared__ uint32_t slot;
    __shared__ uint64_t scan_tmp[kRBlock / kWave];
    __shared__ uint64_t tile_prefix;
    __shared__ uint32_t split_base;
    __shared__ uint32_t any_change;
    __shared__ uint32_t any_merge;
    __shared__ uint64_t sK[kRSpan];  // K[base - kRHalo ...], then the tile's new entries
    __shared__ uint32_t sP[kRSpan];

    // Converged in an earlier round; or the last round only split, and no new
    // child can split (this round would copy every leaf: merges need 8 leaves
    // whose sum is at most n_crit, and no such group was made or changed)
    if (round > 0 && (st->changed[round - 1] == 0 || (st->merged[round - 1] == 0 && st->over[round - 1] == 0)))
        return;
    const uint64_t nl = st->nl[round];
    if (nl == 0 || nl > capacity) return;  // an earlier round overflowed
    const uint32_t tiles = static_cast<uint32_t>((nl + kRTile - 1) / kRTile);
    if (blockIdx.x >= tiles) return;  // more blocks than tiles: the rest stay off the counter
    const uint32_t tid = threadIdx.x;
    const uint32_t epoch = static_cast<uint32_t>(round + 1);
    if (tid == 0) {
        any_change = 0;
        any_merge = 0;
    }

    for (;;) {
        const uint32_t tile = take_tile(st->counters[round], &slot);
        if (tile >= tiles) break;
        const int64_t base = static_cast<int64_t>(tile) * kRTile;
        {  // K and positions of entries base-8 .. base+kRTile+7: all loads in flight at once (an index
           // outside 0 .. nl reads entry 0 or nl instead, and is not stored)
            constexpr int kLoads = (kRSpan + kRBlock - 1) / kRBlock;
            constexpr int kHalf = (kLoads + 1) / 2;  // two batches of loads keep the registers in budget
#pragma unroll
            for (int h = 0; h < kLoads; h += kHalf) {
                uint64_t lk[kHalf];
                uint32_t lp[kHalf];
#pragma unroll
                for (int q = 0; q < kHalf; ++q) {
                    const int64_t g = base - kRHalo + static_cast<int64_t>(tid) + (h + q) * kRBlock;
                    const int64_t c = min(max(g, int64_t{0}), static_cast<int64_t>(nl));
                    lk[q] = K[c];
                    lp[q] = pos[c];
                }
#pragma unroll
                for (int q = 0; q < kHalf; ++q) {
                    const int j = static_cast<int>(tid) + (h + q) * kRBlock;
                    const int64_t g = base - kRHalo + j;
                    if (h + q < kLoads && j < kRSpan && g >= 0 && g <= static_cast<int64_t>(nl)) {
                        sK[j] = lk[q];
                        sP[j] = lp[q];
                    }
                }
            }
        }
        __syncthreads();
        const uint32_t lfirst = tid * kRItems;  // first leaf of this thread, relative to base
        const uint64_t first = static_cast<uint64_t>(base) + lfirst;

        // g1: decision O_i for this thread's leaves
        uint32_t op[kRItems];
        uint64_t kk[kRItems + 1];
        uint32_t pp[kRItems];
        uint32_t osum = 0, nsplit = 0;
        bool changed = false, merged = false;
#pragma unroll
        for (int j = 0; j <= kRItems; ++j) kk[j] = sK[kRHalo + lfirst + j];
#pragma unroll
        for (int j = 0; j < kRItems; ++j) {
            const uint64_t i = first + j;
            const int li = kRHalo + static_cast<int>(lfirst) + j;
            uint32_t o = 0;
            pp[j] = sP[li];
            if (i < nl) {
                const uint64_t ki = kk[j];
                const uint64_t delta = kk[j + 1] - ki;
                const uint32_t cnt = sP[li + 1] - pp[j];
                o = 1;
                if (cnt > n_crit && delta > 1) {
                    o = 8;  // subdivide
                } else if (delta < kKeyEnd) {  // the root never merges
                    // place among its siblings, (K_i mod 8 delta) / delta; delta is a power of 8
                    const uint64_t js = (ki >> (63 - clz64(delta))) & 7u;
                    if (js >= 1 && i >= js && i - js + 8 <= nl && sK[li - js] + 8 * delta == sK[li - js + 8] &&
                        sP[li - js + 8] - sP[li - js] <= n_crit)
                        o = 0;  // 8 sibling leaves with at most n_crit particles: merge
                }
                changed |= (o != 1);
                merged |= (o == 0);
            }
            op[j] = o;
            osum += o;
            nsplit += o == 8;
        }
        if (merged) any_merge = 1;

        // g2: exclusive scan of O (low word) and of the split count (high word)
        uint64_t block_total;
        const uint64_t excl = block_exclusive_sum<uint64_t, kRBlock>(
            (static_cast<uint64_t>(nsplit) << 32) | osum, scan_tmp, &block_total);
        if (tid < kWave) {
            uint64_t prefix = 0;
            uint64_t* w = lb + tile;
            const uint64_t agg = block_total & 0xffffffffull;
            if (tile == 0) {
                if (tid == 0) st_agent(w, lb_word(kFlagInc, epoch, agg));
            } else {
                if (tid == 0) st_agent(w, lb_word(kFlagAgg, epoch, agg));
                prefix = lookback_wave<4>(lb, tile, epoch, &st->err);
                if (tid == 0) st_agent(w, lb_word(kFlagInc, epoch, prefix + agg));
            }
            if (tid == 0) {
                tile_prefix = prefix;
                const uint32_t sc = static_cast<uint32_t>(block_total >> 32);
                split_base = sc ? atomicAdd(&st->nsplit[round], sc) : 0u;
            }
        }
        if (changed) any_change = 1;
        __syncthreads();
        const uint64_t tp = tile_prefix;
        const uint32_t out_total = static_cast<uint32_t>(block_total);  // new entries of this tile
        const bool staged = out_total <= static_cast<uint32_t>(kRSpan);  // block-uniform

        // g3: K' (Eqs. rebalancecopy / rebalancesplit) and the known positions of K'
        uint32_t lo = static_cast<uint32_t>(excl);  // this thread's first new entry, relative to tp
        uint32_t s_at = split_base + static_cast<uint32_t>(excl >> 32);
#pragma unroll
        for (int j = 0; j < kRItems; ++j) {
            const uint64_t i = first + j;
            if (i < nl) {
                const uint64_t ki = kk[j];
                const uint64_t o_prime = tp + lo;
                if (op[j] == 1) {
                    if (staged) {
                        sK[lo] = ki;
                        sP[lo] = pp[j];
                    } else if (o_prime <= capacity) {
                        K_out[o_prime] = ki;
                        pos_out[o_prime] = pp[j];
                    }
                } else if (op[j] == 8) {
                    const uint64_t child = (kk[j + 1] - ki) >> 3;
                    if (staged) {
#pragma unroll
                        for (int c = 0; c < 8; ++c) sK[lo + c] = ki + c * child;
                        sP[lo] = pp[j];  // the other 7 come from the split search
                    } else if (o_prime + 7 <= capacity) {
#pragma unroll
                        for (int c = 0; c < 8; ++c) K_out[o_prime + c] = ki + c * child;
                        pos_out[o_prime] = pp[j];
                    }
                    if (o_prime + 7 <= capacity && s_at < split_capacity) splits[s_at] = i | (o_prime << 32);
                    ++s_at;
                }
            }
            lo += op[j];
        }
        if (staged) {  // the g3 writes above went to LDS (sK / sP were free after g1)
            __syncthreads();
            for (uint32_t j = tid; j < out_total; j += kRBlock) {
                if (tp + j <= capacity) {
                    K_out[tp + j] = sK[j];
                    pos_out[tp + j] = sP[j];  // split children 1..7 are overwritten by the split search
                }
            }
        }
        // the owner of the last leaf closes K' with 8^L
        if (first < nl && nl <= first + kRItems) {
            const uint64_t o_prime = tp + lo;
            st->nl[round + 1] = o_prime;
            if (o_prime <= capacity) {
                K_out[o_prime] = kKeyEnd;
                pos_out[o_prime] = n;
            }
        }
        __syncthreads();
    }
    if (tid == 0 && any_change) atomicOr(&st->changed[round], 1u);
    if (tid == 0 && any_merge) atomicOr(&st->merged[round], 1u);
}

// ---- f for the next round: positions of the inner child boundaries ----------

// Child boundaries of the listed splits: positions in P of the 7 inner
// boundaries of each split leaf. With at most one search per wave (early
// rounds: few splits, long ranges) every search gets a whole wave (63 probes
// per step). Otherwise a wave takes 8 splits, 8 lanes each: a range of at most
// kSmallRange keys is read by its 8 lanes at once (16 keys each, independent
// loads) and every boundary is the count of the range's keys below it; a
// longer range is searched by lanes 1..7, one binary search each, in parallel.
constexpr uint32_t kSmallRange = 128;

__global__ __launch_bounds__(kSearchBlock) void split_search_kernel(const uint64_t* __restrict__ P, uint32_t n,
                                                                     const uint64_t* __restrict__ K,
                                                                     const uint32_t* __restrict__ pos,
                                                                     uint32_t* __restrict__ pos_out,
                                                                     const uint64_t* __restrict__ splits,
                                                                     uint32_t split_capacity, LoopState* st,
                                                                     int round, uint64_t capacity, uint32_t n_crit) {
    const uint64_t nl = st->nl[round];
    if (st->nl[round + 1] > capacity || nl > capacity) return;  // overflowed round: K' is discarded
    const uint32_t listed = min(st->nsplit[round], split_capacity);
    const uint32_t lane = lane_id();
    const uint32_t t = lane & 7u;  // child boundary t (1..7) of the group's split
    const uint32_t waves = gridDim.x * (kSearchBlock / kWave);
    const uint32_t wave = blockIdx.x * (kSearchBlock / kWave) + __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    if (static_cast<uint64_t>(listed) * 7u <= waves) {  // one search per wave (wave-uniform branch)
        for (uint32_t w = wave; w < listed * 7u; w += waves) {
            const uint64_t e = splits[w / 7u];
            const uint32_t c = w % 7u + 1u;
            const uint64_t i = e & 0xffffffffull;
            const uint64_t ki = K[i];
            const uint64_t key = ki + c * ((K[i + 1] - ki) >> 3);
            const uint32_t hi = min(pos[i + 1], n);
            const uint32_t lo = min(pos[i], hi);
            const uint32_t dst = static_cast<uint32_t>(e >> 32) + c;
            const uint32_t at = wave_lower_bound(P, lo, hi, key);
            if (lane == 0 && dst <= capacity) pos_out[dst] = at;
        }
        // the children's counts are not gathered here: let the next round run
        if (listed != 0 && wave == 0 && lane == 0) atomicOr(&st->over[round], 1u);
        return;
    }
    bool wave_over = false;  // one flag write per wave, not per group of splits
    for (uint32_t base = wave * 8u; base < listed; base += waves * 8u) {
        const uint32_t sidx = base + (lane >> 3);
        bool valid = sidx < listed;
        uint32_t lo = 0, hi = 0, dst0 = 0;
        uint64_t ki = 0, step = 0;
        if (valid) {
            const uint64_t e = splits[sidx];
            const uint64_t i = e & 0xffffffffull;
            ki = K[i];
            step = (K[i + 1] - ki) >> 3;
            hi = min(pos[i + 1], n);  // positions never exceed n; the clamps guard memory all the same
            lo = min(pos[i], hi);
            dst0 = static_cast<uint32_t>(e >> 32);
        }
        valid = valid && static_cast<uint64_t>(dst0) + 7u <= capacity;  // always true for a listed split
        const uint64_t key = ki + t * step;
        const bool small = valid && hi - lo <= kSmallRange;
        // short ranges: every lane of the group counts its 16 keys below each boundary
        uint32_t cnt[7] = {0, 0, 0, 0, 0, 0, 0};
        if (small) {
            uint64_t kq[kSmallRange / 8];
#pragma unroll
            for (uint32_t m = 0; m < kSmallRange / 8; ++m) {
                const uint32_t q = lo + t + 8u * m;
                kq[m] = q < hi ? P[q] : ~0ull;
            }
#pragma unroll
            for (uint32_t m = 0; m < kSmallRange / 8; ++m)
#pragma unroll
                for (uint32_t c = 0; c < 7; ++c) cnt[c] += kq[m] < ki + (c + 1) * step ? 1u : 0u;
        }
#pragma unroll
        for (uint32_t c = 0; c < 7; ++c) {  // sums over the group's 8 lanes (all lanes take part)
            cnt[c] += __shfl_xor(cnt[c], 1, kWave);
            cnt[c] += __shfl_xor(cnt[c], 2, kWave);
            cnt[c] += __shfl_xor(cnt[c], 4, kWave);
        }
        uint32_t b = lo;  // this lane's boundary (lane 0 of a group: the range's start)
        if (small && t != 0) {
            uint32_t below = 0;
#pragma unroll
            for (uint32_t c = 0; c < 7; ++c) below = c + 1 == t ? cnt[c] : below;
            b = lo + below;
            pos_out[dst0 + t] = b;
        }
        if (valid && !small && t != 0) {
            b = static_cast<uint32_t>(lower_bound_u64(P, lo, hi, key));
            pos_out[dst0 + t] = b;
        }
        // does a new child hold more than n_crit (and could split: span above 1)?
        const uint32_t before = __shfl(b, static_cast<int>(lane) - 1, kWave);  // lane 0's value is not used
        const bool over = valid && t != 0 && step > 1 && (b - before > n_crit || (t == 7 && hi - b > n_crit));
        wave_over = wave_over || __ballot(over) != 0ull;
    }
    if (wave_over && lane == 0) atomicOr(&st->over[round], 1u);
}

// ---- pick the array of the last complete round --------------------------------

struct Outcome {
    uint32_t last;     // rounds completed (the array after them is the result)
    uint32_t code;     // 0 running, 1 converged, 2 capacity exceeded
    uint64_t nl;       // leaves of that array
    uint32_t buf;      // which of the two arrays holds it (the parity of the rounds that ran)
};

// settle_last: the last enqueued round may settle too; its check round is then
// counted without having been enqueued (the caller allows one more round).
__device__ __forceinline__ Outcome loop_outcome(const LoopState* st, uint32_t enqueued, uint64_t capacity,
                                                bool settle = true, bool settle_last = false) {
    for (uint32_t q = 0; q < enqueued; ++q) {
        if (st->nl[q + 1] > capacity) return {q, 2u, st->nl[q], q & 1u};
        if (st->changed[q] == 0) return {q + 1, 1u, st->nl[q + 1], (q + 1) & 1u};  // round q copied every leaf
        // round q + 1 would copy every leaf: it does not run, and counts
        if (settle && (q + 1 < enqueued || settle_last) && st->merged[q] == 0 && st->over[q] == 0)
            return {q + 2, 1u, st->nl[q + 1], (q + 1) & 1u};
    }
    return {enqueued, 0u, st->nl[enqueued], enqueued & 1u};
}

// Leaves the result array in K[0] (copied from K[1] when an odd number of
// rounds completed), writes its counts, and publishes its leaf count.
__global__ __launch_bounds__(256) void finalize_kernel(LoopState* st, uint32_t enqueued, uint64_t capacity,
                                                       uint64_t* __restrict__ K0, const uint64_t* __restrict__ K1,
                                                       const uint32_t* __restrict__ pos0,
                                                       const uint32_t* __restrict__ pos1,
                                                       uint32_t* __restrict__ counts, uint32_t settle_last) {
    const Outcome o = loop_outcome(st, enqueued, capacity, true, settle_last != 0);
    const uint64_t nl = o.nl <= capacity ? o.nl : 0;
    const bool odd = o.buf != 0;
    const uint32_t* pos = odd ? pos1 : pos0;
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x; i <= nl; i += stride) {
        if (odd) K0[i] = K1[i];
        if (counts && i < nl) counts[i] = pos[i + 1] - pos[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st->final_nl = nl;
        st->final_last = o.last;
        st->final_code = o.code;
    }
}

struct RebalanceWs {
    uint64_t* K_alt;
    uint32_t* pos[2];
    uint64_t* splits;
    uint32_t split_capacity;
    LoopState* st;
    uint64_t* lb;
    size_t lb_words;
    uint32_t* posc;  // level-3 node positions (start-level search)
    size_t bytes;
};

RebalanceWs carve_rebalance(void* ws, size_t n, uint32_t n_crit, size_t cap) {
    Carve c(ws);
    RebalanceWs r{};
    r.K_alt = c.take<uint64_t>(cap + 1);
    r.pos[0] = c.take<uint32_t>(cap + 1);
    r.pos[1] = c.take<uint32_t>(cap + 1);
    // leaves that split in one round hold > n_crit particles each and are disjoint
    const size_t max_splits = std::min<size_t>(cap, n / (static_cast<size_t>(n_crit) + 1)) + 1;
    r.split_capacity = static_cast<uint32_t>(max_splits);
    r.splits = c.take<uint64_t>(max_splits);
    r.st = c.take<LoopState>(1);
    r.lb_words = (cap + kRTile - 1) / kRTile + 1;
    r.lb = c.take<uint64_t>(r.lb_words);
    r.posc = c.take<uint32_t>(kCoarseNodes + 1);
    r.bytes = c.off;
    return r;
}

uint32_t grid_1d(size_t items, int block) { return static_cast<uint32_t>((items + block - 1) / block); }

uint32_t clamp_grid(size_t blocks) {
    return static_cast<uint32_t>(std::max<size_t>(1, std::min<size_t>(blocks, kMaxGrid)));
}

// one wave per search while searches are few
uint32_t search_grid(size_t splits) { return clamp_grid(grid_1d((splits + 7) / 8, kSearchBlock / kWave)); }  // 8 splits a wave

}  // namespace

cstone_status launch_node_counts(const uint64_t* sorted_keys, size_t n, const uint64_t* leaves, size_t n_leaves,
                                 uint32_t* counts, hipStream_t stream) {
    if (n_leaves == 0) return CSTONE_OK;
    hipLaunchKernelGGL(node_counts_kernel, dim3(grid_1d(n_leaves, kCountBlock)), dim3(kCountBlock), 0, stream,
                       sorted_keys, n, leaves, n_leaves, counts);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

size_t rebalance_workspace_bytes(size_t n, uint32_t n_crit, size_t leaf_capacity) {
    return carve_rebalance(nullptr, n, n_crit ? n_crit : 1, leaf_capacity).bytes;
}

cstone_status RebalanceLoop::begin(const uint64_t* P, size_t n, uint32_t n_crit, uint64_t* leaves, size_t nl0,
                                   size_t cap, uint32_t* counts, uint32_t max_iters, void* ws, size_t ws_bytes,
                                   hipStream_t stream, const uint32_t* input_flags, const uint32_t* level6) {
    RebalanceWs w = carve_rebalance(ws, n, n_crit, cap);
    if (ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    if (nl0 < 1 || nl0 > cap || cap >= 0xffffffffull) return CSTONE_ERR_INVALID_ARG;
    P_ = P;
    n_ = n;
    n_crit_ = n_crit;
    leaves_ = leaves;
    nl0_ = nl0;
    cap_ = cap;
    counts_ = counts;
    max_iters_ = std::min<uint32_t>(max_iters ? max_iters : kL + 1, kMaxRounds);
    enqueued_ = 0;
    stream_ = stream;
    ws_ = ws;
    st_ = w.st;
    root_ = nl0 == 1;
    // From the root and to convergence, the loop may skip the rounds that only
    // split every leaf: aim at the level where nodes hold about 8 (n_crit + 1)
    // particles, not finer than kStartFine, and at least level 3.
    start_top_ = 0;
    if (root_ && max_iters_ >= static_cast<uint32_t>(kL + 1) && n > 0) {
        int lf = 1;
        for (double r = static_cast<double>(n) / (static_cast<double>(n_crit) + 1.0); r >= 8.0; r /= 8.0) ++lf;
        lf = std::min(std::max(lf, kStartCoarse), kStartFine);
        if ((size_t{1} << (3 * lf)) <= cap) start_top_ = lf;
    }
    const size_t init_items = std::max<size_t>(w.lb_words, kMaxRounds + 1);
    if (start_top_ && level6)  // the set-up and the start positions from the sort's table together
        hipLaunchKernelGGL(loop_init_table_kernel,
                           dim3(clamp_grid(grid_1d(std::max<size_t>(init_items, (size_t{1} << (3 * start_top_)) + 1), 256))),
                           dim3(256), 0, stream, w.st, static_cast<uint64_t>(nl0), w.lb, w.lb_words, w.pos[0],
                           static_cast<uint32_t>(n), input_flags, P, level6, start_top_, w.posc, w.pos[1]);
    else
        hipLaunchKernelGGL(loop_init_kernel, dim3(clamp_grid(grid_1d(init_items, 256))), dim3(256), 0, stream, w.st,
                           static_cast<uint64_t>(nl0), w.lb, w.lb_words, w.pos[0], static_cast<uint32_t>(n),
                           (root_ && !start_top_) ? 1 : 0, leaves, input_flags);
    if (!root_)
        hipLaunchKernelGGL(positions_kernel, dim3(grid_1d(nl0 + 1, kCountBlock)), dim3(kCountBlock), 0, stream, P, n,
                           leaves, nl0, w.pos[0]);
    if (start_top_) {
        const int lf = start_top_;
        const uint32_t un = static_cast<uint32_t>(n);
        // positions of the level-3 and level-lf nodes: from the sort's level-6
        // table when there is one, else by searching P
        if (!level6)
            hipLaunchKernelGGL(start_coarse_kernel, dim3(grid_1d(kCoarseNodes + 1, 256 / kWave)), dim3(256), 0, stream,
                               P, un, w.posc);
        if (level6) {  // positions at every level up to lf: all minima in one pass
            hipLaunchKernelGGL(start_mins_kernel, dim3(clamp_grid(grid_1d(size_t{1} << (3 * (lf - 1)), 256))),
                               dim3(256), 0, stream, w.pos[1], lf, w.st, 1);
        } else {
            hipLaunchKernelGGL(start_check_kernel, dim3(1), dim3(kCoarseNodes), 0, stream, w.posc, n_crit, lf, w.st);
            if (lf > kStartCoarse) {
                hipLaunchKernelGGL(start_fine_kernel, dim3(kCoarseNodes), dim3(kFineBlock), 0, stream, P, w.posc, lf,
                                   w.st, w.pos[1]);
                if (lf > kStartCoarse + 1)
                    hipLaunchKernelGGL(start_mins_kernel,
                                       dim3(clamp_grid(grid_1d(size_t{1} << (3 * (lf - 1)), 256))), dim3(256), 0,
                                       stream, w.pos[1], lf, w.st, 0);
            }
        }
        hipLaunchKernelGGL(start_write_kernel, dim3(clamp_grid(grid_1d((size_t{1} << (3 * lf)) + 1, 256))), dim3(256),
                           0, stream, w.posc, w.pos[1], lf, n_crit, w.st, leaves, w.pos[0]);
        nl0_ = size_t{1} << (3 * lf);  // round 0 starts with at most this many leaves
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

cstone_status RebalanceLoop::enqueue(uint32_t rounds) {
    RebalanceWs w = carve_rebalance(ws_, n_, n_crit_, cap_);
    if (rounds == 0) {
        rounds = 2;
        if (root_) {  // from the root: about log8(n / (n_crit + 1)) + 2 rounds
            double ratio = static_cast<double>(n_) / (static_cast<double>(n_crit_) + 1.0);
            while (ratio > 1.0) {
                ratio /= 8.0;
                ++rounds;
            }
            // less the rounds a uniform start skips. One level is kept to spare
            // when the start may come out a level coarser (the level above it
            // holds under 2 (n_crit + 1) particles per node on average, so
            // some node may not exceed n_crit); a start coarser than that, or
            // a deeper tree, needs a later batch. After a safe start the
            // check round is not enqueued: when the last round settles the
            // tree, the finalize kernel counts the check round without running
            // it (and a tree that needs more rounds gets a later batch).
            if (start_top_ > 1) {
                const double above = static_cast<double>(n_) / (static_cast<double>(n_crit_) + 1.0) /
                                     static_cast<double>(size_t{1} << (3 * (start_top_ - 1)));
                const bool safe = above >= 2.0;
                const uint32_t skip = static_cast<uint32_t>(start_top_) - (safe ? 0u : 1u);
                rounds = safe ? std::max<uint32_t>(1, rounds - skip - 1) : std::max<uint32_t>(2, rounds - skip);
            }
        }
    }
    rounds = std::min(rounds, max_iters_ - enqueued_);
    uint64_t* bufK[2] = {leaves_, w.K_alt};
    for (uint32_t q = enqueued_; q < enqueued_ + rounds; ++q) {
        // leaves entering round q: at most nl0 * 8^q and the capacity
        double bound = static_cast<double>(nl0_);
        for (uint32_t e = 0; e < q && bound < static_cast<double>(cap_); ++e) bound *= 8.0;
        const size_t rows = static_cast<size_t>(std::min<double>(bound, static_cast<double>(cap_)));
        hipLaunchKernelGGL(round_kernel, dim3(clamp_grid(grid_1d(rows, kRTile))), dim3(kRBlock), 0, stream_,
                           static_cast<uint32_t>(n_), n_crit_, bufK[q & 1], w.pos[q & 1], bufK[(q + 1) & 1],
                           w.pos[(q + 1) & 1], w.splits, w.split_capacity, w.st, static_cast<int>(q),
                           static_cast<uint64_t>(cap_), w.lb);
        const size_t max_splits = std::min<size_t>(rows, w.split_capacity);
        hipLaunchKernelGGL(split_search_kernel, dim3(search_grid(max_splits)),
                           dim3(kSearchBlock), 0, stream_, P_, static_cast<uint32_t>(n_), bufK[q & 1], w.pos[q & 1],
                           w.pos[(q + 1) & 1], w.splits, w.split_capacity, w.st, static_cast<int>(q),
                           static_cast<uint64_t>(cap_), n_crit_);
    }
    enqueued_ += rounds;
    hipLaunchKernelGGL(finalize_kernel, dim3(clamp_grid(grid_1d(cap_ + 1, 256))), dim3(256), 0, stream_, w.st,
                       enqueued_, static_cast<uint64_t>(cap_), leaves_, w.K_alt, w.pos[0], w.pos[1], counts_,
                       enqueued_ < max_iters_ ? 1u : 0u);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

const uint64_t* RebalanceLoop::device_leaf_count() const { return &st_->final_nl; }

cstone_status RebalanceLoop::wait(bool* finished) {
    LoopHeader host;  // the loop state without its tile counters
    CS_HIP(hipMemcpyAsync(&host, static_cast<const LoopHeader*>(st_), sizeof(LoopHeader), hipMemcpyDeviceToHost,
                          stream_));
    CS_HIP(hipStreamSynchronize(stream_));
    input_flags = host.input_flags;
    rounds = host.final_last + host.start_level;
    *finished = true;
    if (host.err) {
        status = CSTONE_ERR_DEVICE;
        return status;
    }
    if (host.final_code == 2) {
        n_leaves = host.nl[host.final_last + 1];  // what the failing round needed
        status = CSTONE_ERR_CAPACITY;
        return status;
    }
    n_leaves = host.final_nl;
    if (host.final_code == 1) {
        status = CSTONE_OK;
    } else if (enqueued_ >= max_iters_) {
        status = CSTONE_ERR_NOT_CONVERGED;
    } else {
        status = CSTONE_OK;
        *finished = false;
    }
    return status;
}

cstone_status run_rebalance(const uint64_t* P, size_t n, uint32_t n_crit, uint64_t* leaves, size_t* n_leaves,
                            size_t cap, uint32_t* counts, uint32_t max_iters, uint32_t* iters_done, void* ws,
                            size_t ws_bytes, hipStream_t stream) {
    RebalanceLoop loop;
    cstone_status s = loop.begin(P, n, n_crit, leaves, *n_leaves, cap, counts, max_iters, ws, ws_bytes, stream,
                                 nullptr);
    if (s != CSTONE_OK) return s;
    bool finished = false;
    uint32_t batch = 0;
    while (!finished) {
        if ((s = loop.enqueue(batch)) != CSTONE_OK) return s;
        loop.wait(&finished);
        batch = 4;
    }
    if (loop.status == CSTONE_ERR_DEVICE) return loop.status;
    *n_leaves = loop.n_leaves;
    if (iters_done) *iters_done = loop.rounds;
    return loop.status;
}


// ---- batched rebalance ----------------------------------------------------------
//
// The cornerstone arrays of all sets sit back to back, each followed by its
// closing key 8^L, with sid[e] the set of entry e (sets stay in order and
// contiguous). A round decides every entry as in the single-set case, with the
// set's own N_crit; a closing entry is always kept (O = 1), and a merge group
// must lie inside one set. The exclusive scan then runs over all entries at
// once, so one launch serves every set; the first entry of each set (key 0)
// records where that set starts in the next array.

namespace {

// Batched round tiles: 256 threads of kRItems entries (with the per-entry set
// ids, 512-thread blocks at 4 waves per SIMD would spill).
constexpr int kBBlock = 256;
constexpr int kBTile = kBBlock * kRItems;
// Blocks of a batched round: as many as stay resident (4 per CU), each taking
// tiles until none are left, so the one tile counter sees about one ticket per
// tile, not one more per block of a larger grid.
constexpr uint32_t kBRoundGrid = 1024;
constexpr int kBSpan = kBTile + 2 * kRHalo;

__global__ __launch_bounds__(256) void batch_init_kernel(LoopState* st, const BatchSet* __restrict__ sets,
                                                         uint32_t n_sets, uint64_t* K, uint32_t* pos, uint32_t* sid,
                                                         uint32_t* starts, uint64_t* lb, size_t lb_words,
                                                         uint32_t* changed_set, size_t changed_words) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (size_t i = t; i < lb_words; i += stride) lb[i] = 0;
    for (size_t i = t; i < changed_words; i += stride) changed_set[i] = 0;
    for (size_t s = t; s < n_sets; s += stride) {  // every set starts as the root leaf
        const BatchSet& S = sets[s];
        K[2 * s] = 0;
        K[2 * s + 1] = kKeyEnd;
        pos[2 * s] = S.part_off;
        pos[2 * s + 1] = S.part_off + S.n;
        sid[2 * s] = sid[2 * s + 1] = static_cast<uint32_t>(s);
        starts[s] = static_cast<uint32_t>(2 * s);
    }
    if (t < kMaxRounds) {
        st->changed[t] = 0;
        st->merged[t] = 0;
        st->over[t] = 0;
        st->counters[t][0] = 0;
        st->nsplit[t] = 0;
    }
    if (t <= kMaxRounds) st->nl[t] = t == 0 ? 2ull * n_sets : 0ull;
    if (t == 0) {
        starts[n_sets] = 2 * n_sets;
        st->err = 0;
        st->input_flags = 0;
    }
}

__global__ __launch_bounds__(kBBlock, 4) void batch_round_kernel(const BatchSet* __restrict__ sets,
                                                               const uint64_t* __restrict__ K,
                                                               const uint32_t* __restrict__ pos,
                                                               const uint32_t* __restrict__ sid,
                                                               uint64_t* __restrict__ K_out,
                                                               uint32_t* __restrict__ pos_out,
                                                               uint32_t* __restrict__ sid_out,
                                                               uint32_t* __restrict__ starts_out, uint32_t n_sets,
                                                               uint32_t* __restrict__ changed_set,
                                                               uint64_t* __restrict__ splits, uint32_t split_capacity,
                                                               LoopState* st, int round, uint64_t capacity,
                                                               uint64_t* lb) {
    __shared__ uint32_t slot;
    __shared__ uint64_t scan_tmp[kBBlock / kWave];
    __shared__ uint64_t tile_prefix;
    __shared__ uint32_t split_base;
    __shared__ uint32_t any_change;
    __shared__ uint64_t sK[kBSpan];  // entries base-8 .., then the tile's new entries
    __shared__ uint32_t sP[kBSpan];
    __shared__ uint32_t sS[kBSpan];
    // sets that changed in this tile, by set id mod kSetFlags: a set holds at
    // least two entries, so a tile spans at most kBTile / 2 + 1 consecutive
    // sets, and they take distinct slots
    constexpr uint32_t kSetFlags = kBTile;
    static_assert((kSetFlags & (kSetFlags - 1)) == 0 && kSetFlags > kBTile / 2 + 1, "distinct slots");
    __shared__ uint8_t sflag[kSetFlags];

    if (round > 0 && st->changed[round - 1] == 0) return;  // every set converged earlier
    const uint64_t M = st->nl[round];
    if (M == 0 || M > capacity) return;  // an earlier round overflowed
    const uint32_t tiles = static_cast<uint32_t>((M + kBTile - 1) / kBTile);
    if (blockIdx.x >= tiles) return;  // more blocks than tiles: the rest stay off the counter
    const uint32_t tid = threadIdx.x;
    const uint32_t epoch = static_cast<uint32_t>(round + 1);
    if (tid == 0) any_change = 0;

    for (;;) {
        const uint32_t tile = take_tile(st->counters[round], &slot);
        if (tile >= tiles) break;
        const int64_t base = static_cast<int64_t>(tile) * kBTile;
        if (base >= kRHalo && base + kBSpan - kRHalo <= static_cast<int64_t>(M)) {
            // block-uniform: the whole span exists; its keys, then its positions and set ids, each
            // batch of loads in flight at once (one base pointer, constant offsets)
            constexpr int kFull = kBSpan / kBBlock;  // whole rows of the span; the rest below
            const size_t g0 = static_cast<size_t>(base - kRHalo) + tid;
            {
                uint64_t lk[kFull];
#pragma unroll
                for (int q = 0; q < kFull; ++q) lk[q] = K[g0 + q * kBBlock];
#pragma unroll
                for (int q = 0; q < kFull; ++q) sK[tid + q * kBBlock] = lk[q];
            }
            {
                uint32_t lp[kFull], ls[kFull];
#pragma unroll
                for (int q = 0; q < kFull; ++q) {
                    lp[q] = pos[g0 + q * kBBlock];
                    ls[q] = sid[g0 + q * kBBlock];
                }
#pragma unroll
                for (int q = 0; q < kFull; ++q) {
                    sP[tid + q * kBBlock] = lp[q];
                    sS[tid + q * kBBlock] = ls[q];
                }
            }
            for (int j = kFull * kBBlock + tid; j < kBSpan; j += kBBlock) {
                sK[j] = K[g0 + (j - tid)];
                sP[j] = pos[g0 + (j - tid)];
                sS[j] = sid[g0 + (j - tid)];
            }
        } else {
            for (int j = tid; j < kBSpan; j += kBBlock) {  // coalesced: entries base-8 .. base+kBTile+7 that exist
                const int64_t g = base - kRHalo + j;
                if (g >= 0 && g < static_cast<int64_t>(M)) {
                    sK[j] = K[g];
                    sP[j] = pos[g];
                    sS[j] = sid[g];
                }
            }
        }
        for (uint32_t j = tid; j < kSetFlags; j += kBBlock) sflag[j] = 0;
        __syncthreads();
        const uint32_t lfirst = tid * kRItems;
        const uint64_t first = static_cast<uint64_t>(base) + lfirst;

        uint32_t op[kRItems];
        uint64_t kk[kRItems + 1];  // this thread's entries and the next one
        uint32_t pp[kRItems], ss[kRItems];
        uint32_t osum = 0, nsplit = 0;
        uint32_t nc = 0, nc_set = 0xffffffffu;  // n_crit of set nc_set
        bool changed = false;
#pragma unroll
        for (int j = 0; j <= kRItems; ++j) kk[j] = sK[kRHalo + lfirst + j];
#pragma unroll
        for (int j = 0; j < kRItems; ++j) {
            const uint64_t e = first + j;
            const int li = kRHalo + static_cast<int>(lfirst) + j;
            uint32_t o = 0;
            pp[j] = sP[li];
            ss[j] = sS[li];
            if (e < M) {
                const uint64_t ke = kk[j];
                o = 1;
                if (ke != kKeyEnd) {  // a leaf (closing entries are kept)
                    const uint32_t s = ss[j];
                    if (s != nc_set) {  // a thread's entries nearly always share one set
                        nc = sets[s].n_crit;
                        nc_set = s;
                    }
                    const uint64_t delta = kk[j + 1] - ke;
                    const uint32_t cnt = sP[li + 1] - pp[j];
                    if (cnt > nc && delta > 1) {
                        o = 8;
                    } else if (delta < kKeyEnd) {
                        const uint64_t js = (ke >> (63 - clz64(delta))) & 7u;
                        if (js >= 1 && e >= js && e - js + 8 < M && sS[li - js] == s && sS[li - js + 8] == s &&
                            sK[li - js] + 8 * delta == sK[li - js + 8] && sP[li - js + 8] - sP[li - js] <= nc)
                            o = 0;
                    }
                    if (o != 1) {
                        changed = true;
                        sflag[s & (kSetFlags - 1)] = 1;
                    }
                }
            }
            op[j] = o;
            osum += o;
            nsplit += o == 8;
        }

        uint64_t block_total;
        const uint64_t excl = block_exclusive_sum<uint64_t, kBBlock>(
            (static_cast<uint64_t>(nsplit) << 32) | osum, scan_tmp, &block_total);
        if (tid < kWave) {
            uint64_t prefix = 0;
            uint64_t* w = lb + tile;
            const uint64_t agg = block_total & 0xffffffffull;
            if (tile == 0) {
                if (tid == 0) st_agent(w, lb_word(kFlagInc, epoch, agg));
            } else {
                if (tid == 0) st_agent(w, lb_word(kFlagAgg, epoch, agg));
                prefix = lookback_wave<4>(lb, tile, epoch, &st->err);
                if (tid == 0) st_agent(w, lb_word(kFlagInc, epoch, prefix + agg));
            }
            if (tid == 0) {
                tile_prefix = prefix;
                const uint32_t sc = static_cast<uint32_t>(block_total >> 32);
                split_base = sc ? atomicAdd(&st->nsplit[round], sc) : 0u;
            }
        }
        if (changed) any_change = 1;
        const uint32_t s_lo = sS[kRHalo];  // set of the tile's first entry (sS is rewritten after the barrier)
        __syncthreads();  // every thread has read the staged entries it needs
        for (uint32_t j = tid; j < kSetFlags; j += kBBlock)  // one flag per set and tile
            if (sflag[j]) atomicOr(&changed_set[s_lo + ((j - s_lo) & (kSetFlags - 1))], 1u);
        const uint64_t tp = tile_prefix;
        const uint32_t out_total = static_cast<uint32_t>(block_total);  // new entries of this tile
        const bool staged = out_total <= static_cast<uint32_t>(kBSpan);  // block-uniform

        uint32_t lo = static_cast<uint32_t>(excl);  // this thread's first new entry, relative to tp
        uint32_t s_at = split_base + static_cast<uint32_t>(excl >> 32);
#pragma unroll
        for (int j = 0; j < kRItems; ++j) {
            const uint64_t e = first + j;
            if (e < M) {
                const uint64_t ke = kk[j];
                const uint32_t s = ss[j];
                const uint64_t o_prime = tp + lo;
                if (op[j] == 1) {
                    if (staged) {
                        sK[lo] = ke;
                        sP[lo] = pp[j];
                        sS[lo] = s;
                    } else if (o_prime <= capacity) {
                        K_out[o_prime] = ke;
                        pos_out[o_prime] = pp[j];
                        sid_out[o_prime] = s;
                    }
                    if (ke == 0 && o_prime <= capacity) starts_out[s] = static_cast<uint32_t>(o_prime);
                    if (e + 1 == M) {  // the last closing key: size of the next array
                        st->nl[round + 1] = o_prime + 1;
                        starts_out[n_sets] = static_cast<uint32_t>(o_prime + 1);
                    }
                } else if (op[j] == 8) {
                    const uint64_t ch = (kk[j + 1] - ke) >> 3;
                    if (staged) {
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            sK[lo + c] = ke + c * ch;
                            sS[lo + c] = s;
                        }
                        sP[lo] = pp[j];  // the other 7 come from the split search
                    } else if (o_prime + 7 <= capacity) {
#pragma unroll
                        for (int c = 0; c < 8; ++c) {
                            K_out[o_prime + c] = ke + c * ch;
                            sid_out[o_prime + c] = s;
                        }
                        pos_out[o_prime] = pp[j];
                    }
                    if (o_prime + 7 <= capacity) {
                        if (ke == 0) starts_out[s] = static_cast<uint32_t>(o_prime);
                        if (s_at < split_capacity) splits[s_at] = e | (o_prime << 32);
                    }
                    ++s_at;
                }
            }
            lo += op[j];
        }
        if (staged) {  // the writes above went to LDS (free after g1): store them coalesced
            __syncthreads();
            for (uint32_t j = tid; j < out_total; j += kBBlock) {
                if (tp + j <= capacity) {
                    K_out[tp + j] = sK[j];
                    pos_out[tp + j] = sP[j];  // split children 1..7 are overwritten by the split search
                    sid_out[tp + j] = sS[j];
                }
            }
        }
        __syncthreads();
    }
    if (tid == 0 && any_change) atomicOr(&st->changed[round], 1u);
}

// Per-set leaves, counts and results from the array of the last complete round.
__global__ __launch_bounds__(256) void batch_finalize_kernel(LoopState* st, uint32_t enqueued, uint64_t capacity,
                                                             const BatchSet* __restrict__ sets, uint32_t n_sets,
                                                             const uint64_t* __restrict__ K0,
                                                             const uint64_t* __restrict__ K1,
                                                             const uint32_t* __restrict__ pos0,
                                                             const uint32_t* __restrict__ pos1,
                                                             const uint32_t* __restrict__ sid0,
                                                             const uint32_t* __restrict__ sid1,
                                                             const uint32_t* __restrict__ starts0,
                                                             const uint32_t* __restrict__ starts1,
                                                             const uint32_t* __restrict__ changed_set,
                                                             const uint32_t* __restrict__ set_flags,
                                                             uint64_t* __restrict__ leaves, uint32_t* __restrict__ counts,
                                                             BatchResult* __restrict__ results,
                                                             const uint32_t* __restrict__ sort_err) {
    const Outcome o = loop_outcome(st, enqueued, capacity, false);  // batched rounds do not record merges
    const uint64_t M = o.nl <= capacity ? o.nl : 0;
    const bool odd = o.last & 1u;
    const uint64_t* K = odd ? K1 : K0;
    const uint32_t* pos = odd ? pos1 : pos0;
    const uint32_t* sid = odd ? sid1 : sid0;
    const uint32_t* starts = odd ? starts1 : starts0;
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    const size_t t0 = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    // kFinItems entries per thread, blockDim.x apart (coalesced): their keys,
    // positions and set ids loaded together (indices clamped to the array),
    // then their sets' records, then the stores
    constexpr int kFinItems = 4;
    const size_t span = static_cast<size_t>(blockDim.x) * kFinItems;
    for (size_t b0 = static_cast<size_t>(blockIdx.x) * span; b0 < M; b0 += static_cast<size_t>(gridDim.x) * span) {
        uint64_t kk[kFinItems];
        uint32_t ss[kFinItems], p0[kFinItems], p1[kFinItems];
#pragma unroll
        for (int q = 0; q < kFinItems; ++q) {
            const size_t e = min(b0 + q * blockDim.x + threadIdx.x, static_cast<size_t>(M - 1));
            kk[q] = K[e];
            ss[q] = sid[e];
            p0[q] = pos[e];
            p1[q] = pos[min(e + 1, static_cast<size_t>(M - 1))];
        }
        uint64_t off[kFinItems], cap[kFinItems];
        uint32_t first[kFinItems], next[kFinItems];
#pragma unroll
        for (int q = 0; q < kFinItems; ++q) {
            off[q] = sets[ss[q]].leaf_off;
            cap[q] = sets[ss[q]].cap;
            first[q] = starts[ss[q]];
            next[q] = starts[ss[q] + 1];
        }
#pragma unroll
        for (int q = 0; q < kFinItems; ++q) {
            const size_t e = b0 + q * blockDim.x + threadIdx.x;
            const uint64_t nl = next[q] - first[q] - 1;
            if (e >= M || nl > cap[q]) continue;  // past the array, or this set outgrew its region
            const uint64_t i = e - first[q];
            leaves[off[q] + i] = kk[q];
            if (i < nl) counts[off[q] + i] = p1[q] - p0[q];  // entry e + 1 is in the same set
        }
    }
    for (size_t s = t0; s < n_sets; s += stride) {
        const uint64_t nl = M ? starts[s + 1] - starts[s] - 1 : 0;
        uint32_t rounds = o.last, status;
        bool converged = false;
        // the first round in which the set changed nothing: flags read 8 rounds at a time
        for (uint32_t q0 = 0; q0 < o.last && !converged; q0 += 8) {
            uint32_t c[8];
#pragma unroll
            for (uint32_t q = 0; q < 8; ++q)
                c[q] = changed_set[static_cast<size_t>(min(q0 + q, o.last - 1)) * n_sets + s];
#pragma unroll
            for (uint32_t q = 0; q < 8; ++q)
                if (!converged && q0 + q < o.last && c[q] == 0) {
                    rounds = q0 + q + 1;
                    converged = true;
                }
        }
        // a device-side wait that gave up (in the sort or a round's look-back)
        // leaves every set's arrays unreliable
        if (st->err != 0 || (sort_err && *sort_err != 0))
            status = CSTONE_ERR_DEVICE;
        else if (set_flags[s] & CSTONE_FLAG_NONFINITE)
            status = CSTONE_ERR_NONFINITE;
        else if (M == 0 || nl > sets[s].cap)
            status = CSTONE_ERR_CAPACITY;
        else if (!converged)
            status = o.code == 2 ? CSTONE_ERR_CAPACITY : CSTONE_ERR_NOT_CONVERGED;
        else
            status = CSTONE_OK;
        results[s] = {static_cast<uint32_t>(nl), static_cast<uint32_t>(nl ? nl + (nl - 1) / 7 : 0), rounds, status};
    }
    if (t0 == 0) {
        st->final_nl = M;
        st->final_last = o.last;
        st->final_code = o.code;
    }
}

struct BatchRebalanceWs {
    uint64_t* K[2];
    uint32_t* pos[2];
    uint32_t* sid[2];
    uint32_t* starts[2];
    uint64_t* splits;
    uint32_t* changed_set;
    LoopState* st;
    uint64_t* lb;
    size_t lb_words;
    size_t bytes;
};

BatchRebalanceWs carve_batch_rebalance(void* ws, uint32_t n_sets, size_t C, size_t split_capacity) {
    Carve c(ws);
    BatchRebalanceWs r{};
    for (int b = 0; b < 2; ++b) {
        r.K[b] = c.take<uint64_t>(C + 1);
        r.pos[b] = c.take<uint32_t>(C + 1);
        r.sid[b] = c.take<uint32_t>(C + 1);
        r.starts[b] = c.take<uint32_t>(static_cast<size_t>(n_sets) + 1);
    }
    r.splits = c.take<uint64_t>(split_capacity);
    r.changed_set = c.take<uint32_t>(static_cast<size_t>(kMaxRounds) * n_sets);
    r.st = c.take<LoopState>(1);
    r.lb_words = (C + kBTile - 1) / kBTile + 1;
    r.lb = c.take<uint64_t>(r.lb_words);
    r.bytes = c.off;
    return r;
}

}  // namespace

size_t batch_rebalance_workspace_bytes(uint32_t n_sets, size_t C, size_t split_capacity) {
    return carve_batch_rebalance(nullptr, n_sets, C, split_capacity).bytes;
}

BatchTreeView batch_rebalance_view(void* ws, uint32_t n_sets, size_t C, size_t split_capacity) {
    BatchRebalanceWs w = carve_batch_rebalance(ws, n_sets, C, split_capacity);
    return {{w.K[0], w.K[1]}, {w.sid[0], w.sid[1]}, {w.starts[0], w.starts[1]}, w.st};
}

cstone_status launch_batch_rebalance(const uint64_t* P, size_t n_total, const BatchSet* sets, uint32_t n_sets,
                                     size_t C,
                                     size_t split_capacity, uint32_t rounds, const uint32_t* set_flags,
                                     uint64_t* leaves, uint32_t* counts, BatchResult* results, void* ws,
                                     size_t ws_bytes, const uint32_t* sort_err, hipStream_t stream) {
    BatchRebalanceWs w = carve_batch_rebalance(ws, n_sets, C, split_capacity);
    if (ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    if (n_sets == 0) return CSTONE_OK;
    if (C >= 0xffffffffull || split_capacity >= 0xffffffffull || C < 2ull * n_sets) return CSTONE_ERR_INVALID_ARG;
    rounds = std::min<uint32_t>(std::max<uint32_t>(rounds, 1), kMaxRounds);
    const size_t changed_words = static_cast<size_t>(kMaxRounds) * n_sets;
    hipLaunchKernelGGL(batch_init_kernel,
                       dim3(clamp_grid(grid_1d(std::max<size_t>({w.lb_words, changed_words, n_sets}), 256))),
                       dim3(256), 0, stream, w.st, sets, n_sets, w.K[0], w.pos[0], w.sid[0], w.starts[0], w.lb,
                       w.lb_words, w.changed_set, changed_words);
    const uint32_t cap_u = static_cast<uint32_t>(split_capacity);
    for (uint32_t q = 0; q < rounds; ++q) {
        const int a = q & 1, b = (q + 1) & 1;
        hipLaunchKernelGGL(batch_round_kernel, dim3(std::min<uint32_t>(clamp_grid(grid_1d(C + 1, kBTile)), kBRoundGrid)),
                           dim3(kBBlock), 0, stream,
                           sets, w.K[a], w.pos[a], w.sid[a], w.K[b], w.pos[b], w.sid[b], w.starts[b], n_sets,
                           w.changed_set + static_cast<size_t>(q) * n_sets, w.splits, cap_u, w.st,
                           static_cast<int>(q), static_cast<uint64_t>(C), w.lb);
        hipLaunchKernelGGL(split_search_kernel, dim3(search_grid(split_capacity)),
                           dim3(kSearchBlock), 0, stream, P, static_cast<uint32_t>(n_total), w.K[a], w.pos[a],
                           w.pos[b], w.splits, cap_u, w.st, static_cast<int>(q), static_cast<uint64_t>(C),
                           0xffffffffu);  // batched rounds do not use the over flag
    }
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(clamp_grid(grid_1d(C + 1, 256))), dim3(256), 0, stream, w.st,
                       rounds, static_cast<uint64_t>(C), sets, n_sets, w.K[0], w.K[1], w.pos[0], w.pos[1], w.sid[0],
                       w.sid[1], w.starts[0], w.starts[1], w.changed_set, set_flags, leaves, counts, results,
                       sort_err);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace cs
