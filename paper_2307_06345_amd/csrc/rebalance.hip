// Leaf counts f (Eq. histogram) and the rebalance loop g = g3.g2.g1 (Sec. 4).
//
// The loop keeps, next to the cornerstone array K, the position of every key
// of K in the sorted particle keys P (the lower bound that f computes). A
// leaf's count is the difference of two adjacent positions, and the combined
// count of 8 sibling leaves is the difference of the positions around them, so
// one kernel per round does g1 (decision), g2 (exclusive scan of O, single
// pass with decoupled look-back) and g3 (writing K'), and hands f of the next
// round the positions of K': copied leaves keep theirs, and only the 7 inner
// boundaries of a split leaf are searched, inside that leaf's own range of P.
// Rounds are enqueued ahead of the host's convergence check; a round that
// starts after convergence (or after a capacity overflow) exits at once.
#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr int kMaxRounds = 64;
constexpr int kCountBlock = 256;
constexpr int kRBlock = 256;
constexpr int kRItems = 4;
constexpr int kRTile = kRBlock * kRItems;
constexpr uint32_t kMaxRoundGrid = 2048;

// Device-side loop state.
struct LoopState {
    uint64_t nl[kMaxRounds + 1];    // leaves entering round r
    uint32_t changed[kMaxRounds];   // some O_i != 1 in round r
    uint32_t counters[kMaxRounds];  // dynamic tile counter of round r
    uint32_t err;
    uint32_t input_flags;           // copy of the caller's key-stage flag word
};

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

// Leaf counts from positions.
__global__ __launch_bounds__(kCountBlock) void counts_from_positions_kernel(const uint32_t* __restrict__ pos,
                                                                             size_t nl,
                                                                             uint32_t* __restrict__ counts) {
    const size_t i = static_cast<size_t>(blockIdx.x) * kCountBlock + threadIdx.x;
    if (i < nl) counts[i] = pos[i + 1] - pos[i];
}

__global__ __launch_bounds__(256) void loop_init_kernel(LoopState* st, uint64_t nl0, uint64_t* lb, size_t lb_words,
                                                        uint32_t* pos, uint32_t n, int root, uint64_t* K,
                                                        const uint32_t* input_flags) {
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    for (size_t i = t; i < lb_words; i += stride) lb[i] = 0;
    if (t < kMaxRounds) {
        st->changed[t] = 0;
        st->counters[t] = 0;
    }
    if (t <= kMaxRounds) st->nl[t] = t == 0 ? nl0 : 0;
    if (t == 0) {
        st->err = 0;
        st->input_flags = input_flags ? *input_flags : 0u;
        if (root) {  // the only one-leaf cornerstone array
            K[0] = 0;
            K[1] = kKeyEnd;
            pos[0] = 0;
            pos[1] = n;
        }
    }
}

// ---- one round: g1 + g2 + g3, and the positions of K' ----------------------

__global__ __launch_bounds__(kRBlock) void round_kernel(const uint64_t* __restrict__ P, uint32_t n, uint32_t n_crit,
                                                         const uint64_t* __restrict__ K,
                                                         const uint32_t* __restrict__ pos,
                                                         uint64_t* __restrict__ K_out, uint32_t* __restrict__ pos_out,
                                                         LoopState* st, int round, uint64_t capacity, uint64_t* lb) {
    __shared__ uint32_t slot;
    __shared__ uint64_t scan_tmp[kRBlock / kWave];
    __shared__ uint64_t tile_prefix;
    __shared__ uint32_t nsplit;
    __shared__ uint16_t split_leaf[kRTile];
    __shared__ uint32_t split_off[kRTile];
    __shared__ uint32_t any_change;

    if (round > 0 && st->changed[round - 1] == 0) return;  // converged in an earlier round
    const uint64_t nl = st->nl[round];
    if (nl == 0 || nl > capacity) return;  // an earlier round overflowed
    const uint32_t tiles = static_cast<uint32_t>((nl + kRTile - 1) / kRTile);
    const uint32_t tid = threadIdx.x;
    const uint32_t epoch = static_cast<uint32_t>(round + 1);
    if (tid == 0) any_change = 0;

    for (;;) {
        const uint32_t tile = take_tile(&st->counters[round], &slot);
        if (tile >= tiles) break;
        if (tid == 0) nsplit = 0;
        const uint64_t tile_first = static_cast<uint64_t>(tile) * kRTile;
        const uint64_t first = tile_first + static_cast<uint64_t>(tid) * kRItems;

        // g1: decision O_i for this thread's leaves
        uint32_t op[kRItems];
        uint64_t sum = 0;
        bool changed = false;
#pragma unroll
        for (int j = 0; j < kRItems; ++j) {
            const uint64_t i = first + j;
            uint32_t o = 0;
            if (i < nl) {
                const uint64_t ki = K[i];
                const uint64_t delta = K[i + 1] - ki;
                const uint32_t cnt = pos[i + 1] - pos[i];
                o = 1;
                if (cnt > n_crit && delta > 1) {
                    o = 8;  // subdivide
                } else if (delta < kKeyEnd) {  // the root never merges
                    const uint64_t js = (ki % (8 * delta)) / delta;  // place among its siblings
                    if (js >= 1 && i >= js && i - js + 8 <= nl && K[i - js] + 8 * delta == K[i - js + 8] &&
                        pos[i - js + 8] - pos[i - js] <= n_crit)
                        o = 0;  // 8 sibling leaves with at most n_crit particles: merge
                }
                changed |= (o != 1);
            }
            op[j] = o;
            sum += o;
        }

        // g2: exclusive scan of O, in the block and then across tiles
        uint64_t block_total;
        const uint64_t excl_thread = block_exclusive_sum<uint64_t, kRBlock>(sum, scan_tmp, &block_total);
        if (tid == 0) {
            uint64_t* w = lb + tile;
            if (tile == 0) {
                st_agent(w, lb_word(kFlagInc, epoch, block_total));
                tile_prefix = 0;
            } else {
                st_agent(w, lb_word(kFlagAgg, epoch, block_total));
                const uint64_t ex = lookback(lb, 1, tile, epoch, &st->err);
                st_agent(w, lb_word(kFlagInc, epoch, ex + block_total));
                tile_prefix = ex;
            }
        }
        if (changed) any_change = 1;
        __syncthreads();
        const uint64_t tp = tile_prefix;

        // g3: K' (Eqs. rebalancecopy / rebalancesplit) and the positions of K'
        uint64_t o_prime = tp + excl_thread;
#pragma unroll
        for (int j = 0; j < kRItems; ++j) {
            const uint64_t i = first + j;
            if (i < nl) {
                const uint64_t ki = K[i];
                if (op[j] == 1) {
                    if (o_prime <= capacity) {
                        K_out[o_prime] = ki;
                        pos_out[o_prime] = pos[i];
                    }
                } else if (op[j] == 8) {
                    if (o_prime + 7 <= capacity) {
                        const uint64_t child = (K[i + 1] - ki) >> 3;
#pragma unroll
                        for (int c = 0; c < 8; ++c) K_out[o_prime + c] = ki + c * child;
                        pos_out[o_prime] = pos[i];
                        const uint32_t s = atomicAdd(&nsplit, 1u);
                        split_leaf[s] = static_cast<uint16_t>(i - tile_first);
                        split_off[s] = static_cast<uint32_t>(o_prime - tp);
                    }
                }
            }
            o_prime += op[j];
        }
        // the owner of the last leaf closes K' with 8^L
        if (first < nl && nl <= first + kRItems) {
            st->nl[round + 1] = o_prime;
            if (o_prime <= capacity) {
                K_out[o_prime] = kKeyEnd;
                pos_out[o_prime] = n;
            }
        }
        __syncthreads();

        // f for the next round: the 7 inner child boundaries of each split leaf,
        // one (leaf, child) pair per thread, searched in the parent's range of P
        const uint32_t work = nsplit * 7u;
        for (uint32_t w = tid; w < work; w += kRBlock) {
            const uint32_t s = w / 7u;
            const uint32_t c = w % 7u + 1u;
            const uint64_t i = tile_first + split_leaf[s];
            const uint64_t ki = K[i];
            const uint64_t key = ki + c * ((K[i + 1] - ki) >> 3);
            pos_out[tp + split_off[s] + c] = static_cast<uint32_t>(lower_bound_u64(P, pos[i], pos[i + 1], key));
        }
        __syncthreads();
    }
    if (tid == 0 && any_change) atomicOr(&st->changed[round], 1u);
}

struct RebalanceWs {
    uint64_t* K_alt;
    uint32_t* pos[2];
    LoopState* st;
    uint64_t* lb;
    size_t lb_words;
    size_t bytes;
};

RebalanceWs carve_rebalance(void* ws, size_t cap) {
    Carve c(ws);
    RebalanceWs r{};
    r.K_alt = c.take<uint64_t>(cap + 1);
    r.pos[0] = c.take<uint32_t>(cap + 1);
    r.pos[1] = c.take<uint32_t>(cap + 1);
    r.st = c.take<LoopState>(1);
    r.lb_words = (cap + kRTile - 1) / kRTile + 1;
    r.lb = c.take<uint64_t>(r.lb_words);
    r.bytes = c.off;
    return r;
}

uint32_t grid_1d(size_t items, int block) { return static_cast<uint32_t>((items + block - 1) / block); }

}  // namespace

cstone_status launch_node_counts(const uint64_t* sorted_keys, size_t n, const uint64_t* leaves, size_t n_leaves,
                                 uint32_t* counts, hipStream_t stream) {
    if (n_leaves == 0) return CSTONE_OK;
    hipLaunchKernelGGL(node_counts_kernel, dim3(grid_1d(n_leaves, kCountBlock)), dim3(kCountBlock), 0, stream,
                       sorted_keys, n, leaves, n_leaves, counts);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

size_t rebalance_workspace_bytes(size_t leaf_capacity) { return carve_rebalance(nullptr, leaf_capacity).bytes; }

cstone_status run_rebalance(const uint64_t* P, size_t n, uint32_t n_crit, uint64_t* leaves, size_t* n_leaves,
                            size_t cap, uint32_t* counts, uint32_t max_iters, uint32_t* iters_done, void* ws,
                            size_t ws_bytes, hipStream_t stream, const uint32_t* input_flags,
                            uint32_t* input_flags_out) {
    RebalanceWs w = carve_rebalance(ws, cap);
    if (ws_bytes < w.bytes) return CSTONE_ERR_INVALID_ARG;
    const size_t nl0 = *n_leaves;
    if (nl0 < 1 || nl0 > cap) return CSTONE_ERR_INVALID_ARG;
    if (max_iters == 0) max_iters = kL + 1;
    if (max_iters > kMaxRounds) max_iters = kMaxRounds;

    uint64_t* bufK[2] = {leaves, w.K_alt};
    const int root = nl0 == 1;
    uint32_t init_grid = grid_1d(std::max<size_t>(w.lb_words, kMaxRounds + 1), 256);
    if (init_grid > 1024) init_grid = 1024;
    hipLaunchKernelGGL(loop_init_kernel, dim3(init_grid), dim3(256), 0, stream, w.st, static_cast<uint64_t>(nl0),
                       w.lb, w.lb_words, w.pos[0], static_cast<uint32_t>(n), root, leaves, input_flags);
    if (!root)
        hipLaunchKernelGGL(positions_kernel, dim3(grid_1d(nl0 + 1, kCountBlock)), dim3(kCountBlock), 0, stream, P, n,
                           leaves, nl0, w.pos[0]);
    CS_HIP(hipGetLastError());

    // rounds expected from the root: about log8(n / (n_crit + 1)) + 2
    uint32_t batch = 2;
    if (root) {
        double ratio = static_cast<double>(n) / (static_cast<double>(n_crit) + 1.0);
        uint32_t est = 2;
        while (ratio > 1.0) {
            ratio /= 8.0;
            ++est;
        }
        batch = est;
    }
    LoopState host{};
    uint32_t done = 0;
    int outcome = 0;  // 1 converged, 2 capacity, 3 not converged
    uint32_t final_round = 0;
    while (outcome == 0) {
        const uint32_t b = std::min(batch, max_iters - done);
        for (uint32_t q = done; q < done + b; ++q) {
            double bound = static_cast<double>(nl0);
            for (uint32_t e = 0; e < q && bound < static_cast<double>(cap); ++e) bound *= 8.0;
            const size_t rows = std::min<double>(bound, static_cast<double>(cap));
            uint32_t grid = grid_1d(rows, kRTile);
            if (grid > kMaxRoundGrid) grid = kMaxRoundGrid;
            if (grid < 1) grid = 1;
            hipLaunchKernelGGL(round_kernel, dim3(grid), dim3(kRBlock), 0, stream, P, static_cast<uint32_t>(n),
                               n_crit, bufK[q & 1], w.pos[q & 1], bufK[(q + 1) & 1], w.pos[(q + 1) & 1], w.st,
                               static_cast<int>(q), static_cast<uint64_t>(cap), w.lb);
        }
        CS_HIP(hipGetLastError());
        done += b;
        CS_HIP(hipMemcpyAsync(&host, w.st, sizeof(LoopState), hipMemcpyDeviceToHost, stream));
        CS_HIP(hipStreamSynchronize(stream));
        if (input_flags_out) *input_flags_out = host.input_flags;
        if (host.err) return CSTONE_ERR_DEVICE;
        for (uint32_t q = 0; q < done; ++q) {
            if (host.nl[q + 1] > cap) {
                outcome = 2;
                final_round = q;
                break;
            }
            if (host.changed[q] == 0) {
                outcome = 1;
                final_round = q;
                break;
            }
        }
        if (outcome == 0 && done >= max_iters) {
            outcome = 3;
            final_round = max_iters;
        }
        batch = 2;
    }

    // array after the last complete round lives in buffer (round + 1) & 1 for
    // a converged loop, round & 1 otherwise
    uint32_t buf;
    size_t nl_final;
    if (outcome == 1) {
        buf = (final_round + 1) & 1;
        nl_final = host.nl[final_round + 1];
    } else if (outcome == 2) {
        buf = final_round & 1;
        nl_final = host.nl[final_round];
    } else {
        buf = final_round & 1;
        nl_final = host.nl[final_round];
    }
    if (buf == 1) CS_HIP(hipMemcpyAsync(leaves, w.K_alt, (nl_final + 1) * sizeof(uint64_t),
                                        hipMemcpyDeviceToDevice, stream));
    if (counts)
        hipLaunchKernelGGL(counts_from_positions_kernel, dim3(grid_1d(nl_final, kCountBlock)), dim3(kCountBlock), 0,
                           stream, w.pos[buf], nl_final, counts);
    CS_HIP(hipGetLastError());
    CS_HIP(hipStreamSynchronize(stream));

    if (iters_done) *iters_done = outcome == 1 ? final_round + 1 : final_round;
    if (outcome == 2) {
        *n_leaves = host.nl[final_round + 1];
        return CSTONE_ERR_CAPACITY;
    }
    *n_leaves = nl_final;
    return outcome == 3 ? CSTONE_ERR_NOT_CONVERGED : CSTONE_OK;
}

}  // namespace cs
