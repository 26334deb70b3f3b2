// Stable LSD radix sort of uint64 keys with a uint32 permutation (the sorted
// particle keys P of Sec. 4 and the node keys of Sec. 5, step 3).
//
// One pass per digit, each a single "onesweep" kernel: a block takes a tile of
// keys, ranks them by digit inside the tile with wave64 ballots (stable: ranks
// follow wave, item, lane order, which is the input order), publishes its
// per-digit totals, and obtains the totals of all earlier tiles by decoupled
// look-back over agent-scope atomics (coherent across the XCDs' separate L2s).
// The tile is then reordered in LDS so that the global stores of every digit
// run are contiguous. A histogram kernel counts all digit positions in one
// read of the keys before the first pass.
#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr int kBits = 8;
constexpr int kRadix = 1 << kBits;
constexpr int kBlock = 256;
constexpr int kItems = 16;
constexpr int kTile = kBlock * kItems;
constexpr int kWaves = kBlock / kWave;
constexpr int kMaxPasses = 8;
constexpr int kHistBlock = 256;

static_assert(kRadix == kBlock, "one digit per thread in the per-tile digit loops");

__global__ __launch_bounds__(256) void sort_init_kernel(uint32_t* ghist, uint32_t* counters, uint32_t* err) {
    for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += blockDim.x) ghist[i] = 0;
    if (threadIdx.x < kMaxPasses) counters[threadIdx.x] = 0;
    if (threadIdx.x == 0) *err = 0;
}

// Digit histograms of every pass in one read of the keys; also clears the
// look-back words (epoch 0 = never written).
__global__ __launch_bounds__(kHistBlock) void sort_hist_kernel(const uint64_t* __restrict__ keys, size_t n,
                                                                int passes, uint32_t* __restrict__ ghist,
                                                                uint64_t* __restrict__ lb, size_t lb_words) {
    __shared__ uint32_t h[kMaxPasses][kRadix];
    for (int i = threadIdx.x; i < kMaxPasses * kRadix; i += kHistBlock) (&h[0][0])[i] = 0;
    __syncthreads();
    const size_t stride = static_cast<size_t>(gridDim.x) * kHistBlock;
    const size_t first = static_cast<size_t>(blockIdx.x) * kHistBlock + threadIdx.x;
    for (size_t i = first; i < n; i += stride) {
        uint64_t k = keys[i];
        for (int p = 0; p < passes; ++p) atomicAdd(&h[p][(k >> (p * kBits)) & (kRadix - 1)], 1u);
    }
    for (size_t i = first; i < lb_words; i += stride) lb[i] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < passes * kRadix; i += kHistBlock) {
        uint32_t c = (&h[0][0])[i];
        if (c) atomicAdd(&ghist[i], c);
    }
}

template <bool FIRST, bool WITH_VALUES>
__global__ __launch_bounds__(kBlock) void onesweep_kernel(const uint64_t* __restrict__ keys_in,
                                                           const uint32_t* __restrict__ vals_in,
                                                           uint64_t* __restrict__ keys_out,
                                                           uint32_t* __restrict__ vals_out, size_t n, int shift,
                                                           const uint32_t* __restrict__ ghist, uint64_t* lb,
                                                           uint32_t* counter, uint32_t epoch, uint32_t* err) {
    __shared__ union {
        uint64_t keys[kTile];
        uint32_t vals[kTile];
    } stage;
    __shared__ uint32_t whist[kWaves][kRadix];
    __shared__ uint64_t ddelta[kRadix];
    __shared__ uint32_t local_start[kRadix];
    __shared__ uint32_t scan_tmp[kWaves];
    __shared__ uint32_t slot;

    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = tid / kWave;
    const uint32_t tile = take_tile(counter, &slot);
    const size_t tile_base = static_cast<size_t>(tile) * kTile;
    const uint32_t tile_count = static_cast<uint32_t>(n - tile_base < kTile ? n - tile_base : kTile);

    for (int w = 0; w < kWaves; ++w) whist[w][tid] = 0;

    uint64_t k[kItems];
    uint32_t v[kItems];
    const size_t wave_base = tile_base + static_cast<size_t>(wave) * kItems * kWave;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        size_t idx = wave_base + static_cast<size_t>(i) * kWave + lane;
        bool ok = idx < n;
        k[i] = ok ? keys_in[idx] : 0ull;
        if (WITH_VALUES) v[i] = FIRST ? static_cast<uint32_t>(idx) : (ok ? vals_in[idx] : 0u);
    }
    __syncthreads();

    // Stable rank of every key among the keys of its wave with the same digit.
    uint32_t rank[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        size_t idx = wave_base + static_cast<size_t>(i) * kWave + lane;
        bool ok = idx < n;
        uint32_t d = static_cast<uint32_t>(k[i] >> shift) & (kRadix - 1);
        uint64_t peers = __ballot(ok);
#pragma unroll
        for (int b = 0; b < kBits; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        uint32_t below = lanes_below(peers);
        uint32_t base = whist[wave][d];
        if (ok && below == 0) whist[wave][d] = base + static_cast<uint32_t>(__popcll(peers));
        rank[i] = base + below;
    }
    __syncthreads();

    // Per digit (one per thread): wave offsets within the tile and the tile total.
    const uint32_t d_own = tid;
    uint32_t total = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        uint32_t c = whist[w][d_own];
        whist[w][d_own] = total;
        total += c;
    }
    uint64_t* my_words = lb + static_cast<size_t>(tile) * kRadix + d_own;
    if (tile == 0)
        st_agent(my_words, lb_word(kFlagInc, epoch, total));
    else
        st_agent(my_words, lb_word(kFlagAgg, epoch, total));

    uint32_t dummy;
    uint32_t lstart = block_exclusive_sum<uint32_t, kBlock>(total, scan_tmp, &dummy);
    uint32_t gbase = block_exclusive_sum<uint32_t, kBlock>(ghist[d_own], scan_tmp, &dummy);
    uint64_t excl = 0;
    if (tile != 0) {
        excl = lookback(lb + d_own, kRadix, tile, epoch, err);
        st_agent(my_words, lb_word(kFlagInc, epoch, excl + total));
    }
    local_start[d_own] = lstart;
    ddelta[d_own] = static_cast<uint64_t>(gbase) + excl - lstart;
    __syncthreads();

    // Reorder the tile by digit in LDS, then store each digit run contiguously.
    uint32_t lpos[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        size_t idx = wave_base + static_cast<size_t>(i) * kWave + lane;
        uint32_t d = static_cast<uint32_t>(k[i] >> shift) & (kRadix - 1);
        lpos[i] = local_start[d] + whist[wave][d] + rank[i];
        if (idx < n) stage.keys[lpos[i]] = k[i];
    }
    __syncthreads();
    uint64_t dst[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        uint32_t j = static_cast<uint32_t>(i) * kBlock + tid;
        if (j < tile_count) {
            uint64_t key = stage.keys[j];
            uint32_t d = static_cast<uint32_t>(key >> shift) & (kRadix - 1);
            dst[i] = j + ddelta[d];
            if (dst[i] < n) keys_out[dst[i]] = key;  // always true; guards memory against a logic error
        }
    }
    if (WITH_VALUES) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            size_t idx = wave_base + static_cast<size_t>(i) * kWave + lane;
            if (idx < n) stage.vals[lpos[i]] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kItems; ++i) {
            uint32_t j = static_cast<uint32_t>(i) * kBlock + tid;
            if (j < tile_count && dst[i] < n) vals_out[dst[i]] = stage.vals[j];
        }
    }
}

struct SortWs {
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* ghist;
    uint32_t* counters;
    uint32_t* err;
    uint64_t* lb;
    size_t lb_words;
    size_t bytes;
};

SortWs carve_sort(void* ws, size_t n, bool with_perm) {
    Carve c(ws);
    SortWs s{};
    s.keys_alt = c.take<uint64_t>(n);
    s.vals_alt = with_perm ? c.take<uint32_t>(n) : nullptr;
    s.ghist = c.take<uint32_t>(kMaxPasses * kRadix);
    s.counters = c.take<uint32_t>(kMaxPasses);
    s.err = c.take<uint32_t>(1);
    size_t tiles = (n + kTile - 1) / kTile;
    s.lb_words = tiles * kRadix;
    s.lb = c.take<uint64_t>(s.lb_words);
    s.bytes = c.off;
    return s;
}

}  // namespace

size_t sort_workspace_bytes(size_t n, bool with_perm) { return carve_sort(nullptr, n, with_perm).bytes; }

int sort_passes(int sig_bits) { return (sig_bits + kBits - 1) / kBits; }

cstone_status launch_sort(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n,
                          int sig_bits, void* ws, size_t ws_bytes, hipStream_t stream, hipEvent_t* pass_events) {
    const bool with_perm = perm_out != nullptr;
    SortWs s = carve_sort(ws, n, with_perm);
    if (ws_bytes < s.bytes) return CSTONE_ERR_INVALID_ARG;
    if (n == 0) return CSTONE_OK;
    const int passes = sort_passes(sig_bits);
    if (passes < 1 || passes > kMaxPasses) return CSTONE_ERR_INVALID_ARG;

    hipLaunchKernelGGL(sort_init_kernel, dim3(1), dim3(256), 0, stream, s.ghist, s.counters, s.err);
    size_t hblocks = (n + kHistBlock * 16 - 1) / (kHistBlock * 16);
    if (hblocks > 1024) hblocks = 1024;
    if (hblocks < 1) hblocks = 1;
    hipLaunchKernelGGL(sort_hist_kernel, dim3(hblocks), dim3(kHistBlock), 0, stream, keys_in, n, passes, s.ghist,
                       s.lb, s.lb_words);

    const uint32_t tiles = static_cast<uint32_t>((n + kTile - 1) / kTile);
    if (pass_events) CS_HIP(hipEventRecord(pass_events[0], stream));
    const uint64_t* src_k = keys_in;
    const uint32_t* src_v = nullptr;
    for (int p = 0; p < passes; ++p) {
        bool to_out = ((passes - 1 - p) % 2) == 0;
        uint64_t* dk = to_out ? keys_out : s.keys_alt;
        uint32_t* dv = with_perm ? (to_out ? perm_out : s.vals_alt) : nullptr;
        const uint32_t* gh = s.ghist + p * kRadix;
        uint32_t epoch = static_cast<uint32_t>(p + 1);
        if (with_perm) {
            if (p == 0)
                hipLaunchKernelGGL((onesweep_kernel<true, true>), dim3(tiles), dim3(kBlock), 0, stream, src_k, src_v,
                                   dk, dv, n, p * kBits, gh, s.lb, s.counters + p, epoch, s.err);
            else
                hipLaunchKernelGGL((onesweep_kernel<false, true>), dim3(tiles), dim3(kBlock), 0, stream, src_k,
                                   src_v, dk, dv, n, p * kBits, gh, s.lb, s.counters + p, epoch, s.err);
        } else {
            hipLaunchKernelGGL((onesweep_kernel<false, false>), dim3(tiles), dim3(kBlock), 0, stream, src_k, src_v,
                               dk, dv, n, p * kBits, gh, s.lb, s.counters + p, epoch, s.err);
        }
        src_k = dk;
        src_v = dv;
        if (pass_events) CS_HIP(hipEventRecord(pass_events[p + 1], stream));
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace cs
