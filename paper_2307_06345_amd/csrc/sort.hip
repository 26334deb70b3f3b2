// Stable LSD radix sort of uint64 keys with a uint32 permutation (the sorted
// particle keys P of Sec. 4 and the node keys of Sec. 5, step 3).
//
// One pass per digit (8 or 9 bits), each a single "onesweep" kernel. A block
// takes the tile of its block index, ranks its keys by digit with wave64
// ballots (stable: ranks follow wave, item, lane order, which is the input
// order), reorders the tile by digit in LDS, and only then obtains the counts
// of all earlier tiles by decoupled look-back over agent-scope atomics
// (coherent across the XCDs' separate L2s), so the wait overlaps local work.
// Every digit run is then stored contiguously. Each pass also counts the next
// pass's digit, so only the first digit needs a histogram of its own (which the
// key kernel of a build provides while writing the keys).
#include <algorithm>

#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr int kMaxRadix = 512;  // 9-bit digits
constexpr int kMaxPasses = 8;
constexpr int kHistBlock = 256;
constexpr int kMinTile = 2048;  // smallest tile of any variant (sizes the look-back rows)

__global__ __launch_bounds__(256) void sort_init_kernel(uint32_t* ghist, size_t ghist_words, uint32_t* err,
                                                        uint64_t* lb, size_t lb_words, uint32_t* extra) {
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = t; i < lb_words; i += stride) lb[i] = 0;  // flag 0: not yet written
    for (size_t i = t; i < ghist_words; i += stride) ghist[i] = 0;
    if (t == 0) {
        *err = 0;
        if (extra) *extra = 0;  // a caller's word cleared along the way
    }
}

// Set-up of a build's sort from the key kernel's per-block parts (rows of
// kKeyDigitsMax x kMaxRadix words, one per key block): block j < digits *
// kMaxRadix / kSetupCols sums columns [j * kSetupCols, (j + 1) * kSetupCols)
// over the parts' rows (column p * kMaxRadix + v: digit value v of pass p),
// reading whole row segments; the last block ORs the blocks' flags into *flag;
// all blocks clear what sort_init_kernel clears (but the counts summed here).
constexpr uint32_t kSetupCols = kWave;
constexpr uint32_t kSetupGroups = kKeyBlocksMax / kSetupCols;  // row groups of a summing block
__global__ __launch_bounds__(kKeyBlocksMax) void sort_setup_kernel(uint32_t* ghist, size_t ghist_words, uint32_t* err,
                                                                  uint64_t* lb, size_t lb_words,
                                                                  const uint32_t* __restrict__ parts, uint32_t nparts,
                                                                  uint32_t radix, uint32_t digits,
                                                                  const uint32_t* __restrict__ bad,
                                                                  uint32_t* flag, uint32_t* level6) {
    __shared__ uint32_t red[kKeyBlocksMax];
    const uint32_t tid = threadIdx.x;
    const size_t t = static_cast<size_t>(blockIdx.x) * blockDim.x + tid;
    const size_t stride = static_cast<size_t>(gridDim.x) * blockDim.x;
    for (size_t i = t; i < lb_words; i += stride) lb[i] = 0;
    if (level6)
        for (size_t i = t; i < kLevel6Cells; i += stride) level6[i] = kCellEmpty;
    for (size_t i = digits * radix + t; i < ghist_words; i += stride) ghist[i] = 0;
    const uint32_t sums = digits * kMaxRadix / kSetupCols;
    const uint32_t j = blockIdx.x;
    if (j < sums) {  // block-uniform
        constexpr uint32_t kRows = kKeyBlocksMax / kSetupGroups;  // rows per thread at most
        const uint32_t col = j * kSetupCols + tid % kSetupCols, g = tid / kSetupCols;
        uint32_t acc = 0;
        // rows g, g + kSetupGroups, ...: every load in flight (a row past nparts
        // reads row 0, not counted)
        uint32_t v[kRows];
#pragma unroll
        for (uint32_t q = 0; q < kRows; ++q) {
            const uint32_t r = g + q * kSetupGroups;
            v[q] = parts[static_cast<size_t>(r < nparts ? r : 0u) * (kKeyDigitsMax * kMaxRadix) + col];
        }
#pragma unroll
        for (uint32_t q = 0; q < kRows; ++q) acc += g + q * kSetupGroups < nparts ? v[q] : 0u;
        red[tid] = acc;
        __syncthreads();
        if (tid < kSetupCols) {
            uint32_t total = 0;
            for (uint32_t w = 0; w < kSetupGroups; ++w) total += red[w * kSetupCols + tid];
            const uint32_t p = col / kMaxRadix, d = col % kMaxRadix;
            if (d < radix) ghist[p * radix + d] = total;
        }
    } else if (j == sums) {  // block-uniform: the flags
        const uint32_t f = tid < nparts ? bad[tid] : 0u;
        const uint32_t any = __syncthreads_or(f != 0);
        if (tid == 0) {
            *flag = any ? CSTONE_FLAG_NONFINITE : 0u;
            *err = 0;
        }
    }
}

// Counts of the first pass's digit ((key >> shift) & mask, mask = radix - 1).
__global__ __launch_bounds__(kHistBlock) void sort_hist0_kernel(const uint64_t* __restrict__ keys, uint32_t n,
                                                                 uint32_t shift, uint32_t mask,
                                                                 uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[kMaxRadix];
    for (int i = threadIdx.x; i < kMaxRadix; i += kHistBlock) h[i] = 0;
    __syncthreads();
    const uint32_t stride = gridDim.x * kHistBlock;
    for (uint32_t i = blockIdx.x * kHistBlock + threadIdx.x; i < n; i += stride)
        atomicAdd(&h[static_cast<uint32_t>(keys[i] >> shift) & mask], 1u);
    __syncthreads();
    for (int i = threadIdx.x; i <= static_cast<int>(mask); i += kHistBlock)
        if (h[i]) atomicAdd(&ghist[i], h[i]);
}

// Look-back words. 32-bit: [31:30] flag, [29:0] value (n < 2^30), cleared
// for every pass (double buffer: pass p clears the rows pass p+1 will use).
// 64-bit: flag, 14-bit epoch (the pass that wrote it) and value, cleared once.
struct Lb32 {
    using word = uint32_t;
    __device__ static word make(uint32_t flag, uint32_t, uint64_t v) {
        return (flag << 30) | static_cast<uint32_t>(v & 0x3fffffffu);
    }
    __device__ static uint32_t flag(word w, uint32_t) { return w >> 30; }
    __device__ static uint64_t value(word w) { return w & 0x3fffffffu; }
    __device__ static word load(const word* p) {
        return __hip_atomic_load(const_cast<word*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static void store(word* p, word w) {
        __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // store w if the word still holds `seen`
    __device__ static void replace(word* p, word seen, word w) {
        __hip_atomic_compare_exchange_strong(p, &seen, w, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    }
};
struct Lb64 {
    using word = uint64_t;
    __device__ static word make(uint32_t flag, uint32_t epoch, uint64_t v) {
        return (static_cast<uint64_t>(flag) << 62) | (static_cast<uint64_t>(epoch & 0x3fffu) << 48) |
               (v & kValueMask);
    }
    __device__ static uint32_t flag(word w, uint32_t epoch) {
        return ((w >> 48) & 0x3fffu) == (epoch & 0x3fffu) ? static_cast<uint32_t>(w >> 62) : 0u;
    }
    __device__ static uint64_t value(word w) { return w & kValueMask; }
    __device__ static word load(const word* p) { return ld_agent(p); }
    __device__ static void store(word* p, word w) { st_agent(p, w); }
    __device__ static void replace(word* p, word seen, word w) {
        __hip_atomic_compare_exchange_strong(p, &seen, w, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    }
};

// Walk of one digit's exclusive prefix back over the tiles before this one
// (rows of `radix` words): from tile p down to `first`, WIN predecessors per
// round trip, nearest first, summing aggregates into excl until an inclusive
// prefix. Returns true when the prefix is complete; false when the word of
// tile p was still empty after `patience` waits (p and excl keep the progress,
// so a later call resumes there).
template <class LB, int WIN>
__device__ __forceinline__ bool digit_lookback_step(const typename LB::word* col, uint32_t radix, int64_t lo,
                                                    uint32_t epoch, uint32_t patience, int64_t& p, uint64_t& excl) {
    uint32_t waits = 0;
    while (p >= lo) {
        typename LB::word w[WIN];
#pragma unroll
        for (int q = 0; q < WIN; ++q) w[q] = p - q >= lo ? LB::load(col + static_cast<size_t>(p - q) * radix) : 0;
        bool done = false, stalled = false;
#pragma unroll
        for (int q = 0; q < WIN; ++q) {
            if (done || stalled || p < lo) continue;
            const uint32_t f = LB::flag(w[q], epoch);
            if (f == 0) {
                stalled = true;
                continue;
            }
            excl += LB::value(w[q]);
            if (f == 2) done = true;
            --p;
        }
        if (done) return true;
        if (stalled) {
            if (++waits > patience) return false;
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return true;
}

template <int BITS>
__device__ __forceinline__ uint32_t digit_of(uint64_t k, uint32_t shift) {
    return static_cast<uint32_t>(k >> shift) & ((1u << BITS) - 1u);
}

// Lanes of this wave whose digit equals this lane's, among the lanes in `valid`.
template <int BITS>
__device__ __forceinline__ uint64_t match_digit(uint32_t d, uint64_t valid) {
    uint32_t lo = static_cast<uint32_t>(valid), hi = static_cast<uint32_t>(valid >> 32);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
        const uint32_t bit = (d >> b) & 1u;
        const uint64_t bal = __ballot(bit);
        const uint32_t keep_if_clear = bit - 1u;  // all ones where this lane's bit is 0
        lo &= static_cast<uint32_t>(bal) ^ keep_if_clear;
        hi &= static_cast<uint32_t>(bal >> 32) ^ keep_if_clear;
    }
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// One tile of a pass: `base` .. `base + count` of the keys, in the segment
// whose first tile is `first` and whose particles start at `seg_base`
// (segment-relative permutation values; the plain sort is one segment).
// Minimum waves per SIMD (the second launch bound): room for two blocks per
// CU (4 SIMDs) when a block's LDS (mostly the 8-byte keys of its tile) stays
// below half of the CU's 160 KB, so that one block's waits overlap the other's
// work; otherwise one block, which may then use up to 256 VGPRs a lane.
template <int BLOCK, int ITEMS>
constexpr int kMinBlocks = (BLOCK <= 512 && BLOCK * ITEMS * 8 <= 72 * 1024 ? 2 : 1) * BLOCK / (4 * kWave);

// Tile of block b. Blocks are dealt to the 8 XCDs in turn; every XCD takes
// kXcdGroup consecutive tiles of each round of 8 kXcdGroup blocks, so that
// where one tile's run of a digit ends and the next tile's run begins (a
// partly written 64-byte segment) both writes meet in the same L2. The last,
// incomplete round keeps tile = block. A tile may then wait on a tile whose
// block has not started: each XCD starts its own share of the grid, at its
// own pace, and kernels on other streams may hold an XCD full. Such a wait
// does not depend on that block: after a while the waiting block counts the
// missing tile's digits itself (the look-back's fallback).
constexpr uint32_t kXcdGroup = 16;
// Waits (each one look-back round trip and a short sleep) before a block counts
// a missing predecessor tile's digits itself: by default far longer than a
// started block takes to publish its counts. Settable per device (0 sends
// every wait to the fallback, which tests use).
constexpr uint32_t kLookbackPatience = 256;
__constant__ uint32_t g_lookback_patience = kLookbackPatience;

__device__ __forceinline__ uint32_t tile_of_block(uint32_t b, uint32_t nblocks) {
    constexpr uint32_t R = 8u * kXcdGroup;
    if (b >= nblocks / R * R) return b;
    const uint32_t r = b / R, q = b % R;
    return (r * 8u + q % 8u) * kXcdGroup + q / 8u;
}

struct TileDesc {
    uint32_t tile, base, count, first, seg_base;
};

template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool WITH_VALUES, class LB, bool FULL>
__device__ __forceinline__ void onesweep_tile(const TileDesc td, const uint64_t* __restrict__ keys_in,
                                              const uint32_t* __restrict__ vals_in, uint64_t* __restrict__ keys_out,
                                              uint32_t* __restrict__ vals_out, uint32_t n, uint32_t shift,
                                              const uint32_t* __restrict__ ghist, uint32_t* __restrict__ ghist_next,
                                              uint32_t shift_next, typename LB::word* lb, uint32_t epoch,
                                              uint32_t* err, uint64_t* stage, uint16_t (*whist)[1 << BITS],
                                              uint32_t* nhist, uint32_t* ddelta, uint64_t* scan_tmp,
                                              const uint4* __restrict__ table) {
    constexpr int RADIX = 1 << BITS;
    constexpr int W = BLOCK / kWave;
    constexpr int TILE = BLOCK * ITEMS;
    uint32_t* stage32 = reinterpret_cast<uint32_t*>(stage);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / kWave);  // wave-uniform, in a scalar register
    const uint32_t tile = td.tile;
    const uint32_t tile_base = td.base;
    const uint32_t tile_count = FULL ? static_cast<uint32_t>(TILE) : td.count;
    const uint32_t end = tile_base + tile_count;  // keys at or past `end` belong to others
    const uint32_t wave_base = tile_base + wave * ITEMS * kWave;

    // this pass's digit counts of the whole set, for the global digit offsets
    const uint32_t gcount = tid < RADIX ? ghist[tid] : 0u;
    // item i of this lane sits at wave_base + lane + i * kWave: one base pointer
    // and constant offsets (a 32-bit index per item would keep 16 widened
    // indices live from the key loads to the value loads)
    const uint64_t* kp = keys_in + (wave_base + lane);
    uint64_t k[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = wave_base + i * kWave + lane;
        k[i] = (FULL || idx < end) ? kp[i * kWave] : 0ull;
    }
    __syncthreads();  // counters cleared

    // stable rank of every key among the keys of its wave with the same digit
    // (below TILE <= 2^16: two ranks per register, which keeps the keys out of
    // scratch)
    static_assert(TILE <= 65536, "ranks and tile positions are packed in 16 bits");
    uint32_t rank2[(ITEMS + 1) / 2];
#pragma unroll
    for (int i = 0; i < (ITEMS + 1) / 2; ++i) rank2[i] = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = wave_base + i * kWave + lane;
        const bool ok = FULL || idx < end;
        const uint32_t d = digit_of<BITS>(k[i], shift);
        if (ghist_next && ok) atomicAdd(&nhist[digit_of<BITS>(k[i], shift_next)], 1u);
        const uint64_t peers = match_digit<BITS>(d, FULL ? ~0ull : __ballot(ok));
        const uint32_t below = lanes_below(peers);
        const uint32_t base = whist[wave][d];
        if (ok && below == 0) whist[wave][d] = static_cast<uint16_t>(base + static_cast<uint32_t>(__popcll(peers)));
        rank2[i / 2] |= ((base + below) & 0xffffu) << ((i & 1) * 16);
    }
    __syncthreads();

    // per digit (one per thread): wave offsets and tile total; publish the aggregate
    uint32_t total = 0;
    if (tid < RADIX) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
            const uint32_t c = whist[w][tid];
            whist[w][tid] = static_cast<uint16_t>(total);
            total += c;
        }
        LB::store(lb + static_cast<size_t>(tile) * RADIX + tid, LB::make(tile == td.first ? 2u : 1u, epoch, total));
    }
    // one scan for both: high word global start of the digit, low word its tile-local start
    uint64_t dummy;
    const uint64_t both = block_exclusive_sum<uint64_t, BLOCK>((static_cast<uint64_t>(gcount) << 32) | total,
                                                               scan_tmp, &dummy);
    const uint32_t lst = static_cast<uint32_t>(both);
    const uint32_t gbase = static_cast<uint32_t>(both >> 32);
    if (tid < RADIX) {
#pragma unroll
        for (int w = 0; w < W; ++w) whist[w][tid] += static_cast<uint16_t>(lst);  // tile-local start of (digit, wave)
    }
    __syncthreads();

    // reorder the tile by digit in LDS before waiting on the other tiles
    uint32_t lpos2[(ITEMS + 1) / 2];  // tile positions, two per register
#pragma unroll
    for (int i = 0; i < (ITEMS + 1) / 2; ++i) lpos2[i] = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = wave_base + i * kWave + lane;
        const uint32_t lp = (whist[wave][digit_of<BITS>(k[i], shift)] + ((rank2[i / 2] >> ((i & 1) * 16)) & 0xffffu)) & 0xffffu;
        lpos2[i / 2] |= lp << ((i & 1) * 16);
        if (FULL || idx < end) stage[lp] = k[i];
    }
    // the permutation values are only needed for the scatter: start loading them
    // (not earlier: the keys must be dead by then to keep the registers in budget)
    __builtin_amdgcn_sched_barrier(0);
    uint32_t v[ITEMS];
    if constexpr (WITH_VALUES && FIRST) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) v[i] = wave_base + i * kWave + lane - td.seg_base;
    } else if constexpr (WITH_VALUES) {
        const uint32_t* vp = vals_in + (wave_base + lane);
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = wave_base + i * kWave + lane;
            v[i] = (FULL || idx < end) ? vp[i * kWave] : 0u;
        }
    }
    // every digit's exclusive prefix over the tiles before this one (one
    // digit per thread). A walk that has waited g_lookback_patience times on a
    // tile gets that tile's digit counts from this block instead (the
    // fallback): the block counts them from the tile's keys and publishes
    // them as the tile's aggregates, unless the tile's own block has written
    // its word by then. The counts are the ones that block would publish, so
    // the result is the same either way, and no wait depends on another block
    // having started. Each round settles at least one tile, so the loop ends.
    __shared__ uint32_t help;
    uint64_t excl = 0;
    int64_t p = static_cast<int64_t>(tile) - 1;
    bool done = tid >= static_cast<uint32_t>(RADIX) || tile == td.first;
    for (uint32_t round = 0;; ++round) {
        if (!done)
            done = digit_lookback_step<LB, WIN>(lb + tid, RADIX, td.first, epoch, g_lookback_patience, p, excl);
        if (!__syncthreads_or(!done)) break;
        if (round > tile - td.first) {  // never: every round settles a tile
            if (tid == 0) atomicOr(err, kErrSpin);
            break;
        }
        if (tid == 0) help = 0;
        for (int i = tid; i < RADIX; i += BLOCK) ddelta[i] = 0;  // the helped tile's digit counts
        __syncthreads();
        if (!done) atomicMax(&help, static_cast<uint32_t>(p));  // the nearest tile a walk waits on
        __syncthreads();
        const uint32_t q = help;
        uint32_t q_base, q_count;
        if (table) {
            const uint4 t = table[q];
            q_base = t.x;
            q_count = t.y;
        } else {
            q_base = q * static_cast<uint32_t>(TILE);
            q_count = min(n - q_base, static_cast<uint32_t>(TILE));
        }
        for (uint32_t j = tid; j < q_count; j += BLOCK) atomicAdd(&ddelta[digit_of<BITS>(keys_in[q_base + j], shift)], 1u);
        __syncthreads();
        if (tid < RADIX) {
            typename LB::word* w = lb + static_cast<size_t>(q) * RADIX + tid;
            const typename LB::word seen = LB::load(w);
            if (LB::flag(seen, epoch) == 0) LB::replace(w, seen, LB::make(1u, epoch, ddelta[tid]));
        }
        __syncthreads();  // help and the counts are reused by the next round
    }
    if (tid < RADIX) {
        if (tile != td.first) LB::store(lb + static_cast<size_t>(tile) * RADIX + tid, LB::make(2u, epoch, excl + total));
        // destination of tile-local position j is j + ddelta (mod 2^32; every index is below 2^32)
        ddelta[tid] = td.seg_base + gbase + static_cast<uint32_t>(excl) - lst;
        if (ghist_next && nhist[tid]) atomicAdd(&ghist_next[tid], nhist[tid]);
    }
    __syncthreads();

    // store each digit run contiguously; keep the digits (two per register)
    // for the values, which follow the keys through the same LDS buffer
    uint32_t dpk[(ITEMS + 1) / 2];
#pragma unroll
    for (int i = 0; i < (ITEMS + 1) / 2; ++i) dpk[i] = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
        if (FULL || j < tile_count) {
            const uint64_t key = stage[j];
            const uint32_t d = digit_of<BITS>(key, shift);
            dpk[i / 2] |= d << ((i & 1) * 16);
            const uint32_t to = j + ddelta[d];
            if (to < n) keys_out[to] = key;  // always true; guards memory against a logic error
        }
    }
    if (WITH_VALUES) {
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = wave_base + i * kWave + lane;
            if (FULL || idx < end) stage32[(lpos2[i / 2] >> ((i & 1) * 16)) & 0xffffu] = v[i];
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
            if (FULL || j < tile_count) {
                const uint32_t to = j + ddelta[(dpk[i / 2] >> ((i & 1) * 16)) & 0xffffu];
                if (to < n) vals_out[to] = stage32[j];
            }
        }
    }
}


template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool WITH_VALUES, class LB>
__global__ __launch_bounds__(BLOCK, (kMinBlocks<BLOCK, ITEMS>)) void onesweep_kernel(const uint64_t* __restrict__ keys_in,
                                                          const uint32_t* __restrict__ vals_in,
                                                          uint64_t* __restrict__ keys_out,
                                                          uint32_t* __restrict__ vals_out, uint32_t n, uint32_t shift,
                                                          const uint32_t* __restrict__ ghist,
                                                          uint32_t* __restrict__ ghist_next, uint32_t shift_next,
                                                          typename LB::word* lb, typename LB::word* lb_clear,
                                                          uint32_t epoch, uint32_t* err) {
    constexpr int RADIX = 1 << BITS;
    constexpr int W = BLOCK / kWave;
    constexpr int TILE = BLOCK * ITEMS;
    static_assert(BLOCK >= RADIX, "one digit per thread in the digit loops");
    // the tile reordered by digit (keys, then values)
    __shared__ uint64_t stage[TILE];
    __shared__ uint16_t whist[W][RADIX];
    __shared__ uint32_t nhist[RADIX];
    __shared__ uint32_t ddelta[RADIX];
    __shared__ uint64_t scan_tmp[W];
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = tile_of_block(blockIdx.x, gridDim.x);
    if (lb_clear && tid < RADIX) lb_clear[static_cast<size_t>(tile) * RADIX + tid] = 0;  // rows of the next pass
    for (int i = tid; i < W * RADIX; i += BLOCK) (&whist[0][0])[i] = 0;
    if (tid < RADIX) nhist[tid] = 0;
    const uint32_t base = tile * static_cast<uint32_t>(TILE);
    const TileDesc td{tile, base, min(n - base, static_cast<uint32_t>(TILE)), 0u, 0u};
    if (td.count == static_cast<uint32_t>(TILE))
        onesweep_tile<BITS, BLOCK, ITEMS, WIN, FIRST, WITH_VALUES, LB, true>(
            td, keys_in, vals_in, keys_out, vals_out, n, shift, ghist, ghist_next, shift_next, lb, epoch, err, stage,
            whist, nhist, ddelta, scan_tmp, nullptr);
    else
        onesweep_tile<BITS, BLOCK, ITEMS, WIN, FIRST, WITH_VALUES, LB, false>(
            td, keys_in, vals_in, keys_out, vals_out, n, shift, ghist, ghist_next, shift_next, lb, epoch, err, stage,
            whist, nhist, ddelta, scan_tmp, nullptr);
}

// Segmented pass: many independent key sets in one launch. Block b sorts
// tile tiles[b] = {first key, key count, first tile of its set, set}; every
// set has its own digit histograms (ghist + set * hist_stride) and its own
// look-back chain, and its permutation values count from the set's start.
template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool WITH_VALUES, class LB>
__global__ __launch_bounds__(BLOCK, (kMinBlocks<BLOCK, ITEMS>)) void onesweep_seg_kernel(const uint64_t* __restrict__ keys_in,
                                                              const uint32_t* __restrict__ vals_in,
                                                              uint64_t* __restrict__ keys_out,
                                                              uint32_t* __restrict__ vals_out, uint32_t n,
                                                              uint32_t shift, const uint32_t* __restrict__ ghist,
                                                              uint32_t* __restrict__ ghist_next, uint32_t shift_next,
                                                              uint32_t hist_stride, const uint4* __restrict__ tiles,
                                                              const uint32_t* __restrict__ seg_base,
                                                              typename LB::word* lb, typename LB::word* lb_clear,
                                                              uint32_t epoch, uint32_t* err,
                                                              const uint32_t* __restrict__ live_tiles) {
    constexpr int RADIX = 1 << BITS;
    constexpr int W = BLOCK / kWave;
    constexpr int TILE = BLOCK * ITEMS;
    static_assert(BLOCK >= RADIX, "one digit per thread in the digit loops");
    __shared__ uint64_t stage[TILE];
    __shared__ uint16_t whist[W][RADIX];
    __shared__ uint32_t nhist[RADIX];
    __shared__ uint32_t ddelta[RADIX];
    __shared__ uint64_t scan_tmp[W];
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = tile_of_block(blockIdx.x, gridDim.x);
    // a tile table written on the device: blocks past its length have nothing to do
    if (live_tiles && tile >= *live_tiles) return;
    const uint4 t = tiles[tile];
    if (live_tiles && (t.y == 0 || t.y > static_cast<uint32_t>(TILE) || t.x > n - t.y)) return;
    if (lb_clear && tid < RADIX) lb_clear[static_cast<size_t>(tile) * RADIX + tid] = 0;
    for (int i = tid; i < W * RADIX; i += BLOCK) (&whist[0][0])[i] = 0;
    if (tid < RADIX) nhist[tid] = 0;
    const TileDesc td{tile, t.x, t.y, t.z, seg_base[t.w]};
    const uint32_t* gh = ghist + static_cast<size_t>(t.w) * hist_stride;
    uint32_t* gn = ghist_next ? ghist_next + static_cast<size_t>(t.w) * hist_stride : nullptr;
    if (td.count == static_cast<uint32_t>(TILE))
        onesweep_tile<BITS, BLOCK, ITEMS, WIN, FIRST, WITH_VALUES, LB, true>(
            td, keys_in, vals_in, keys_out, vals_out, n, shift, gh, gn, shift_next, lb, epoch, err, stage, whist,
            nhist, ddelta, scan_tmp, tiles);
    else
        onesweep_tile<BITS, BLOCK, ITEMS, WIN, FIRST, WITH_VALUES, LB, false>(
            td, keys_in, vals_in, keys_out, vals_out, n, shift, gh, gn, shift_next, lb, epoch, err, stage, whist,
            nhist, ddelta, scan_tmp, tiles);
}

// Pass over a tile table written on the device whose length is known only
// there (*live_tiles): a small grid of blocks takes tiles in order from
// *counter until none are left, so a tile's predecessors are always taken by
// running blocks (look-back progress); blocks beyond the table's length leave
// at once, so an empty table costs no atomics. Tiles carry {first key, key count, first tile of the segment,
// segment}, as in the segmented pass.
template <int BITS, int BLOCK, int ITEMS, int WIN, class LB>
__global__ __launch_bounds__(BLOCK, (kMinBlocks<BLOCK, ITEMS>)) void onesweep_list_kernel(
    const uint64_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in, uint64_t* __restrict__ keys_out,
    uint32_t* __restrict__ vals_out, uint32_t n, uint32_t shift, const uint32_t* __restrict__ ghist,
    uint32_t* __restrict__ ghist_next, uint32_t shift_next, uint32_t hist_stride, const uint4* __restrict__ tiles,
    const uint32_t* __restrict__ seg_base, typename LB::word* lb, typename LB::word* lb_clear, uint32_t epoch,
    uint32_t* err, const uint32_t* __restrict__ live_tiles, uint32_t* counter) {
    constexpr int RADIX = 1 << BITS;
    constexpr int W = BLOCK / kWave;
    constexpr int TILE = BLOCK * ITEMS;
    __shared__ uint64_t stage[TILE];
    __shared__ uint16_t whist[W][RADIX];
    __shared__ uint32_t nhist[RADIX];
    __shared__ uint32_t ddelta[RADIX];
    __shared__ uint64_t scan_tmp[W];
    __shared__ uint32_t slot;
    const uint32_t tid = threadIdx.x;
    const uint32_t live = *live_tiles;
    if (blockIdx.x >= live) return;  // more blocks than tiles: the rest stay off the counter
    for (;;) {
        if (tid == 0) slot = atomicAdd(counter, 1u);
        __syncthreads();
        const uint32_t tile = slot;
        if (tile >= live) break;
        const uint4 t = tiles[tile];
        if (t.y == 0 || t.y > static_cast<uint32_t>(TILE) || t.x > n - t.y) {  // never: the table is sized
            if (tid == 0) atomicOr(err, kErrSpin);
            break;
        }
        if (lb_clear && tid < RADIX) lb_clear[static_cast<size_t>(tile) * RADIX + tid] = 0;
        for (int i = tid; i < W * RADIX; i += BLOCK) (&whist[0][0])[i] = 0;
        if (tid < RADIX) nhist[tid] = 0;
        const TileDesc td{tile, t.x, t.y, t.z, seg_base[t.w]};
        const uint32_t* gh = ghist + static_cast<size_t>(t.w) * hist_stride;
        uint32_t* gn = ghist_next ? ghist_next + static_cast<size_t>(t.w) * hist_stride : nullptr;
        if (td.count == static_cast<uint32_t>(TILE))
            onesweep_tile<BITS, BLOCK, ITEMS, WIN, false, true, LB, true>(
                td, keys_in, vals_in, keys_out, vals_out, n, shift, gh, gn, shift_next, lb, epoch, err, stage, whist,
                nhist, ddelta, scan_tmp, tiles);
        else
            onesweep_tile<BITS, BLOCK, ITEMS, WIN, false, true, LB, false>(
                td, keys_in, vals_in, keys_out, vals_out, n, shift, gh, gn, shift_next, lb, epoch, err, stage, whist,
                nhist, ddelta, scan_tmp, tiles);
        __syncthreads();  // shared state and the slot are reused by the next tile
    }
}

// ---- prefix split: the top two digits, then every bucket on its own ---------
//
// For particle keys the three most significant digits (27 bits: the level-9
// octant of a key) are sorted first, by onesweep passes. The keys then
// form runs of one prefix ("buckets"), each still in input order. A block
// owns the buckets that start in its chunk of kLocalChunk keys and sorts each
// segment of at most kLocalCap keys in LDS, by an LSD sort over only the bits
// in which the segment's keys differ (stable, so input order is kept among
// equal keys). A bucket longer than kLocalCap is listed instead; the listed
// buckets are sorted on their low bits by segmented onesweep passes whose tile
// table the listing blocks write.

constexpr int kLocalBlock = 512;
constexpr int kLocalItems = 4;
constexpr int kLocalBlocksPerCU = 4;                        // LDS of a block stays below 40 KB
constexpr uint32_t kLocalCap = kLocalBlock * kLocalItems;  // keys one block holds and sorts in LDS
constexpr uint32_t kLocalLook = 64;                         // look-ahead past the chunk for its last bucket's end
constexpr uint32_t kLocalChunk = kLocalCap - kLocalLook;    // a block owns the buckets starting in its chunk
constexpr uint32_t kErrLarge = 1u << 9;                     // bucket list overflow (not reachable by the sizing)
constexpr uint32_t kCountMax = 160;  // buckets up to this size are ranked by counting, larger ones by LDS passes

struct LargeList {
    uint32_t* count;  // [0] buckets listed, [1] tiles listed
    uint4* tiles;     // {first key, key count, first tile of the bucket, bucket}
    uint32_t* start;  // first key of each bucket
    uint32_t* hist;   // per bucket: digit counts of every low pass (stride words)
    void* lb;         // look-back rows of the first low pass (32- or 64-bit words)
    uint32_t stride, row_words, tile, max_buckets, max_tiles, wide;
};

template <int BITS, int BLOCK, int ITEMS>
struct LocalSmem {
    uint64_t keys[BLOCK * ITEMS];
    uint32_t vals[BLOCK * ITEMS];
    uint16_t whist[BLOCK / kWave][1 << BITS];
    uint16_t starts[BLOCK * ITEMS + 1];  // bucket starts of a segment (window positions), then its end
    uint32_t cnt[ITEMS * (BLOCK / kWave)];
    uint32_t scan[BLOCK / kWave];
    uint64_t bits[BLOCK / kWave];
    uint32_t setbits[BLOCK * ITEMS / 32];  // segmented sorts: window positions where a key set starts
    uint32_t first, last, end, run_end, slot, tile0, nb, maxb, next_set;
};

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v = min(v, static_cast<uint32_t>(__shfl_xor(v, d, kWave)));
    return v;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t v) {
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) v = max(v, static_cast<uint32_t>(__shfl_xor(v, d, kWave)));
    return v;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t v) {
    uint32_t lo = static_cast<uint32_t>(v), hi = static_cast<uint32_t>(v >> 32);
#pragma unroll
    for (int d = kWave / 2; d >= 1; d >>= 1) {
        lo |= __shfl_xor(lo, d, kWave);
        hi |= __shfl_xor(hi, d, kWave);
    }
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// First index >= from whose key is >= bound, for keys ordered by prefix and a
// bound whose bits below the prefix are zero (so "key < bound" holds on a
// leading run). One wave: lane l probes from + 2^l - 1, then the bracket the
// probes leave is searched 64 ways per step. All lanes must call it.
__device__ __forceinline__ uint32_t run_end(const uint64_t* a, uint32_t n, uint32_t from, uint64_t bound) {
    const uint32_t lane = lane_id();
    const uint64_t probe = static_cast<uint64_t>(from) + ((1ull << (lane & 31u)) - 1u);
    const bool beyond = lane >= 32u || probe >= n || a[probe] >= bound;
    const uint32_t f = static_cast<uint32_t>(__builtin_ctzll(__ballot(beyond)));  // lanes >= 32 are set
    const uint64_t lo = f ? static_cast<uint64_t>(from) + (1ull << (f - 1)) : from;  // probe f-1 lies in the run
    const uint64_t pf = static_cast<uint64_t>(from) + ((1ull << f) - 1u);
    const uint64_t hi = f < 32u && pf < n ? pf : n;  // probe f (or the end) is past it
    return wave_lower_bound(a, static_cast<uint32_t>(lo), static_cast<uint32_t>(hi), bound);
}

// Smallest window position in [j, e) where a key set starts, else e (the
// same value in every lane).
__device__ __forceinline__ uint32_t next_set_start(const uint32_t* setbits, uint32_t j, uint32_t e) {
    while (j < e) {
        const uint32_t w = setbits[j >> 5] >> (j & 31u);
        if (w) return min(j + static_cast<uint32_t>(__builtin_ctz(w)), e);
        j = (j | 31u) + 1u;
    }
    return e;
}

// Sort keys [a, a + m) with their values (1 <= m <= BLOCK * ITEMS) into the
// same places of kout / vout, reading them from the block's window in LDS
// (at window offset a - wlo) if `in_lds`, else from kin / vin. Keys sit in a
// wave-blocked layout, so the ballot ranks follow input order and every pass
// is stable.
template <int BITS, int BLOCK, int ITEMS>
__device__ __forceinline__ void lds_sort_segment(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                 uint32_t* vout,
                                                 uint32_t a, uint32_t m, bool in_lds, uint32_t wlo,
                                                 LocalSmem<BITS, BLOCK, ITEMS>& sm) {
    constexpr int RADIX = 1 << BITS;
    constexpr int W = BLOCK / kWave;
    static_assert(BLOCK >= RADIX, "one digit per thread in the digit loops");
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const uint32_t wbase = wave * ITEMS * kWave;
    const uint32_t off = a - wlo;
    const uint64_t k0 = in_lds ? sm.keys[off] : kin[a];
    uint64_t k[ITEMS];
    uint32_t v[ITEMS];
    uint64_t diff = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = wbase + i * kWave + lane;
        const bool ok = p < m;
        if (in_lds) {
            k[i] = ok ? sm.keys[off + p] : k0;
            v[i] = ok ? sm.vals[off + p] : 0u;
        } else {
            k[i] = ok ? kin[a + p] : k0;
            v[i] = ok ? vin[a + p] : 0u;
        }
        diff |= k[i] ^ k0;
    }
    // only the bits in which the segment's keys differ need sorting
    diff = wave_or64(diff);
    if (lane == 0) sm.bits[wave] = diff;
    __syncthreads();
    uint64_t all = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) all |= sm.bits[w];
    const int passes = (64 - clz64(all) + BITS - 1) / BITS;
    for (int pass = 0; pass < passes; ++pass) {
        const uint32_t shift = static_cast<uint32_t>(pass * BITS);
        for (int i = tid; i < W * RADIX; i += BLOCK) (&sm.whist[0][0])[i] = 0;
        __syncthreads();
        uint32_t rank[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const bool ok = wbase + i * kWave + lane < m;
            const uint32_t d = digit_of<BITS>(k[i], shift);
            const uint64_t peers = match_digit<BITS>(d, __ballot(ok));
            const uint32_t below = lanes_below(peers);
            const uint32_t base = sm.whist[wave][d];
            if (ok && below == 0) sm.whist[wave][d] = static_cast<uint16_t>(base + static_cast<uint32_t>(__popcll(peers)));
            rank[i] = base + below;
        }
        __syncthreads();
        uint32_t total = 0;
        if (tid < RADIX) {
#pragma unroll
            for (int w = 0; w < W; ++w) {
                const uint32_t c = sm.whist[w][tid];
                sm.whist[w][tid] = static_cast<uint16_t>(total);
                total += c;
            }
        }
        uint32_t sum;
        const uint32_t start = block_exclusive_sum<uint32_t, BLOCK>(total, sm.scan, &sum);
        if (tid < RADIX) {
#pragma unroll
            for (int w = 0; w < W; ++w) sm.whist[w][tid] += static_cast<uint16_t>(start);
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            if (wbase + i * kWave + lane < m) {
                const uint32_t dst = sm.whist[wave][digit_of<BITS>(k[i], shift)] + rank[i];
                sm.keys[dst] = k[i];
                sm.vals[dst] = v[i];
            }
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t p = wbase + i * kWave + lane;
            if (p < m) {
                k[i] = sm.keys[p];
                v[i] = sm.vals[p];
            }
        }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t p = wbase + i * kWave + lane;
        if (p < m) {
            kout[a + p] = k[i];
            vout[a + p] = v[i];
        }
    }
    __syncthreads();  // the shared arrays may be reused for another segment
}

// Sort the buckets at window positions [f, e) (f and e bucket starts, or e the
// window's end at the end of the keys) into kout / vout; the window's keys and
// values are in LDS. If no bucket is longer than kCountMax, every key is ranked
// inside its bucket by counting the keys that precede it (smaller, or equal and
// earlier); otherwise the segment goes through the LDS passes. With SEG, a
// key set's first key also starts a bucket, and the LDS passes take each
// set's part of the segment on its own.
template <int BITS, int BLOCK, int ITEMS, bool SEG>
__device__ __forceinline__ void lds_sort_window(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                uint32_t* vout,
                                                uint32_t n, uint32_t lo, uint32_t f, uint32_t e, uint32_t pshift,
                                                LocalSmem<BITS, BLOCK, ITEMS>& sm) {
    constexpr int W = BLOCK / kWave;
    static_assert(ITEMS * W <= kWave, "one wave scans the per-(item, wave) start counts");
    const uint32_t tid = threadIdx.x, lane = lane_id(), wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    if (tid == 0) sm.maxb = 0;
    uint64_t k[ITEMS];
    uint64_t smask[ITEMS];
    uint32_t start_bits = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
        const bool in = j >= f && j < e;
        k[i] = in ? sm.keys[j] : 0ull;
        bool st = in && (j == f || (sm.keys[j - 1] >> pshift) != (k[i] >> pshift));
        if constexpr (SEG) st = st || (in && ((sm.setbits[j >> 5] >> (j & 31u)) & 1u));
        smask[i] = __ballot(st);
        start_bits |= static_cast<uint32_t>(st) << i;
        if (lane == 0) sm.cnt[i * W + wave] = static_cast<uint32_t>(__popcll(smask[i]));
    }
    __syncthreads();
    if (wave == 0) {  // (item, wave) pieces in window order: exclusive counts of starts before each
        const uint32_t c = lane < ITEMS * W ? sm.cnt[lane] : 0u;
        const uint32_t inc = wave_inclusive_sum(c);
        if (lane < ITEMS * W) sm.cnt[lane] = inc - c;
        if (lane == kWave - 1) sm.nb = inc;
    }
    __syncthreads();
    uint32_t id[ITEMS];  // bucket of each key: starts at or before it, minus one
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
        const uint32_t base = sm.cnt[i * W + wave];
        const uint32_t below = lanes_below(smask[i]);
        id[i] = base + below + ((start_bits >> i) & 1u) - 1u;
        if ((start_bits >> i) & 1u) sm.starts[base + below] = static_cast<uint16_t>(j);
    }
    if (tid == 0) sm.starts[sm.nb] = static_cast<uint16_t>(e);
    __syncthreads();
    uint32_t longest = 0;
#pragma unroll
    for (int i = 0; i < ITEMS; ++i)
        if ((start_bits >> i) & 1u) {
            const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
            longest = max(longest, static_cast<uint32_t>(sm.starts[id[i] + 1]) - j);
        }
    longest = wave_max_u32(longest);
    if (lane == 0) atomicMax(&sm.maxb, longest);
    __syncthreads();
    if (sm.maxb > kCountMax) {
        if constexpr (SEG) {
            // one set's keys at a time; the first part is read from the window,
            // the rest from memory (the LDS passes overwrite the window, and
            // the parts this block wrote lie before the part being read)
            uint32_t a = f;
            bool in_lds = true;
            while (a < e) {
                const uint32_t b = next_set_start(sm.setbits, a + 1u, e);
                lds_sort_segment<BITS, BLOCK, ITEMS>(kin, vin, kout, vout, lo + a, b - a, in_lds, lo, sm);
                in_lds = false;
                a = b;
            }
        } else {
            lds_sort_segment<BITS, BLOCK, ITEMS>(kin, vin, kout, vout, lo + f, e - f, true, lo, sm);
        }
        return;
    }
    // rank every key in its bucket; only keys whose place changes are written
    // (a bucket's moved keys fill exactly each other's places)
    uint32_t dst[ITEMS];
    uint32_t v[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
        dst[i] = lo + j;
        if (j >= f && j < e) {
            const uint32_t bs = sm.starts[id[i]], be = sm.starts[id[i] + 1];
            const uint64_t kp = k[i];
            uint32_t rank = 0;
            for (uint32_t q = bs; q < be; ++q) {
                const uint64_t kq = sm.keys[q];
                rank += (kq < kp || (kq == kp && q < j)) ? 1u : 0u;
            }
            dst[i] = lo + bs + rank;
            if (dst[i] != lo + j) v[i] = sm.vals[j];
        }
    }
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
        if (j >= f && j < e && dst[i] != lo + j && dst[i] < n) {  // dst < n always; guards memory
            kout[dst[i]] = k[i];
            vout[dst[i]] = v[i];
        }
    }
    __syncthreads();  // the shared arrays may be reused
}

// List bucket [start, start + len) for the low passes: reserve its slot and a
// run of tiles, write the tiles, and clear its digit counts and the look-back
// rows its first low pass will use.
template <int BITS, int BLOCK, int ITEMS>
__device__ __forceinline__ void list_large(const LargeList& L, uint32_t start, uint32_t len, uint32_t* err,
                           LocalSmem<BITS, BLOCK, ITEMS>& sm) {
    const uint32_t tid = threadIdx.x;
    const uint32_t tiles = (len + L.tile - 1) / L.tile;
    if (tid == 0) {
        uint32_t b = atomicAdd(&L.count[0], 1u);
        const uint32_t t0 = atomicAdd(&L.count[1], tiles);
        if (b >= L.max_buckets || t0 > L.max_tiles - tiles) {
            atomicOr(err, kErrLarge);
            b = 0xffffffffu;
        }
        sm.slot = b;
        sm.tile0 = t0;
    }
    __syncthreads();
    const uint32_t b = sm.slot, t0 = sm.tile0;
    if (b == 0xffffffffu) return;
    if (tid == 0) L.start[b] = start;
    for (uint32_t t = tid; t < tiles; t += BLOCK)
        L.tiles[t0 + t] = make_uint4(start + t * L.tile, min(L.tile, len - t * L.tile), t0, b);
    uint32_t* h = L.hist + static_cast<size_t>(b) * L.stride;
    for (uint32_t i = tid; i < L.stride; i += BLOCK) h[i] = 0;
    const size_t w0 = static_cast<size_t>(t0) * L.row_words, w1 = static_cast<size_t>(t0 + tiles) * L.row_words;
    if (L.wide) {
        for (size_t i = w0 + tid; i < w1; i += BLOCK) static_cast<uint64_t*>(L.lb)[i] = 0;
    } else {
        for (size_t i = w0 + tid; i < w1; i += BLOCK) static_cast<uint32_t*>(L.lb)[i] = 0;
    }
}

// Block b: the buckets (runs of equal key >> pshift) that start in keys
// [b * chunk, (b + 1) * chunk), read from kin / vin, sorted into kout / vout.
// The block reads its chunk and the look-ahead after it (keys and values) into
// LDS at once; only a last bucket that runs past the look-ahead is searched for
// and read again.
//
// The sort is in place. A block writes only the buckets it owns; what it
// reads of other blocks' buckets (the look-ahead, the key before its chunk,
// the run-end search) it uses only for prefixes, which sorting inside a bucket
// leaves unchanged at every position.
//
// level6 (NULL, or kLevel6Cells words set to kCellEmpty): the first position
// of every non-empty level-6 node (key >> 45), found with the bucket starts.
//
// SEG: the keys are n_sets key sets back to back, set s starting at
// seg_base[s] (non-decreasing), each ordered by prefix on its own; every set's
// first key starts a bucket and no bucket runs past its set. chunk_set[b] is
// the first set starting at or after block b's first key, chunk_set[chunks +
// 1 + b] where that set starts (n if none).
template <int BITS, int BLOCK, int ITEMS, bool SEG>
__global__ __launch_bounds__(BLOCK, kLocalBlocksPerCU * BLOCK / (4 * kWave)) void local_sort_kernel(
    uint64_t* keys, uint32_t* vals, uint32_t n, uint32_t pshift, LargeList large, uint32_t* err, uint32_t* level6,
    const uint32_t* seg_base, uint32_t n_sets, const uint32_t* chunk_set) {
    const uint64_t* kin = keys;
    const uint32_t* vin = vals;
    uint64_t* kout = keys;
    uint32_t* vout = vals;
    constexpr uint32_t CAP = BLOCK * ITEMS, CHUNK = kLocalChunk;
    static_assert(CHUNK < CAP, "the window holds the chunk and a look-ahead");
    __shared__ LocalSmem<BITS, BLOCK, ITEMS> sm;
    const uint32_t tid = threadIdx.x;
    const uint32_t lo = blockIdx.x * CHUNK;
    const uint32_t hi = static_cast<uint32_t>(min(static_cast<uint64_t>(n), static_cast<uint64_t>(lo) + CHUNK));
    const uint32_t wend = static_cast<uint32_t>(min(static_cast<uint64_t>(n), static_cast<uint64_t>(lo) + CAP));
    const uint32_t wn = wend - lo, own = hi - lo;
    if (tid == 0) {
        sm.first = 0xffffffffu;
        sm.last = 0u;
        sm.end = 0xffffffffu;
        sm.next_set = n_sets;
    }
    // the chunk's first set and where it starts, read before the window so
    // that the round trip overlaps its load
    uint32_t s0 = 0, first_at = 0;
    if constexpr (SEG) {
        for (uint32_t i = tid; i < CAP / 32; i += BLOCK) sm.setbits[i] = 0;
        s0 = chunk_set[blockIdx.x];
        first_at = chunk_set[gridDim.x + 1 + blockIdx.x];
    }
    // every load of the window in flight at once (a load under a per-item
    // branch would wait before the next one is issued)
    if (wn == CAP) {  // block-uniform: a whole window, one base pointer and constant offsets
        const uint64_t* kb = kin + (lo + tid);
        const uint32_t* vb = vin + (lo + tid);
        uint64_t wk[ITEMS];
        uint32_t wv[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            wk[i] = kb[i * BLOCK];
            wv[i] = vb[i * BLOCK];
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            sm.keys[i * BLOCK + tid] = wk[i];
            sm.vals[i * BLOCK + tid] = wv[i];
        }
    } else {  // the last windows: a position past the window reads its last entry (wn >= 1), not stored
        uint64_t wk[ITEMS];
        uint32_t wv[ITEMS];
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = min(static_cast<uint32_t>(i) * BLOCK + tid, wn - 1u);
            wk[i] = kin[lo + j];
            wv[i] = vin[lo + j];
        }
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
            if (j < wn) {
                sm.keys[j] = wk[i];
                sm.vals[j] = wv[i];
            }
        }
    }
    const uint64_t before = lo ? kin[lo - 1] >> pshift : ~0ull;  // the same word in every lane
    if constexpr (SEG) {
        // mark the set starts in the window (none in most windows); the first
        // set starting at or after the window's end gives the end of a last
        // bucket that runs past it
        if (first_at < wend) {  // block-uniform
            __syncthreads();
            for (uint32_t q = s0 + tid; q < n_sets; q += BLOCK) {
                const uint32_t at = seg_base[q];
                if (at >= wend) {
                    atomicMin(&sm.next_set, q);
                    break;
                }
                if (at >= lo) atomicOr(&sm.setbits[(at - lo) >> 5], 1u << ((at - lo) & 31u));
            }
        }
    }
    __syncthreads();
    // bucket starts: the first and last in the chunk, the first after it; the
    // wave's are read off ballots (item i of lane l sits at i * BLOCK + the
    // wave's first thread + l, so the lowest and highest set lane give them)
    uint32_t first = 0xffffffffu, last = 0u, after = 0xffffffffu;  // wave-uniform
    const uint32_t wave0 = tid - lane_id();
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t j = static_cast<uint32_t>(i) * BLOCK + tid;
        bool st = false;
        if (j < wn) {
            const uint64_t pj = sm.keys[j] >> pshift;
            const uint64_t pp = j ? sm.keys[j - 1] >> pshift : before;
            st = pj != pp;
            if constexpr (SEG) st = st || ((sm.setbits[j >> 5] >> (j & 31u)) & 1u);
            // a level-6 node starts here too if the key's top 18 bits changed
            const uint32_t up = 45u - pshift;
            if (st && j < own && level6 && (pj >> up) != (pp >> up)) level6[pj >> up] = lo + j;
        }
        const uint64_t in_chunk = __ballot(st && j < own), past = __ballot(st && j >= own);
        const uint32_t base = static_cast<uint32_t>(i) * BLOCK + wave0;
        if (in_chunk) {
            first = min(first, base + static_cast<uint32_t>(__builtin_ctzll(in_chunk)));
            last = max(last, base + 63u - static_cast<uint32_t>(__builtin_clzll(in_chunk)));
        }
        if (past) after = min(after, base + static_cast<uint32_t>(__builtin_ctzll(past)));
    }
    if (lane_id() == 0) {
        if (first != 0xffffffffu) {
            atomicMin(&sm.first, first);
            atomicMax(&sm.last, last);
        }
        if (after != 0xffffffffu) atomicMin(&sm.end, after);
    }
    __syncthreads();
    const uint32_t f = sm.first, l = sm.last;
    if (f == 0xffffffffu) return;  // no bucket starts here
    const uint64_t last_prefix = sm.keys[l] >> pshift;
    // where the last bucket's keys end at the latest: the keys' end, or the
    // next set's start
    uint32_t bound_end = n;
    if constexpr (SEG)
        bound_end = first_at >= wend ? first_at : (sm.next_set < n_sets ? seg_base[sm.next_set] : n);
    uint32_t e = sm.end;
    if (e == 0xffffffffu && wend == bound_end) e = wn;  // the last bucket ends with the window
    if (e != 0xffffffffu) {
        lds_sort_window<BITS, BLOCK, ITEMS, SEG>(kin, vin, kout, vout, n, lo, f, e, pshift, sm);
        return;
    }
    // the last bucket runs past the window: the buckets before it from LDS, then it alone
    if (l > f) lds_sort_window<BITS, BLOCK, ITEMS, SEG>(kin, vin, kout, vout, n, lo, f, l, pshift, sm);
    // (its own slot: with l == f no barrier separates this from the reads of sm.end above)
    if (tid < kWave) {
        const uint32_t ee = run_end(kin, bound_end, wend, (last_prefix + 1u) << pshift);
        if (tid == 0) sm.run_end = ee;
    }
    __syncthreads();
    const uint32_t start = lo + l, len = sm.run_end - start;
    if (len <= CAP)
        lds_sort_segment<BITS, BLOCK, ITEMS>(kin, vin, kout, vout, start, len, false, lo, sm);
    else
        list_large<BITS, BLOCK, ITEMS>(large, start, len, err, sm);
}

// Counts of the lowest digit in every listed tile, into its bucket's row.
__global__ __launch_bounds__(512) void large_hist_kernel(const uint64_t* __restrict__ keys, uint32_t n,
                                                         LargeList L, uint32_t mask) {
    __shared__ uint32_t h[kMaxRadix];
    const uint32_t live = L.count[1];
    for (uint32_t tile = blockIdx.x; tile < live; tile += gridDim.x) {
        const uint4 t = L.tiles[tile];
        if (t.y == 0 || t.y > L.tile || t.x > n - t.y || t.w >= L.max_buckets) continue;  // never: the table is sized
        for (uint32_t i = threadIdx.x; i <= mask; i += 512) h[i] = 0;
        __syncthreads();
        for (uint32_t j = t.x + threadIdx.x; j < t.x + t.y; j += 512)
            atomicAdd(&h[static_cast<uint32_t>(keys[j]) & mask], 1u);
        __syncthreads();
        uint32_t* g = L.hist + static_cast<size_t>(t.w) * L.stride;
        for (uint32_t i = threadIdx.x; i <= mask; i += 512)
            if (h[i]) atomicAdd(&g[i], h[i]);
        __syncthreads();
    }
}

// ---- variants ------------------------------------------------------------------

struct PassArgs {
    const uint64_t* keys_in;
    const uint32_t* vals_in;
    uint64_t* keys_out;
    uint32_t* vals_out;
    uint32_t n, shift;
    const uint32_t* ghist;
    uint32_t* ghist_next;
    uint32_t shift_next;
    void* lb;        // look-back rows of this pass
    void* lb_clear;  // 32-bit words: rows the next pass will use, cleared here
    uint32_t epoch;
    uint32_t* err;
    bool wide;  // 64-bit look-back words (n >= 2^30)
};

template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool VALS>
void launch_one(const PassArgs& a, hipStream_t stream) {
    constexpr uint32_t tile = BLOCK * ITEMS;
    const dim3 grid((a.n + tile - 1) / tile), block(BLOCK);
    if (a.wide)
        hipLaunchKernelGGL((onesweep_kernel<BITS, BLOCK, ITEMS, WIN, FIRST, VALS, Lb64>), grid, block, 0, stream,
                           a.keys_in, a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next,
                           a.shift_next, static_cast<uint64_t*>(a.lb), nullptr, a.epoch, a.err);
    else
        hipLaunchKernelGGL((onesweep_kernel<BITS, BLOCK, ITEMS, WIN, FIRST, VALS, Lb32>), grid, block, 0, stream,
                           a.keys_in, a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next,
                           a.shift_next, static_cast<uint32_t*>(a.lb), static_cast<uint32_t*>(a.lb_clear), a.epoch,
                           a.err);
}

template <int BITS, int BLOCK, int ITEMS, int WIN>
void launch_pass_t(const PassArgs& a, bool first, bool with_values, hipStream_t stream) {
    if (with_values && first)
        launch_one<BITS, BLOCK, ITEMS, WIN, true, true>(a, stream);
    else if (with_values)
        launch_one<BITS, BLOCK, ITEMS, WIN, false, true>(a, stream);
    else
        launch_one<BITS, BLOCK, ITEMS, WIN, false, false>(a, stream);
}

struct SegArgs {
    const uint4* tiles;
    const uint32_t* seg_base;
    uint32_t n_tiles;  // blocks launched
    uint32_t hist_stride;
    const uint32_t* live_tiles;  // NULL, or the device word holding how many tiles are in use
};

template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool VALS>
void launch_one_seg(const PassArgs& a, const SegArgs& g, hipStream_t stream) {
    const dim3 grid(g.n_tiles), block(BLOCK);
    if (a.wide)
        hipLaunchKernelGGL((onesweep_seg_kernel<BITS, BLOCK, ITEMS, WIN, FIRST, VALS, Lb64>), grid, block, 0, stream,
                           a.keys_in, a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next,
                           a.shift_next, g.hist_stride, g.tiles, g.seg_base, static_cast<uint64_t*>(a.lb), nullptr,
                           a.epoch, a.err, g.live_tiles);
    else
        hipLaunchKernelGGL((onesweep_seg_kernel<BITS, BLOCK, ITEMS, WIN, FIRST, VALS, Lb32>), grid, block, 0, stream,
                           a.keys_in, a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next,
                           a.shift_next, g.hist_stride, g.tiles, g.seg_base, static_cast<uint32_t*>(a.lb),
                           static_cast<uint32_t*>(a.lb_clear), a.epoch, a.err, g.live_tiles);
}

template <int BITS, int BLOCK, int ITEMS, int WIN>
void launch_seg_t(const PassArgs& a, const SegArgs& g, bool first, bool with_values, hipStream_t stream) {
    if (with_values && first)
        launch_one_seg<BITS, BLOCK, ITEMS, WIN, true, true>(a, g, stream);
    else if (with_values)
        launch_one_seg<BITS, BLOCK, ITEMS, WIN, false, true>(a, g, stream);
    else
        launch_one_seg<BITS, BLOCK, ITEMS, WIN, false, false>(a, g, stream);
}

constexpr uint32_t kListGrid = 512;  // blocks of a pass over a device-written tile table

template <int BITS, int BLOCK, int ITEMS, int WIN>
void launch_list_t(const PassArgs& a, const SegArgs& g, uint32_t* counter, hipStream_t stream) {
    const dim3 grid(std::min(g.n_tiles, kListGrid)), block(BLOCK);
    if (a.wide)
        hipLaunchKernelGGL((onesweep_list_kernel<BITS, BLOCK, ITEMS, WIN, Lb64>), grid, block, 0, stream, a.keys_in,
                           a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next, a.shift_next,
                           g.hist_stride, g.tiles, g.seg_base, static_cast<uint64_t*>(a.lb), nullptr, a.epoch, a.err,
                           g.live_tiles, counter);
    else
        hipLaunchKernelGGL((onesweep_list_kernel<BITS, BLOCK, ITEMS, WIN, Lb32>), grid, block, 0, stream, a.keys_in,
                           a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next, a.shift_next,
                           g.hist_stride, g.tiles, g.seg_base, static_cast<uint32_t*>(a.lb),
                           static_cast<uint32_t*>(a.lb_clear), a.epoch, a.err, g.live_tiles, counter);
}

struct Variant {
    int bits, block, items, window;
    bool split;  // particle keys take the split sort (9-bit digits only), else plain LSD passes
    void (*launch)(const PassArgs&, bool, bool, hipStream_t);
    void (*launch_seg)(const PassArgs&, const SegArgs&, bool, bool, hipStream_t);
    void (*launch_list)(const PassArgs&, const SegArgs&, uint32_t*, hipStream_t);
};

#define CS_VARIANT(B, BL, IT, WI, SP) \
    {B, BL, IT, WI, SP, launch_pass_t<B, BL, IT, WI>, launch_seg_t<B, BL, IT, WI>, launch_list_t<B, BL, IT, WI>}
// Shapes: digit bits, block, keys per thread, look-back window, split sort
// for particle keys. A block needs at least one thread per digit, so
// 256-thread blocks take 8-bit digits; 1024-thread blocks hold one block per
// CU. The 9-bit shapes without the split run 7 plain LSD passes, which a
// strongly clustered set (many level-9 buckets over the bucket kernel's
// sizes) can favour.
const Variant kVariants[] = {
    CS_VARIANT(9, 512, 16, 4, true),  CS_VARIANT(8, 512, 16, 4, false), CS_VARIANT(9, 512, 12, 4, true),
    CS_VARIANT(9, 512, 32, 4, true),  CS_VARIANT(9, 1024, 8, 4, true),  CS_VARIANT(9, 1024, 16, 4, true),
    CS_VARIANT(8, 256, 16, 4, false), CS_VARIANT(9, 512, 16, 4, false), CS_VARIANT(9, 512, 12, 4, false),
};
#undef CS_VARIANT
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

// Shape used where the autotune table has no entry: 9-bit digits, 512 x 16
// tiles, the split sort.
constexpr int kBuiltinVariant = 0;

// Split sorts of particle keys: 9-bit digits, the top three first (the
// level-9 octant), then four low passes for the listed buckets
// (63 = 3 * 9 + 36 bits). The top passes end in the output arrays, where the
// buckets are sorted in place and the low passes end too.
constexpr int kSplitBits = 9;
constexpr int kSplitTop = 3;
constexpr int kLowPasses = 4;
constexpr uint32_t kSplitShift = 63 - kSplitTop * kSplitBits;  // the prefix is key >> 36
static_assert(kSplitTop % 2 == 1 && kLowPasses % 2 == 0, "top passes and low passes end in the output arrays");
constexpr int kGhistWords = kMaxPasses * kMaxRadix + 64;      // digit counts, then the bucket-list counters

struct SortWs {
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* ghist;
    uint32_t* err;
    void* lb;  // two row sets of 32-bit words, or one of 64-bit words
    size_t lb_bytes;
    size_t rows;  // look-back rows: tiles of the smallest tile size, plus the listed buckets' extra tiles
    // bucket list of a split sort (with_perm only)
    uint32_t* large_count;
    uint4* large_tiles;
    uint32_t* large_start;
    uint32_t* large_hist;
    size_t max_buckets, max_tiles_any;
    // per-block first-digit counts and flags of a build's key kernel
    uint32_t* key_parts;
    uint32_t* key_bad;
    size_t bytes;
};

SortWs carve_sort(void* ws, size_t n, bool with_perm) {
    Carve c(ws);
    SortWs s{};
    s.keys_alt = c.take<uint64_t>(n);
    s.vals_alt = with_perm ? c.take<uint32_t>(n) : nullptr;
    s.ghist = c.take<uint32_t>(kGhistWords);
    s.large_count = s.ghist + kMaxPasses * kMaxRadix;
    s.err = c.take<uint32_t>(1);
    // a listed bucket holds more than kLocalCap keys; its tiles number at most
    // its keys / tile + 1
    s.max_buckets = with_perm ? n / (kLocalCap + 1) : 0;
    s.max_tiles_any = (n + kMinTile - 1) / kMinTile + s.max_buckets;
    s.rows = s.max_tiles_any;
    s.lb_bytes = s.rows * kMaxRadix * 8;  // 2 x 32-bit sets, or 1 x 64-bit set
    s.lb = c.take<uint8_t>(s.lb_bytes);
    if (with_perm) {
        s.large_tiles = c.take<uint4>(s.max_tiles_any);
        s.large_start = c.take<uint32_t>(s.max_buckets + 1);
        s.large_hist = c.take<uint32_t>((s.max_buckets + 1) * kLowPasses * kMaxRadix);
        s.key_parts = c.take<uint32_t>(static_cast<size_t>(kKeyBlocksMax) * kKeyDigitsMax * kMaxRadix);
        s.key_bad = c.take<uint32_t>(kKeyBlocksMax);
    }
    s.bytes = c.off;
    return s;
}

// Whether a sort of n particle keys takes the split path.
bool use_split(size_t n, int sig_bits, bool with_perm, const Variant& var) {
    return with_perm && sig_bits == 63 && var.split && n > 0;
}

}  // namespace

size_t sort_workspace_bytes(size_t n, bool with_perm) { return carve_sort(nullptr, n, with_perm).bytes; }

int sort_builtin_variant() { return kBuiltinVariant; }

namespace {
const Variant& variant_or_builtin(int v) { return kVariants[v >= 0 && v < kNumVariants ? v : kBuiltinVariant]; }
}  // namespace

int sort_passes(size_t n, int sig_bits, bool with_perm, int variant) {
    const Variant& var = variant_or_builtin(variant);
    if (use_split(n, sig_bits, with_perm, var)) return 4;  // top pass 1, the later top passes, buckets, low passes
    return (sig_bits + var.bits - 1) / var.bits;
}

cstone_status sort_prepare(void* ws, size_t n, bool with_perm, hipStream_t stream, uint32_t* clear_word,
                           int variant) {
    SortWs s = carve_sort(ws, n, with_perm);
    // only the first pass's look-back rows need clearing: each pass clears the
    // rows of the next (32-bit words), or words carry the pass's epoch (64-bit)
    const Variant& var = variant_or_builtin(variant);
    const size_t tile = static_cast<size_t>(var.block) * var.items;
    const size_t words = ((n + tile - 1) / tile) << var.bits;
    const bool wide = n >= (1ull << 30);
    const size_t lb_words = std::min(s.lb_bytes / 8, wide ? words : (words + 1) / 2);
    const size_t init_grid = std::max<size_t>(4, std::min<size_t>((lb_words + 255) / 256, 1024));
    hipLaunchKernelGGL(sort_init_kernel, dim3(init_grid), dim3(256), 0, stream, s.ghist,
                       static_cast<size_t>(kGhistWords), s.err, static_cast<uint64_t*>(s.lb), lb_words, clear_word);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

void sort_key_parts(void* ws, size_t n, bool with_perm, int sig_bits, int variant, uint32_t** hist_parts,
                    uint32_t** bad_parts, uint32_t* mask, uint32_t* shift, uint32_t* digits) {
    const Variant& var = variant_or_builtin(variant);
    const bool split = use_split(n, sig_bits, with_perm, var);
    *mask = (1u << var.bits) - 1u;
    *shift = split ? kSplitShift : 0u;
    *digits = split ? static_cast<uint32_t>(kSplitTop) : 1u;
    const SortWs s = carve_sort(ws, n, with_perm);
    *hist_parts = s.key_parts;
    *bad_parts = s.key_bad;
}

cstone_status sort_setup_from_keys(void* ws, size_t n, bool with_perm, int variant, uint32_t parts, uint32_t* flag,
                                   uint32_t* level6, hipStream_t stream) {
    if (!with_perm || parts == 0 || parts > kKeyBlocksMax) return CSTONE_ERR_INVALID_ARG;
    if (variant < 0 || variant >= kNumVariants) return CSTONE_ERR_INVALID_ARG;
    SortWs s = carve_sort(ws, n, with_perm);
    const Variant& var = kVariants[variant];
    const size_t tile = static_cast<size_t>(var.block) * var.items;
    const size_t words = ((n + tile - 1) / tile) << var.bits;
    const bool wide = n >= (1ull << 30);
    const size_t lb_words = std::min(s.lb_bytes / 8, wide ? words : (words + 1) / 2);
    const uint32_t radix = 1u << var.bits;
    const uint32_t digits = use_split(n, 63, with_perm, var) ? static_cast<uint32_t>(kSplitTop) : 1u;
    // the summing blocks and the flag block, and enough blocks besides for the clearing
    const uint32_t grid = std::max<uint32_t>(digits * kMaxRadix / kSetupCols + 1, kMaxRadix + 1);
    hipLaunchKernelGGL(sort_setup_kernel, dim3(grid), dim3(kKeyBlocksMax), 0, stream, s.ghist,
                       static_cast<size_t>(kGhistWords), s.err, static_cast<uint64_t*>(s.lb), lb_words, s.key_parts,
                       parts, radix, digits, s.key_bad, flag, level6);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

bool sort_uses_split(size_t n, int sig_bits, bool with_perm, int variant) {
    return use_split(n, sig_bits, with_perm, variant_or_builtin(variant));
}

namespace {

// Split sort (see the prefix-split kernels): top passes keys_in -> keys_out ->
// alt -> keys_out, buckets sorted in place in keys_out, low passes over the
// listed buckets keys_out -> alt -> ... -> keys_out.
cstone_status launch_split(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n,
                           const SortWs& s, const Variant& var, bool wide, hipStream_t stream,
                           hipEvent_t* pass_events, uint32_t* err, uint32_t* level6, bool top_counted) {
    constexpr int radix = 1 << kSplitBits;
    uint32_t* lb32[2] = {static_cast<uint32_t*>(s.lb), static_cast<uint32_t*>(s.lb) + s.rows * kMaxRadix};
    if (pass_events) CS_HIP(hipEventRecord(pass_events[0], stream));
    const uint64_t* src_k = keys_in;
    const uint32_t* src_v = nullptr;
    for (int p = 0; p < kSplitTop; ++p) {
        const bool to_out = ((kSplitTop - 1 - p) % 2) == 0;
        PassArgs a{};
        a.keys_in = src_k;
        a.vals_in = src_v;
        a.keys_out = to_out ? keys_out : s.keys_alt;
        a.vals_out = to_out ? perm_out : s.vals_alt;
        a.n = static_cast<uint32_t>(n);
        a.shift = kSplitShift + p * kSplitBits;
        a.ghist = s.ghist + p * radix;
        // every top digit's counts came from the key kernel (top_counted), else
        // each top pass counts the next one's
        a.ghist_next = p + 1 < kSplitTop && !top_counted ? s.ghist + (p + 1) * radix : nullptr;
        a.shift_next = kSplitShift + (p + 1) * kSplitBits;
        a.wide = wide;
        a.lb = wide ? s.lb : static_cast<void*>(lb32[p & 1]);
        a.lb_clear = (!wide && p + 1 < kSplitTop) ? static_cast<void*>(lb32[(p + 1) & 1]) : nullptr;
        a.epoch = static_cast<uint32_t>(p + 1);
        a.err = err;
        var.launch(a, p == 0, true, stream);
        src_k = a.keys_out;
        src_v = a.vals_out;
        // events after the first and the last top pass only: the later top
        // passes are timed together, with no event between their launches
        if (pass_events && (p == 0 || p == kSplitTop - 1))
            CS_HIP(hipEventRecord(pass_events[p == 0 ? 1 : 2], stream));
    }
    const uint32_t tile = static_cast<uint32_t>(var.block * var.items);
    LargeList L{};
    L.count = s.large_count;
    L.tiles = s.large_tiles;
    L.start = s.large_start;
    L.hist = s.large_hist;
    L.lb = wide ? s.lb : static_cast<void*>(lb32[0]);
    L.stride = kLowPasses * kMaxRadix;
    L.row_words = kMaxRadix;
    L.tile = tile;
    L.max_buckets = static_cast<uint32_t>(s.max_buckets);
    L.max_tiles = static_cast<uint32_t>((n + tile - 1) / tile + s.max_buckets);
    L.wide = wide ? 1u : 0u;
    const uint32_t chunks = static_cast<uint32_t>((n + kLocalChunk - 1) / kLocalChunk);
    hipLaunchKernelGGL((local_sort_kernel<kSplitBits, kLocalBlock, kLocalItems, false>), dim3(chunks),
                       dim3(kLocalBlock), 0, stream, keys_out, perm_out, static_cast<uint32_t>(n), kSplitShift, L, err,
                       level6, static_cast<const uint32_t*>(nullptr), 0u, static_cast<const uint32_t*>(nullptr));
    if (pass_events) CS_HIP(hipEventRecord(pass_events[3], stream));
    if (s.max_buckets > 0) {  // some bucket may be longer than one block sorts
        hipLaunchKernelGGL(large_hist_kernel, dim3(std::min(L.max_tiles, kListGrid)), dim3(512), 0, stream, keys_out,
                           static_cast<uint32_t>(n), L, static_cast<uint32_t>(radix - 1));
        SegArgs g{s.large_tiles, s.large_start, L.max_tiles, L.stride, s.large_count + 1};
        for (int p = 0; p < kLowPasses; ++p) {
            const bool from_alt = (p % 2) == 1;
            PassArgs a{};
            a.keys_in = from_alt ? s.keys_alt : keys_out;
            a.vals_in = from_alt ? s.vals_alt : perm_out;
            a.keys_out = from_alt ? keys_out : s.keys_alt;
            a.vals_out = from_alt ? perm_out : s.vals_alt;
            a.n = static_cast<uint32_t>(n);
            a.shift = static_cast<uint32_t>(p * kSplitBits);
            a.ghist = s.large_hist + p * radix;
            a.ghist_next = p + 1 < kLowPasses ? s.large_hist + (p + 1) * radix : nullptr;
            a.shift_next = static_cast<uint32_t>((p + 1) * kSplitBits);
            a.wide = wide;
            a.lb = wide ? s.lb : static_cast<void*>(lb32[p & 1]);
            a.lb_clear = (!wide && p + 1 < kLowPasses) ? static_cast<void*>(lb32[(p + 1) & 1]) : nullptr;
            a.epoch = static_cast<uint32_t>(kSplitTop + 1 + p);
            a.err = err;
            var.launch_list(a, g, s.large_count + 2 + p, stream);  // a tile counter per pass, cleared at set-up
        }
    }
    if (pass_events) CS_HIP(hipEventRecord(pass_events[4], stream));
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace

cstone_status launch_sort(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n,
                          int sig_bits, void* ws, size_t ws_bytes, hipStream_t stream, hipEvent_t* pass_events,
                          bool prepared, int variant, uint32_t* err_word, uint32_t* level6) {
    const bool with_perm = perm_out != nullptr;
    SortWs s = carve_sort(ws, n, with_perm);
    if (ws_bytes < s.bytes) return CSTONE_ERR_INVALID_ARG;
    if (n == 0) return CSTONE_OK;
    if (n > 0xffffffffull) return CSTONE_ERR_INVALID_ARG;
    if (variant >= kNumVariants) return CSTONE_ERR_INVALID_ARG;
    if (prepared && variant < 0) return CSTONE_ERR_INVALID_ARG;  // the set-up fixed the shape
    if (variant < 0) variant = with_perm && sig_bits == 63 ? sort_resolve_variant(n) : kBuiltinVariant;
    const Variant& var = kVariants[variant];
    const int radix = 1 << var.bits;
    const int passes = (sig_bits + var.bits - 1) / var.bits;
    if (passes < 1 || passes > kMaxPasses) return CSTONE_ERR_INVALID_ARG;
    const bool wide = n >= (1ull << 30);  // 30-bit look-back values otherwise

    const bool split = use_split(n, sig_bits, with_perm, var);
    if (!prepared) {
        cstone_status st = sort_prepare(ws, n, with_perm, stream, nullptr, variant);
        if (st != CSTONE_OK) return st;
        const size_t hblocks =
            std::max<size_t>(1, std::min<size_t>((n + kHistBlock * 16 - 1) / (kHistBlock * 16), 1024));
        hipLaunchKernelGGL(sort_hist0_kernel, dim3(hblocks), dim3(kHistBlock), 0, stream, keys_in,
                           static_cast<uint32_t>(n), split ? kSplitShift : 0u, static_cast<uint32_t>(radix - 1),
                           s.ghist);
    }
    uint32_t* err = err_word ? err_word : s.err;
    if (split)
        return launch_split(keys_in, keys_out, perm_out, n, s, var, wide, stream, pass_events, err, level6, prepared);

    uint32_t* lb32[2] = {static_cast<uint32_t*>(s.lb), static_cast<uint32_t*>(s.lb) + s.rows * kMaxRadix};
    if (pass_events) CS_HIP(hipEventRecord(pass_events[0], stream));
    const uint64_t* src_k = keys_in;
    const uint32_t* src_v = nullptr;
    for (int p = 0; p < passes; ++p) {
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        PassArgs a{};
        a.keys_in = src_k;
        a.vals_in = src_v;
        a.keys_out = to_out ? keys_out : s.keys_alt;
        a.vals_out = with_perm ? (to_out ? perm_out : s.vals_alt) : nullptr;
        a.n = static_cast<uint32_t>(n);
        a.shift = static_cast<uint32_t>(p * var.bits);
        a.ghist = s.ghist + p * radix;
        a.ghist_next = p + 1 < passes ? s.ghist + (p + 1) * radix : nullptr;
        a.shift_next = static_cast<uint32_t>((p + 1) * var.bits) & 63u;
        a.wide = wide;
        a.lb = wide ? s.lb : static_cast<void*>(lb32[p & 1]);
        a.lb_clear = (!wide && p + 1 < passes) ? static_cast<void*>(lb32[(p + 1) & 1]) : nullptr;
        a.epoch = static_cast<uint32_t>(p + 1);
        a.err = err;
        var.launch(a, p == 0, with_perm, stream);
        src_k = a.keys_out;
        src_v = a.vals_out;
        if (pass_events) CS_HIP(hipEventRecord(pass_events[p + 1], stream));  // one interval per pass
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}


// ---- segmented sort ---------------------------------------------------------

int sort_variant_count() { return kNumVariants; }

cstone_status set_lookback_patience(uint32_t waits) {
    CS_HIP(hipMemcpyToSymbol(HIP_SYMBOL(g_lookback_patience), &waits, sizeof waits));
    return CSTONE_OK;
}

SortVariantInfo sort_variant_info(int v) {
    const Variant& x = kVariants[(v >= 0 && v < kNumVariants) ? v : 0];
    return {x.bits, x.block, x.items, x.block * x.items, x.split ? 1 : 0};
}


namespace {

struct SegWs {
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* ghist;  // [set][pass][digit], then the bucket-list counters
    uint32_t stride;  // words per set
    uint32_t* err;
    void* lb;
    size_t lb_bytes;
    size_t rows;
    // split sorts (9-bit variants): the bucket list and each chunk's first set
    bool split;
    uint32_t* large_count;
    uint4* large_tiles;
    uint32_t* large_start;
    uint32_t* large_hist;
    uint32_t* chunk_set;
    size_t max_buckets, max_list_tiles, chunks;
    size_t bytes;
};

bool seg_split(int variant) { return kVariants[variant].split; }

SegWs carve_seg(void* ws, size_t n_total, size_t n_tiles, uint32_t n_sets, int variant) {
    const Variant& var = kVariants[variant];
    Carve c(ws);
    SegWs s{};
    s.split = seg_split(variant);
    s.keys_alt = c.take<uint64_t>(n_total);
    s.vals_alt = c.take<uint32_t>(n_total);
    s.stride = static_cast<uint32_t>(((64 + var.bits - 1) / var.bits) << var.bits);
    s.ghist = c.take<uint32_t>(static_cast<size_t>(n_sets) * s.stride + 64);
    s.large_count = s.ghist + static_cast<size_t>(n_sets) * s.stride;  // [0] buckets, [1] tiles, [2..] pass counters
    s.err = c.take<uint32_t>(1);
    s.rows = n_tiles;
    if (s.split) {
        // a listed bucket holds more than kLocalCap keys of one set; its tiles
        // number at most its keys / tile + 1
        const size_t tile = static_cast<size_t>(var.block) * var.items;
        s.max_buckets = n_total / (kLocalCap + 1);
        s.max_list_tiles = (n_total + tile - 1) / tile + s.max_buckets;
        s.rows = std::max(s.rows, s.max_list_tiles);
        s.chunks = (n_total + kLocalChunk - 1) / kLocalChunk;
    }
    s.lb_bytes = s.rows * kMaxRadix * 8;  // 2 x 32-bit sets, or 1 x 64-bit set
    s.lb = c.take<uint8_t>(s.lb_bytes);
    if (s.split) {
        s.large_tiles = c.take<uint4>(s.max_list_tiles);
        s.large_start = c.take<uint32_t>(s.max_buckets + 1);
        s.large_hist = c.take<uint32_t>((s.max_buckets + 1) * kLowPasses * kMaxRadix);
        s.chunk_set = c.take<uint32_t>(2 * (s.chunks + 1));
    }
    s.bytes = c.off;
    return s;
}

// chunk_set[b] = first set whose start is at or after b * kLocalChunk (n_sets
// if none), chunk_set[chunks + 1 + b] = that start (n if none).
__global__ __launch_bounds__(256) void chunk_set_kernel(const uint32_t* __restrict__ seg_base, uint32_t n_sets,
                                                        uint32_t* __restrict__ chunk_set, uint32_t chunks,
                                                        uint32_t n) {
    const uint32_t b = blockIdx.x * 256u + threadIdx.x;
    if (b >= chunks) return;
    const uint64_t at = static_cast<uint64_t>(b) * kLocalChunk;
    uint32_t lo = 0, hi = n_sets;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) / 2;
        if (seg_base[mid] < at) lo = mid + 1;
        else hi = mid;
    }
    chunk_set[b] = lo;
    chunk_set[chunks + 1 + b] = lo < n_sets ? seg_base[lo] : n;
}

}  // namespace

size_t sort_seg_workspace_bytes(size_t n_total, size_t n_tiles, uint32_t n_sets, int variant) {
    return carve_seg(nullptr, n_total, n_tiles, n_sets, variant).bytes;
}

cstone_status sort_seg_prepare(void* ws, size_t n_total, size_t n_tiles, uint32_t n_sets, int variant,
                               hipStream_t stream) {
    SegWs s = carve_seg(ws, n_total, n_tiles, n_sets, variant);
    // the first pass's rows (one per tile); each pass clears the next's, or
    // 64-bit words carry the pass's epoch
    const size_t lb_words = std::min(s.lb_bytes / 8, n_tiles * kMaxRadix);
    const size_t gwords = static_cast<size_t>(n_sets) * s.stride + 64;  // with the bucket-list counters
    const size_t init_grid =
        std::max<size_t>(4, std::min<size_t>((std::max(lb_words, gwords) + 255) / 256, 2048));
    hipLaunchKernelGGL(sort_init_kernel, dim3(init_grid), dim3(256), 0, stream, s.ghist, gwords, s.err,
                       static_cast<uint64_t*>(s.lb), lb_words, static_cast<uint32_t*>(nullptr));
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

uint32_t* sort_seg_first_histogram(void* ws, size_t n_total, size_t n_tiles, uint32_t n_sets, int variant,
                                   uint32_t* stride, uint32_t* mask, uint32_t* shift) {
    SegWs s = carve_seg(ws, n_total, n_tiles, n_sets, variant);
    *stride = s.stride;
    *mask = (1u << kVariants[variant].bits) - 1u;
    *shift = s.split ? kSplitShift : 0u;
    return s.ghist;
}

namespace {

// Segmented split sort: the top passes per set (keys_in -> keys_out -> alt ->
// keys_out), the buckets of every set in place, then the low passes over the
// listed buckets, as in the split sort of one key set.
cstone_status launch_split_seg(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n_total,
                               const uint4* tiles, uint32_t n_tiles, const uint32_t* seg_base, uint32_t n_sets,
                               bool wide, const SegWs& s, const Variant& var, uint32_t* err, hipStream_t stream) {
    constexpr int radix = 1 << kSplitBits;
    uint32_t* lb32[2] = {static_cast<uint32_t*>(s.lb), static_cast<uint32_t*>(s.lb) + s.rows * kMaxRadix};
    const uint32_t chunks = static_cast<uint32_t>(s.chunks);
    hipLaunchKernelGGL(chunk_set_kernel, dim3((chunks + 255) / 256), dim3(256), 0, stream, seg_base, n_sets,
                       s.chunk_set, chunks, static_cast<uint32_t>(n_total));
    SegArgs g{tiles, seg_base, n_tiles, s.stride, nullptr};
    const uint64_t* src_k = keys_in;
    const uint32_t* src_v = nullptr;
    for (int p = 0; p < kSplitTop; ++p) {
        const bool to_out = ((kSplitTop - 1 - p) % 2) == 0;
        PassArgs a{};
        a.keys_in = src_k;
        a.vals_in = src_v;
        a.keys_out = to_out ? keys_out : s.keys_alt;
        a.vals_out = to_out ? perm_out : s.vals_alt;
        a.n = static_cast<uint32_t>(n_total);
        a.shift = kSplitShift + p * kSplitBits;
        a.ghist = s.ghist + p * radix;
        a.ghist_next = p + 1 < kSplitTop ? s.ghist + (p + 1) * radix : nullptr;
        a.shift_next = kSplitShift + (p + 1) * kSplitBits;
        a.wide = wide;
        a.lb = wide ? s.lb : static_cast<void*>(lb32[p & 1]);
        a.lb_clear = (!wide && p + 1 < kSplitTop) ? static_cast<void*>(lb32[(p + 1) & 1]) : nullptr;
        a.epoch = static_cast<uint32_t>(p + 1);
        a.err = err;
        var.launch_seg(a, g, p == 0, true, stream);
        src_k = a.keys_out;
        src_v = a.vals_out;
    }
    const uint32_t tile = static_cast<uint32_t>(var.block * var.items);
    LargeList L{};
    L.count = s.large_count;
    L.tiles = s.large_tiles;
    L.start = s.large_start;
    L.hist = s.large_hist;
    L.lb = wide ? s.lb : static_cast<void*>(lb32[0]);
    L.stride = kLowPasses * kMaxRadix;
    L.row_words = kMaxRadix;
    L.tile = tile;
    L.max_buckets = static_cast<uint32_t>(s.max_buckets);
    L.max_tiles = static_cast<uint32_t>(s.max_list_tiles);
    L.wide = wide ? 1u : 0u;
    hipLaunchKernelGGL((local_sort_kernel<kSplitBits, kLocalBlock, kLocalItems, true>), dim3(chunks),
                       dim3(kLocalBlock), 0, stream, keys_out, perm_out, static_cast<uint32_t>(n_total), kSplitShift,
                       L, err, static_cast<uint32_t*>(nullptr), seg_base, n_sets,
                       static_cast<const uint32_t*>(s.chunk_set));
    if (s.max_buckets > 0) {  // some bucket may be longer than one block sorts
        hipLaunchKernelGGL(large_hist_kernel, dim3(std::min(L.max_tiles, kListGrid)), dim3(512), 0, stream, keys_out,
                           static_cast<uint32_t>(n_total), L, static_cast<uint32_t>(radix - 1));
        SegArgs gl{s.large_tiles, s.large_start, L.max_tiles, L.stride, s.large_count + 1};
        for (int p = 0; p < kLowPasses; ++p) {
            const bool from_alt = (p % 2) == 1;
            PassArgs a{};
            a.keys_in = from_alt ? s.keys_alt : keys_out;
            a.vals_in = from_alt ? s.vals_alt : perm_out;
            a.keys_out = from_alt ? keys_out : s.keys_alt;
            a.vals_out = from_alt ? perm_out : s.vals_alt;
            a.n = static_cast<uint32_t>(n_total);
            a.shift = static_cast<uint32_t>(p * kSplitBits);
            a.ghist = s.large_hist + p * radix;
            a.ghist_next = p + 1 < kLowPasses ? s.large_hist + (p + 1) * radix : nullptr;
            a.shift_next = static_cast<uint32_t>((p + 1) * kSplitBits);
            a.wide = wide;
            a.lb = wide ? s.lb : static_cast<void*>(lb32[p & 1]);
            a.lb_clear = (!wide && p + 1 < kLowPasses) ? static_cast<void*>(lb32[(p + 1) & 1]) : nullptr;
            a.epoch = static_cast<uint32_t>(kSplitTop + 1 + p);
            a.err = err;
            var.launch_list(a, gl, s.large_count + 2 + p, stream);  // a tile counter per pass, cleared at set-up
        }
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace

cstone_status launch_sort_segmented(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out,
                                    size_t n_total, const uint4* tiles, uint32_t n_tiles, const uint32_t* seg_base,
                                    uint32_t n_sets, size_t max_set, int sig_bits, int variant, void* ws,
                                    size_t ws_bytes, hipStream_t stream, uint32_t* err_word) {
    if (variant < 0 || variant >= kNumVariants) return CSTONE_ERR_INVALID_ARG;
    SegWs s = carve_seg(ws, n_total, n_tiles, n_sets, variant);
    if (ws_bytes < s.bytes) return CSTONE_ERR_INVALID_ARG;
    if (n_total == 0 || n_tiles == 0) return CSTONE_OK;
    if (n_total > 0xffffffffull || !perm_out) return CSTONE_ERR_INVALID_ARG;
    const Variant& var = kVariants[variant];
    const int radix = 1 << var.bits;
    const int passes = (sig_bits + var.bits - 1) / var.bits;
    if (passes < 1 || static_cast<uint32_t>(passes * radix) > s.stride) return CSTONE_ERR_INVALID_ARG;
    const bool wide = max_set >= (1ull << 30);
    uint32_t* err = err_word ? err_word : s.err;
    if (s.split && sig_bits == 63)
        return launch_split_seg(keys_in, keys_out, perm_out, n_total, tiles, n_tiles, seg_base, n_sets, wide, s, var,
                                err, stream);
    if (s.split) return CSTONE_ERR_INVALID_ARG;  // its first histogram was taken on the top digit
    uint32_t* lb32[2] = {static_cast<uint32_t*>(s.lb), static_cast<uint32_t*>(s.lb) + s.rows * kMaxRadix};
    SegArgs g{tiles, seg_base, n_tiles, s.stride, nullptr};
    const uint64_t* src_k = keys_in;
    const uint32_t* src_v = nullptr;
    for (int p = 0; p < passes; ++p) {
        const bool to_out = ((passes - 1 - p) % 2) == 0;
        PassArgs a{};
        a.keys_in = src_k;
        a.vals_in = src_v;
        a.keys_out = to_out ? keys_out : s.keys_alt;
        a.vals_out = to_out ? perm_out : s.vals_alt;
        a.n = static_cast<uint32_t>(n_total);
        a.shift = static_cast<uint32_t>(p * var.bits);
        a.ghist = s.ghist + p * radix;
        a.ghist_next = p + 1 < passes ? s.ghist + (p + 1) * radix : nullptr;
        a.shift_next = static_cast<uint32_t>((p + 1) * var.bits) & 63u;
        a.wide = wide;
        a.lb = wide ? s.lb : static_cast<void*>(lb32[p & 1]);
        a.lb_clear = (!wide && p + 1 < passes) ? static_cast<void*>(lb32[(p + 1) & 1]) : nullptr;
        a.epoch = static_cast<uint32_t>(p + 1);
        a.err = err;
        var.launch_seg(a, g, p == 0, true, stream);
        src_k = a.keys_out;
        src_v = a.vals_out;
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace cs
