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
#include <atomic>
#include <cstdlib>

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

// Counts of the lowest digit (mask = radix - 1).
__global__ __launch_bounds__(kHistBlock) void sort_hist0_kernel(const uint64_t* __restrict__ keys, uint32_t n,
                                                                 uint32_t mask, uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[kMaxRadix];
    for (int i = threadIdx.x; i < kMaxRadix; i += kHistBlock) h[i] = 0;
    __syncthreads();
    const uint32_t stride = gridDim.x * kHistBlock;
    for (uint32_t i = blockIdx.x * kHistBlock + threadIdx.x; i < n; i += stride)
        atomicAdd(&h[static_cast<uint32_t>(keys[i]) & mask], 1u);
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
};

// Exclusive prefix of one digit over the tiles before `tile` (rows of `radix`
// words). WIN predecessors are read per round trip, nearest first; the walk
// stops at the first inclusive prefix and waits at the first empty word.
template <class LB, int WIN>
__device__ __forceinline__ uint64_t digit_lookback(const typename LB::word* col, uint32_t radix, uint32_t tile,
                                                   uint32_t first, uint32_t epoch, uint32_t* err) {
    // tiles first .. tile-1 precede this one in its segment; `first` published an inclusive prefix
    uint64_t excl = 0;
    uint32_t spins = 0;
    const int64_t lo = first;
    int64_t p = static_cast<int64_t>(tile) - 1;
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
        if (done) break;
        if (stalled) {
            if (++spins > kSpinLimit) {
                atomicOr(err, kErrSpin);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
    }
    return excl;
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
                                              uint32_t* nhist, uint32_t* ddelta, uint64_t* scan_tmp) {
    constexpr int RADIX = 1 << BITS;
    constexpr int W = BLOCK / kWave;
    constexpr int TILE = BLOCK * ITEMS;
    uint32_t* stage32 = reinterpret_cast<uint32_t*>(stage);
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = lane_id();
    const uint32_t wave = tid / kWave;
    const uint32_t tile = td.tile;
    const uint32_t tile_base = td.base;
    const uint32_t tile_count = FULL ? static_cast<uint32_t>(TILE) : td.count;
    const uint32_t end = tile_base + tile_count;  // keys at or past `end` belong to others
    const uint32_t wave_base = tile_base + wave * ITEMS * kWave;

    // this pass's digit counts of the whole set, for the global digit offsets
    const uint32_t gcount = tid < RADIX ? ghist[tid] : 0u;
    uint64_t k[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = wave_base + i * kWave + lane;
        k[i] = (FULL || idx < end) ? keys_in[idx] : 0ull;
    }
    __syncthreads();  // counters cleared

    // stable rank of every key among the keys of its wave with the same digit
    uint32_t rank[ITEMS];
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
        rank[i] = base + below;
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
    uint32_t lpos[ITEMS];
#pragma unroll
    for (int i = 0; i < ITEMS; ++i) {
        const uint32_t idx = wave_base + i * kWave + lane;
        lpos[i] = whist[wave][digit_of<BITS>(k[i], shift)] + rank[i];
        if (FULL || idx < end) stage[lpos[i]] = k[i];
    }
    // the permutation values are only needed for the scatter: start loading them
    // (not earlier: the keys must be dead by then to keep the registers in budget)
    __builtin_amdgcn_sched_barrier(0);
    uint32_t v[ITEMS];
    if (WITH_VALUES) {
#pragma unroll
        for (int i = 0; i < ITEMS; ++i) {
            const uint32_t idx = wave_base + i * kWave + lane;
            v[i] = FIRST ? idx - td.seg_base : ((FULL || idx < end) ? vals_in[idx] : 0u);
        }
    }
    if (tid < RADIX) {
        uint64_t excl = 0;
        if (tile != td.first) {
            excl = digit_lookback<LB, WIN>(lb + tid, RADIX, tile, td.first, epoch, err);
            LB::store(lb + static_cast<size_t>(tile) * RADIX + tid, LB::make(2u, epoch, excl + total));
        }
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
            if (FULL || idx < end) stage32[lpos[i]] = v[i];
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

// Tile of block b. Blocks are dealt to the 8 XCDs in turn; with XG > 1 every
// XCD takes XG consecutive tiles in a row, so that where one tile's run of a
// digit ends and the next tile's run begins (a partly written 64-byte
// segment) both writes meet in the same L2. A tile then waits only on tiles
// whose blocks are at most 8 XG - 1 dispatches later: the look-back progresses
// whenever 8 XG blocks of the pass can be resident. With XG = 8 that is 64 of
// the 256-512 a CU-filling pass holds, so even several passes sharing the GPU
// (sorts on other streams) leave one of them enough to finish and free room.
// The last, incomplete round of 8 XG blocks keeps tile = block.
template <int XG>
__device__ __forceinline__ uint32_t tile_of_block(uint32_t b, uint32_t nblocks) {
    constexpr uint32_t R = 8u * XG;
    if (XG == 1 || b >= nblocks / R * R) return b;
    const uint32_t r = b / R, q = b % R;
    return (r * 8u + q % 8u) * XG + q / 8u;
}

template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool WITH_VALUES, class LB, int XG>
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
    // tiles follow the block index: the dispatcher starts lower blocks first,
    // so every tile a block waits for is running or done
    const uint32_t tile = tile_of_block<XG>(blockIdx.x, gridDim.x);
    if (lb_clear && tid < RADIX) lb_clear[static_cast<size_t>(tile) * RADIX + tid] = 0;  // rows of the next pass
    for (int i = tid; i < W * RADIX; i += BLOCK) (&whist[0][0])[i] = 0;
    if (tid < RADIX) nhist[tid] = 0;
    const uint32_t base = tile * static_cast<uint32_t>(TILE);
    const TileDesc td{tile, base, min(n - base, static_cast<uint32_t>(TILE)), 0u, 0u};
    if (td.count == static_cast<uint32_t>(TILE))
        onesweep_tile<BITS, BLOCK, ITEMS, WIN, FIRST, WITH_VALUES, LB, true>(
            td, keys_in, vals_in, keys_out, vals_out, n, shift, ghist, ghist_next, shift_next, lb, epoch, err, stage,
            whist, nhist, ddelta, scan_tmp);
    else
        onesweep_tile<BITS, BLOCK, ITEMS, WIN, FIRST, WITH_VALUES, LB, false>(
            td, keys_in, vals_in, keys_out, vals_out, n, shift, ghist, ghist_next, shift_next, lb, epoch, err, stage,
            whist, nhist, ddelta, scan_tmp);
}

// Segmented pass: many independent key sets in one launch. Block b sorts
// tile tiles[b] = {first key, key count, first tile of its set, set}; every
// set has its own digit histograms (ghist + set * hist_stride) and its own
// look-back chain, and its permutation values count from the set's start.
template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool WITH_VALUES, class LB, int XG>
__global__ __launch_bounds__(BLOCK, (kMinBlocks<BLOCK, ITEMS>)) void onesweep_seg_kernel(const uint64_t* __restrict__ keys_in,
                                                              const uint32_t* __restrict__ vals_in,
                                                              uint64_t* __restrict__ keys_out,
                                                              uint32_t* __restrict__ vals_out, uint32_t n,
                                                              uint32_t shift, const uint32_t* __restrict__ ghist,
                                                              uint32_t* __restrict__ ghist_next, uint32_t shift_next,
                                                              uint32_t hist_stride, const uint4* __restrict__ tiles,
                                                              const uint32_t* __restrict__ seg_base,
                                                              typename LB::word* lb, typename LB::word* lb_clear,
                                                              uint32_t epoch, uint32_t* err) {
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
    const uint32_t tile = tile_of_block<XG>(blockIdx.x, gridDim.x);
    if (lb_clear && tid < RADIX) lb_clear[static_cast<size_t>(tile) * RADIX + tid] = 0;
    for (int i = tid; i < W * RADIX; i += BLOCK) (&whist[0][0])[i] = 0;
    if (tid < RADIX) nhist[tid] = 0;
    const uint4 t = tiles[tile];
    const TileDesc td{tile, t.x, t.y, t.z, seg_base[t.w]};
    const uint32_t* gh = ghist + static_cast<size_t>(t.w) * hist_stride;
    uint32_t* gn = ghist_next ? ghist_next + static_cast<size_t>(t.w) * hist_stride : nullptr;
    if (td.count == static_cast<uint32_t>(TILE))
        onesweep_tile<BITS, BLOCK, ITEMS, WIN, FIRST, WITH_VALUES, LB, true>(
            td, keys_in, vals_in, keys_out, vals_out, n, shift, gh, gn, shift_next, lb, epoch, err, stage, whist,
            nhist, ddelta, scan_tmp);
    else
        onesweep_tile<BITS, BLOCK, ITEMS, WIN, FIRST, WITH_VALUES, LB, false>(
            td, keys_in, vals_in, keys_out, vals_out, n, shift, gh, gn, shift_next, lb, epoch, err, stage, whist,
            nhist, ddelta, scan_tmp);
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

template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool VALS, int XG>
void launch_one(const PassArgs& a, hipStream_t stream) {
    constexpr uint32_t tile = BLOCK * ITEMS;
    const dim3 grid((a.n + tile - 1) / tile), block(BLOCK);
    if (a.wide)
        hipLaunchKernelGGL((onesweep_kernel<BITS, BLOCK, ITEMS, WIN, FIRST, VALS, Lb64, XG>), grid, block, 0, stream,
                           a.keys_in, a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next,
                           a.shift_next, static_cast<uint64_t*>(a.lb), nullptr, a.epoch, a.err);
    else
        hipLaunchKernelGGL((onesweep_kernel<BITS, BLOCK, ITEMS, WIN, FIRST, VALS, Lb32, XG>), grid, block, 0, stream,
                           a.keys_in, a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next,
                           a.shift_next, static_cast<uint32_t*>(a.lb), static_cast<uint32_t*>(a.lb_clear), a.epoch,
                           a.err);
}

template <int BITS, int BLOCK, int ITEMS, int WIN, int XG>
void launch_pass_t(const PassArgs& a, bool first, bool with_values, hipStream_t stream) {
    if (with_values && first)
        launch_one<BITS, BLOCK, ITEMS, WIN, true, true, XG>(a, stream);
    else if (with_values)
        launch_one<BITS, BLOCK, ITEMS, WIN, false, true, XG>(a, stream);
    else
        launch_one<BITS, BLOCK, ITEMS, WIN, false, false, XG>(a, stream);
}

struct SegArgs {
    const uint4* tiles;
    const uint32_t* seg_base;
    uint32_t n_tiles;
    uint32_t hist_stride;
};

template <int BITS, int BLOCK, int ITEMS, int WIN, bool FIRST, bool VALS, int XG>
void launch_one_seg(const PassArgs& a, const SegArgs& g, hipStream_t stream) {
    const dim3 grid(g.n_tiles), block(BLOCK);
    if (a.wide)
        hipLaunchKernelGGL((onesweep_seg_kernel<BITS, BLOCK, ITEMS, WIN, FIRST, VALS, Lb64, XG>), grid, block, 0, stream,
                           a.keys_in, a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next,
                           a.shift_next, g.hist_stride, g.tiles, g.seg_base, static_cast<uint64_t*>(a.lb), nullptr,
                           a.epoch, a.err);
    else
        hipLaunchKernelGGL((onesweep_seg_kernel<BITS, BLOCK, ITEMS, WIN, FIRST, VALS, Lb32, XG>), grid, block, 0, stream,
                           a.keys_in, a.vals_in, a.keys_out, a.vals_out, a.n, a.shift, a.ghist, a.ghist_next,
                           a.shift_next, g.hist_stride, g.tiles, g.seg_base, static_cast<uint32_t*>(a.lb),
                           static_cast<uint32_t*>(a.lb_clear), a.epoch, a.err);
}

template <int BITS, int BLOCK, int ITEMS, int WIN, int XG>
void launch_seg_t(const PassArgs& a, const SegArgs& g, bool first, bool with_values, hipStream_t stream) {
    if (with_values && first)
        launch_one_seg<BITS, BLOCK, ITEMS, WIN, true, true, XG>(a, g, stream);
    else if (with_values)
        launch_one_seg<BITS, BLOCK, ITEMS, WIN, false, true, XG>(a, g, stream);
    else
        launch_one_seg<BITS, BLOCK, ITEMS, WIN, false, false, XG>(a, g, stream);
}

struct Variant {
    int bits, block, items, window, xcd_group;
    void (*launch)(const PassArgs&, bool, bool, hipStream_t);
    void (*launch_seg)(const PassArgs&, const SegArgs&, bool, bool, hipStream_t);
};

#define CS_VARIANT(B, BL, IT, WI, XG) {B, BL, IT, WI, XG, launch_pass_t<B, BL, IT, WI, XG>, launch_seg_t<B, BL, IT, WI, XG>}
const Variant kVariants[] = {
    CS_VARIANT(9, 512, 16, 4, 8), CS_VARIANT(9, 512, 16, 4, 1), CS_VARIANT(8, 512, 16, 4, 8),
    CS_VARIANT(9, 512, 12, 4, 8), CS_VARIANT(9, 512, 32, 4, 8), CS_VARIANT(8, 512, 16, 4, 1),
    CS_VARIANT(9, 512, 12, 4, 1), CS_VARIANT(9, 512, 32, 4, 1),
};
#undef CS_VARIANT
constexpr int kNumVariants = sizeof(kVariants) / sizeof(kVariants[0]);

int builtin_variant() {
    static const int v = [] {
        const char* e = std::getenv("CSTONE_SORT_VARIANT");
        int x = e ? std::atoi(e) : 0;  // 9-bit digits, 512 x 16 tiles, 8 tiles in a row per XCD
        return (x >= 0 && x < kNumVariants) ? x : 0;
    }();
    return v;
}

std::atomic<int> g_tuned_variant{-1};  // set by the autotuner

int default_variant() {
    const int t = g_tuned_variant.load(std::memory_order_relaxed);
    return t >= 0 ? t : builtin_variant();
}

struct SortWs {
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* ghist;
    uint32_t* err;
    void* lb;  // two row sets of 32-bit words, or one of 64-bit words
    size_t lb_bytes;
    size_t rows;  // tiles of the smallest tile size
    size_t bytes;
};

SortWs carve_sort(void* ws, size_t n, bool with_perm) {
    Carve c(ws);
    SortWs s{};
    s.keys_alt = c.take<uint64_t>(n);
    s.vals_alt = with_perm ? c.take<uint32_t>(n) : nullptr;
    s.ghist = c.take<uint32_t>(kMaxPasses * kMaxRadix);
    s.err = c.take<uint32_t>(1);
    s.rows = (n + kMinTile - 1) / kMinTile;
    s.lb_bytes = s.rows * kMaxRadix * 8;  // 2 x 32-bit sets, or 1 x 64-bit set
    s.lb = c.take<uint8_t>(s.lb_bytes);
    s.bytes = c.off;
    return s;
}

}  // namespace

size_t sort_workspace_bytes(size_t n, bool with_perm) { return carve_sort(nullptr, n, with_perm).bytes; }

int sort_passes(int sig_bits) {
    const int bits = kVariants[default_variant()].bits;
    return (sig_bits + bits - 1) / bits;
}

cstone_status sort_prepare(void* ws, size_t n, bool with_perm, hipStream_t stream, uint32_t* clear_word,
                           int variant) {
    SortWs s = carve_sort(ws, n, with_perm);
    // only the first pass's look-back rows need clearing: each pass clears the
    // rows of the next (32-bit words), or words carry the pass's epoch (64-bit)
    const Variant& var = kVariants[variant >= 0 && variant < kNumVariants ? variant : default_variant()];
    const size_t tile = static_cast<size_t>(var.block) * var.items;
    const size_t words = ((n + tile - 1) / tile) << var.bits;
    const bool wide = n >= (1ull << 30);
    const size_t lb_words = std::min(s.lb_bytes / 8, wide ? words : (words + 1) / 2);
    const size_t init_grid = std::max<size_t>(4, std::min<size_t>((lb_words + 255) / 256, 1024));
    hipLaunchKernelGGL(sort_init_kernel, dim3(init_grid), dim3(256), 0, stream, s.ghist,
                       static_cast<size_t>(kMaxPasses) * kMaxRadix, s.err, static_cast<uint64_t*>(s.lb), lb_words,
                       clear_word);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

uint32_t* sort_first_histogram(void* ws, size_t n, bool with_perm, uint32_t* mask) {
    *mask = (1u << kVariants[default_variant()].bits) - 1u;
    return carve_sort(ws, n, with_perm).ghist;
}

cstone_status launch_sort(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out, size_t n,
                          int sig_bits, void* ws, size_t ws_bytes, hipStream_t stream, hipEvent_t* pass_events,
                          bool prepared, int variant) {
    const bool with_perm = perm_out != nullptr;
    SortWs s = carve_sort(ws, n, with_perm);
    if (ws_bytes < s.bytes) return CSTONE_ERR_INVALID_ARG;
    if (n == 0) return CSTONE_OK;
    if (n > 0xffffffffull) return CSTONE_ERR_INVALID_ARG;
    if (variant >= kNumVariants) return CSTONE_ERR_INVALID_ARG;
    if (prepared && variant >= 0 && variant != default_variant()) return CSTONE_ERR_INVALID_ARG;
    const Variant& var = kVariants[variant >= 0 ? variant : default_variant()];
    const int radix = 1 << var.bits;
    const int passes = (sig_bits + var.bits - 1) / var.bits;
    if (passes < 1 || passes > kMaxPasses) return CSTONE_ERR_INVALID_ARG;
    const bool wide = n >= (1ull << 30);  // 30-bit look-back values otherwise

    if (!prepared) {
        cstone_status st = sort_prepare(ws, n, with_perm, stream, nullptr, variant);
        if (st != CSTONE_OK) return st;
        const size_t hblocks =
            std::max<size_t>(1, std::min<size_t>((n + kHistBlock * 16 - 1) / (kHistBlock * 16), 1024));
        hipLaunchKernelGGL(sort_hist0_kernel, dim3(hblocks), dim3(kHistBlock), 0, stream, keys_in,
                           static_cast<uint32_t>(n), static_cast<uint32_t>(radix - 1), s.ghist);
    }

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
        a.err = s.err;
        var.launch(a, p == 0, with_perm, stream);
        src_k = a.keys_out;
        src_v = a.vals_out;
        if (pass_events) CS_HIP(hipEventRecord(pass_events[p + 1], stream));
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}


// ---- segmented sort ---------------------------------------------------------

int sort_variant_count() { return kNumVariants; }

SortVariantInfo sort_variant_info(int v) {
    const Variant& x = kVariants[(v >= 0 && v < kNumVariants) ? v : 0];
    return {x.bits, x.block, x.items, x.block * x.items};
}

int sort_default_variant() { return default_variant(); }

void sort_set_tuned_variant(int v) { g_tuned_variant.store((v >= 0 && v < kNumVariants) ? v : -1); }

namespace {

struct SegWs {
    uint64_t* keys_alt;
    uint32_t* vals_alt;
    uint32_t* ghist;  // [set][pass][digit]
    uint32_t stride;  // words per set
    uint32_t* err;
    void* lb;
    size_t lb_bytes;
    size_t rows;
    size_t bytes;
};

SegWs carve_seg(void* ws, size_t n_total, size_t n_tiles, uint32_t n_sets, int variant) {
    const Variant& var = kVariants[variant];
    Carve c(ws);
    SegWs s{};
    s.keys_alt = c.take<uint64_t>(n_total);
    s.vals_alt = c.take<uint32_t>(n_total);
    s.stride = static_cast<uint32_t>(((64 + var.bits - 1) / var.bits) << var.bits);
    s.ghist = c.take<uint32_t>(static_cast<size_t>(n_sets) * s.stride);
    s.err = c.take<uint32_t>(1);
    s.rows = n_tiles;
    s.lb_bytes = s.rows * kMaxRadix * 8;  // 2 x 32-bit sets, or 1 x 64-bit set
    s.lb = c.take<uint8_t>(s.lb_bytes);
    s.bytes = c.off;
    return s;
}

}  // namespace

size_t sort_seg_workspace_bytes(size_t n_total, size_t n_tiles, uint32_t n_sets, int variant) {
    return carve_seg(nullptr, n_total, n_tiles, n_sets, variant).bytes;
}

cstone_status sort_seg_prepare(void* ws, size_t n_total, size_t n_tiles, uint32_t n_sets, int variant,
                               hipStream_t stream) {
    SegWs s = carve_seg(ws, n_total, n_tiles, n_sets, variant);
    const size_t lb_words = s.lb_bytes / 8;
    const size_t gwords = static_cast<size_t>(n_sets) * s.stride;
    const size_t init_grid =
        std::max<size_t>(4, std::min<size_t>((std::max(lb_words, gwords) + 255) / 256, 2048));
    hipLaunchKernelGGL(sort_init_kernel, dim3(init_grid), dim3(256), 0, stream, s.ghist, gwords, s.err,
                       static_cast<uint64_t*>(s.lb), lb_words, static_cast<uint32_t*>(nullptr));
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

uint32_t* sort_seg_first_histogram(void* ws, size_t n_total, size_t n_tiles, uint32_t n_sets, int variant,
                                   uint32_t* stride, uint32_t* mask) {
    SegWs s = carve_seg(ws, n_total, n_tiles, n_sets, variant);
    *stride = s.stride;
    *mask = (1u << kVariants[variant].bits) - 1u;
    return s.ghist;
}

cstone_status launch_sort_segmented(const uint64_t* keys_in, uint64_t* keys_out, uint32_t* perm_out,
                                    size_t n_total, const uint4* tiles, uint32_t n_tiles, const uint32_t* seg_base,
                                    uint32_t n_sets, size_t max_set, int sig_bits, int variant, void* ws,
                                    size_t ws_bytes, hipStream_t stream) {
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
    uint32_t* lb32[2] = {static_cast<uint32_t*>(s.lb), static_cast<uint32_t*>(s.lb) + s.rows * kMaxRadix};
    SegArgs g{tiles, seg_base, n_tiles, s.stride};
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
        a.err = s.err;
        var.launch_seg(a, g, p == 0, true, stream);
        src_k = a.keys_out;
        src_v = a.vals_out;
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace cs
