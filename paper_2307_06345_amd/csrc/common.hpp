// Device and host helpers shared by the HIP kernels of the octree build.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "cstone.h"

namespace cs {

constexpr int kL = 21;
constexpr uint64_t kKeyEnd = 1ull << 63;  // 8^21, closes every cornerstone array
constexpr int kWave = 64;

// Error word kept in workspaces: a device-side wait that gave up sets it.
constexpr uint32_t kErrSpin = 1u << 8;  // internal error bits sit above the public CSTONE_FLAG_* bits

// Spin budget for look-back waits (each spin sleeps ~64 cycles); a wait that
// exhausts it marks the error word and proceeds, so every wave terminates.
constexpr uint32_t kSpinLimit = 1u << 20;

#define CS_HIP(expr)                                     \
    do {                                                 \
        hipError_t cs_e_ = (expr);                       \
        if (cs_e_ != hipSuccess) return CSTONE_ERR_DEVICE; \
    } while (0)

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Bump allocator over a caller workspace (256-byte aligned slices).
struct Carve {
    char* base;
    size_t off = 0;
    explicit Carve(void* p) : base(static_cast<char*>(p)) {}
    template <class T>
    T* take(size_t count) {
        T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
        off = align_up(off + count * sizeof(T), 256);
        return p;
    }
};

// ---- wave64 primitives ---------------------------------------------------

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Number of set bits of `mask` in lanes below this one.
__device__ __forceinline__ uint32_t lanes_below(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
}

template <class T>
__device__ __forceinline__ T wave_inclusive_sum(T v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T o = __shfl_up(v, d, kWave);
        if (lane >= static_cast<uint32_t>(d)) v += o;
    }
    return v;
}

// Block-wide exclusive sum; `lds` holds one T per wave. Returns the exclusive
// prefix of this thread and writes the block total to *total.
template <class T, int BLOCK>
__device__ __forceinline__ T block_exclusive_sum(T v, T* lds, T* total) {
    constexpr int W = BLOCK / kWave;
    const uint32_t lane = lane_id();
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);  // wave-uniform
    T inc = wave_inclusive_sum(v);
    if (lane == kWave - 1) lds[wave] = inc;
    __syncthreads();
    T wave_prefix = 0, sum = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        T s = lds[w];
        if (w < static_cast<int>(wave)) wave_prefix += s;
        sum += s;
    }
    __syncthreads();
    *total = sum;
    return wave_prefix + inc - v;
}

// ---- agent-scope (cross-XCD) atomics for decoupled look-back ----------------

__device__ __forceinline__ uint64_t ld_agent(const uint64_t* p) {
    return __hip_atomic_load(const_cast<uint64_t*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Look-back status word: [63:62] flag (0 empty, 1 tile aggregate, 2 inclusive
// prefix), [61:48] epoch (which pass / round wrote it), [47:0] value.
constexpr uint64_t kFlagAgg = 1ull << 62;
constexpr uint64_t kFlagInc = 2ull << 62;
constexpr uint64_t kValueMask = (1ull << 48) - 1;

__device__ __forceinline__ uint64_t lb_word(uint64_t flag, uint32_t epoch, uint64_t value) {
    return flag | (static_cast<uint64_t>(epoch & 0x3fffu) << 48) | (value & kValueMask);
}

// Exclusive prefix of tile `tile` for one counter: walk back over the
// predecessors' words (stride `stride` between tiles) until an inclusive
// prefix is found. Words of another epoch count as not yet written.
__device__ __forceinline__ uint64_t lookback(const uint64_t* words, size_t stride, uint32_t tile,
                                             uint32_t epoch, uint32_t* err) {
    uint64_t excl = 0;
    int64_t p = static_cast<int64_t>(tile) - 1;
    uint32_t spins = 0;
    while (p >= 0) {
        uint64_t w = ld_agent(words + static_cast<size_t>(p) * stride);
        uint64_t flag = w & (3ull << 62);
        bool mine = ((w >> 48) & 0x3fffu) == (epoch & 0x3fffu);
        if (flag == 0 || !mine) {
            if (++spins > kSpinLimit) {
                atomicOr(err, kErrSpin);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += w & kValueMask;
        if (flag == kFlagInc) break;
        --p;
    }
    return excl;
}

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Exclusive prefix of `tile` over one counter (words[p] for tile p), resolved
// by a whole wave: each step reads the 64 * R nearest unresolved predecessors
// at once (R independent loads per lane, lane l holding tiles top - l - 64 r),
// so a long run of aggregates costs one round trip per 64 * R tiles. Every
// lane returns the same value; all 64 lanes must call it together.
template <int R = 4>
__device__ __forceinline__ uint64_t lookback_wave(const uint64_t* words, uint32_t tile, uint32_t epoch,
                                                  uint32_t* err) {
    const uint32_t lane = lane_id();
    uint64_t excl = 0;
    int64_t top = static_cast<int64_t>(tile) - 1;
    uint32_t spins = 0;
    while (top >= 0) {
        uint64_t w[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int64_t p = top - lane - static_cast<int64_t>(r) * kWave;
            w[r] = p >= 0 ? ld_agent(words + p) : 0ull;
        }
        bool found = false, wait = false;
        uint64_t part = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {  // sub-windows, nearest first
            if (found || wait) continue;
            const int64_t p = top - lane - static_cast<int64_t>(r) * kWave;
            const bool valid = p >= 0;
            const uint64_t flag = w[r] & (3ull << 62);
            const bool mine = ((w[r] >> 48) & 0x3fffu) == (epoch & 0x3fffu);
            const bool ready = !valid || (flag != 0 && mine);
            const uint64_t inc = __ballot(valid && ready && flag == kFlagInc);
            const uint64_t pending = __ballot(!ready);
            // lanes up to and including the nearest inclusive prefix (all if none)
            const uint64_t upto = inc ? ((inc & (~inc + 1)) << 1) - 1 : ~0ull;
            if (pending & upto) {
                wait = true;  // resume from this sub-window
                top -= static_cast<int64_t>(r) * kWave;
                continue;
            }
            part += (valid && ((upto >> lane) & 1ull)) ? (w[r] & kValueMask) : 0ull;
            if (inc) found = true;
        }
        excl += wave_sum<uint64_t>(part);
        if (found) break;
        if (wait) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicOr(err, kErrSpin);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        top -= static_cast<int64_t>(R) * kWave;
    }
    return excl;
}

// First index in [lo, hi) of a sorted array whose key is >= k, searched by a
// whole wave with 63 probes per step (log64 dependent loads instead of log2).
// lo, hi and k must be the same in every lane; all 64 lanes must call it.
__device__ __forceinline__ uint32_t wave_lower_bound(const uint64_t* a, uint32_t lo, uint32_t hi, uint64_t k) {
    const uint32_t lane = lane_id();
    while (hi - lo > kWave) {
        const uint32_t len = hi - lo;
        bool below = false;
        if (lane < kWave - 1) {
            const uint32_t s = lo + static_cast<uint32_t>((static_cast<uint64_t>(len) * (lane + 1)) >> 6);
            below = a[s] < k;
        }
        const uint32_t c = static_cast<uint32_t>(__popcll(__ballot(below)));  // probes below k form a prefix
        const uint32_t new_lo = c ? lo + static_cast<uint32_t>((static_cast<uint64_t>(len) * c) >> 6) + 1 : lo;
        const uint32_t new_hi =
            c < kWave - 1 ? lo + static_cast<uint32_t>((static_cast<uint64_t>(len) * (c + 1)) >> 6) : hi;
        lo = new_lo;
        hi = new_hi;
    }
    const bool below = lane < hi - lo && a[lo + lane] < k;
    return lo + static_cast<uint32_t>(__popcll(__ballot(below)));
}

// Dynamic tile index: blocks take tiles in launch order through an atomic
// counter, so a block waiting on tile t-1 knows t-1 is already owned by a
// running block (forward progress for the look-back).
__device__ __forceinline__ uint32_t take_tile(uint32_t* counter, uint32_t* lds_slot) {
    if (threadIdx.x == 0) *lds_slot = atomicAdd(counter, 1u);
    __syncthreads();
    uint32_t t = *lds_slot;
    __syncthreads();
    return t;
}

__device__ __forceinline__ int clz64(uint64_t v) { return v ? __clzll(static_cast<long long>(v)) : 64; }

// First index in [lo, hi) whose key is >= k (hi if none).
__device__ __forceinline__ uint64_t lower_bound_u64(const uint64_t* a, uint64_t lo, uint64_t hi, uint64_t k) {
    while (lo < hi) {
        uint64_t mid = lo + ((hi - lo) >> 1);
        if (a[mid] < k)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

}  // namespace cs
