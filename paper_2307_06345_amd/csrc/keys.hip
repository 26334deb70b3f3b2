// SFC keys from FP64 coordinates (Sec. 3): quantisation to the 2^21 grid,
// Morton interleave, and Skilling's 3D Hilbert curve evaluated as a finite
// state machine over bit planes with a 2-plane lookup table held in LDS.
#include "common.hpp"
#include "hilbert.hpp"
#include "internal.hpp"

namespace cs {
namespace {

__device__ const HilbertTables d_hilbert = kHilbert;

// ---- quantisation and Morton spread --------------------------------------

__device__ __forceinline__ uint32_t quantize(double c, double lo, double s) {
    double t = (c - lo) * s;  // two IEEE roundings; built with -ffp-contract=off
    if (!(t >= 0.0)) return 0u;
    if (t >= 2097152.0) return (1u << kL) - 1u;
    return static_cast<uint32_t>(t);
}

// Spread the 21 low bits of v so bit b lands on bit 3b.
__device__ __forceinline__ uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint64_t morton_of(uint32_t ix, uint32_t iy, uint32_t iz) {
    return (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
}

// The Morton code's octal digits are the raw plane octants (x as the 4s bit),
// so the Hilbert machine consumes it 6 bits (two planes) at a time.
__device__ __forceinline__ uint64_t hilbert_from_morton(uint64_t m, const uint16_t* two, const uint16_t* first) {
    uint32_t e = first[(m >> 60) & 7u];
    uint64_t key = e & 7u;
    uint32_t state = e >> 3;
#pragma unroll
    for (int pair = 9; pair >= 0; --pair) {
        uint32_t o = static_cast<uint32_t>(m >> (6 * pair)) & 63u;
        uint32_t t = two[state * 64 + o];
        key = (key << 6) | (t & 63u);
        state = t >> 6;
    }
    return key;
}

constexpr int kKeysBlock = 256;   // batched key kernel: one tile per block
// plain key kernel: few large blocks (grid-stride), so that the blocks'
// histogram flushes (512 global atomics each, all on the same 512 counters)
// are few; 2 blocks of 1024 per CU still fill every SIMD
constexpr int kKeysBlockPlain = 1024;
constexpr size_t kKeysMaxBlocks = kKeyBlocksMax;

template <int CURVE>
__device__ __forceinline__ uint64_t key_of(double cx, double cy, double cz, double lo0, double lo1, double lo2,
                                           double s0, double s1, double s2, const uint16_t* two,
                                           const uint16_t* first) {
    const uint64_t m = morton_of(quantize(cx, lo0, s0), quantize(cy, lo1, s1), quantize(cz, lo2, s2));
    return CURVE == CSTONE_HILBERT ? hilbert_from_morton(m, two, first) : m;
}

__device__ __forceinline__ bool finite3(double a, double b, double c) {
    return __builtin_isfinite(a) && __builtin_isfinite(b) && __builtin_isfinite(c);
}

// PAIRED: every thread encodes two neighbouring particles with 16-byte loads
// and stores (all four arrays 16-byte aligned); the odd last particle, if any,
// is done by thread 0 of block 0.
template <int CURVE, bool PAIRED>
__global__ __launch_bounds__(kKeysBlockPlain) void keys_kernel(const double* __restrict__ x,
                                                          const double* __restrict__ y,
                                                          const double* __restrict__ z, size_t n, double lo0,
                                                          double lo1, double lo2, double s0, double s1, double s2,
                                                          uint64_t* __restrict__ keys, uint32_t* flags,
                                                          uint32_t* hist_parts, uint32_t hmask, uint32_t hshift,
                                                          uint32_t* bad_parts, uint32_t hdigits, uint32_t hbits) {
    __shared__ uint16_t two[kStates * 64];
    __shared__ uint16_t first[8];
    __shared__ uint32_t h[kKeyDigitsMax * 512];
    if (CURVE == CSTONE_HILBERT) {
        for (int i = threadIdx.x; i < kStates * 64; i += kKeysBlockPlain) two[i] = d_hilbert.two[i];
        if (threadIdx.x < 8) first[threadIdx.x] = d_hilbert.first[threadIdx.x];
    }
    if (hist_parts)
        for (uint32_t i = threadIdx.x; i < hdigits * 512; i += kKeysBlockPlain) h[i] = 0;
    __syncthreads();
    // counts of digit d (d < hdigits) of a key, part d of the block's row
    auto count = [&](uint64_t k) {
        for (uint32_t d = 0; d < hdigits; ++d) atomicAdd(&h[d * 512 + ((k >> (hshift + d * hbits)) & hmask)], 1u);
    };
    bool bad = false;
    const size_t stride = static_cast<size_t>(gridDim.x) * kKeysBlockPlain;
    const size_t t0 = static_cast<size_t>(blockIdx.x) * kKeysBlockPlain + threadIdx.x;
    if (PAIRED) {
        const size_t pairs = n / 2;
        const double2* x2 = reinterpret_cast<const double2*>(x);
        const double2* y2 = reinterpret_cast<const double2*>(y);
        const double2* z2 = reinterpret_cast<const double2*>(z);
        ulonglong2* k2 = reinterpret_cast<ulonglong2*>(keys);
        for (size_t p = t0; p < pairs; p += stride) {
            const double2 cx = x2[p], cy = y2[p], cz = z2[p];
            bad |= !(finite3(cx.x, cy.x, cz.x) && finite3(cx.y, cy.y, cz.y));
            ulonglong2 k;
            k.x = key_of<CURVE>(cx.x, cy.x, cz.x, lo0, lo1, lo2, s0, s1, s2, two, first);
            k.y = key_of<CURVE>(cx.y, cy.y, cz.y, lo0, lo1, lo2, s0, s1, s2, two, first);
            k2[p] = k;
            if (hist_parts) {
                count(k.x);
                count(k.y);
            }
        }
        if ((n & 1) && t0 == 0) {
            const size_t p = n - 1;
            bad |= !finite3(x[p], y[p], z[p]);
            const uint64_t k = key_of<CURVE>(x[p], y[p], z[p], lo0, lo1, lo2, s0, s1, s2, two, first);
            keys[p] = k;
            if (hist_parts) count(k);
        }
    } else {
        for (size_t p = t0; p < n; p += stride) {
            const double cx = x[p], cy = y[p], cz = z[p];
            bad |= !finite3(cx, cy, cz);
            const uint64_t k = key_of<CURVE>(cx, cy, cz, lo0, lo1, lo2, s0, s1, s2, two, first);
            keys[p] = k;
            if (hist_parts) count(k);
        }
    }
    if (flags && __ballot(bad) != 0ull && lane_id() == 0) atomicOr(flags, CSTONE_FLAG_NONFINITE);
    // per-block results are stored, not accumulated, so nothing has to be
    // cleared before this kernel
    if (bad_parts) {
        const int any = __syncthreads_or(bad ? 1 : 0);
        if (threadIdx.x == 0) bad_parts[blockIdx.x] = any ? CSTONE_FLAG_NONFINITE : 0u;
    }
    if (hist_parts) {
        __syncthreads();
        uint32_t* mine = hist_parts + static_cast<size_t>(blockIdx.x) * (kKeyDigitsMax * 512);
        for (uint32_t d = 0; d < hdigits; ++d)
            for (uint32_t i = threadIdx.x; i <= hmask; i += kKeysBlockPlain) mine[d * 512 + i] = h[d * 512 + i];
    }
}

template <int CURVE, bool PAIRED>
void launch_keys_t(size_t blocks, hipStream_t stream, const double* x, const double* y, const double* z, size_t n,
                   const cstone_box& box, const double* s, uint64_t* keys, uint32_t* flags, uint32_t* hist_parts,
                   uint32_t hmask, uint32_t hshift, uint32_t* bad_parts, uint32_t hdigits, uint32_t hbits) {
    hipLaunchKernelGGL((keys_kernel<CURVE, PAIRED>), dim3(blocks), dim3(kKeysBlockPlain), 0, stream, x, y, z, n,
                       box.lo[0], box.lo[1], box.lo[2], s[0], s[1], s[2], keys, flags, hist_parts, hmask, hshift,
                       bad_parts, hdigits, hbits);
}

// Batched keys: block b encodes tile tiles[b] = {first particle, count, -, set}
// with that set's box and curve, and counts the lowest digit into the set's
// histogram.
__global__ __launch_bounds__(kKeysBlock) void keys_batch_kernel(const double* __restrict__ x,
                                                                const double* __restrict__ y,
                                                                const double* __restrict__ z,
                                                                const uint4* __restrict__ tiles,
                                                                const BatchSet* __restrict__ sets,
                                                                uint64_t* __restrict__ keys, uint32_t* set_flags,
                                                                uint32_t* hist0, uint32_t hist_stride,
                                                                uint32_t hmask, uint32_t hshift) {
    __shared__ uint16_t two[kStates * 64];
    __shared__ uint16_t first[8];
    __shared__ uint32_t h[512];
    const uint4 t = tiles[blockIdx.x];
    const BatchSet& S = sets[t.w];
    const bool hilbert = S.curve == CSTONE_HILBERT;
    if (hilbert) {
        for (int i = threadIdx.x; i < kStates * 64; i += kKeysBlock) two[i] = d_hilbert.two[i];
        if (threadIdx.x < 8) first[threadIdx.x] = d_hilbert.first[threadIdx.x];
    }
    for (int i = threadIdx.x; i < 512; i += kKeysBlock) h[i] = 0;
    __syncthreads();
    const double lo0 = S.lo[0], lo1 = S.lo[1], lo2 = S.lo[2];
    const double s0 = S.scale[0], s1 = S.scale[1], s2 = S.scale[2];
    bool bad = false;
    const uint32_t end = t.x + t.y;
    for (uint32_t p = t.x + threadIdx.x; p < end; p += kKeysBlock) {
        const double cx = x[p], cy = y[p], cz = z[p];
        bad |= !finite3(cx, cy, cz);
        const uint64_t k = hilbert ? key_of<CSTONE_HILBERT>(cx, cy, cz, lo0, lo1, lo2, s0, s1, s2, two, first)
                                   : key_of<CSTONE_MORTON>(cx, cy, cz, lo0, lo1, lo2, s0, s1, s2, two, first);
        keys[p] = k;
        atomicAdd(&h[static_cast<uint32_t>(k >> hshift) & hmask], 1u);
    }
    if (__ballot(bad) != 0ull && lane_id() == 0) atomicOr(&set_flags[t.w], CSTONE_FLAG_NONFINITE);
    __syncthreads();
    uint32_t* hs = hist0 + static_cast<size_t>(t.w) * hist_stride;
    for (uint32_t i = threadIdx.x; i <= hmask; i += kKeysBlock)
        if (h[i]) atomicAdd(&hs[i], h[i]);
}

}  // namespace

cstone_status launch_keys_batch(const double* x, const double* y, const double* z, const uint4* tiles,
                                uint32_t n_tiles, const BatchSet* sets, uint64_t* keys, uint32_t* set_flags,
                                uint32_t* hist0, uint32_t hist_stride, uint32_t hist_mask, uint32_t hist_shift,
                                hipStream_t stream) {
    if (n_tiles == 0) return CSTONE_OK;
    if (hist_mask >= 512 || hist_shift >= 64) return CSTONE_ERR_INVALID_ARG;
    hipLaunchKernelGGL(keys_batch_kernel, dim3(n_tiles), dim3(kKeysBlock), 0, stream, x, y, z, tiles, sets, keys,
                       set_flags, hist0, hist_stride, hist_mask, hist_shift);
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

cstone_status launch_keys(const double* x, const double* y, const double* z, size_t n, const cstone_box& box,
                          cstone_curve curve, uint64_t* keys, uint32_t* flags, hipStream_t stream,
                          uint32_t* hist_parts, uint32_t hist_mask, uint32_t hist_shift, uint32_t* bad_parts,
                          uint32_t* blocks_used, uint32_t hist_digits) {
    if (blocks_used) *blocks_used = 0;
    if (n == 0) return CSTONE_OK;
    const uint32_t hist_bits = static_cast<uint32_t>(__builtin_popcount(hist_mask));
    if (hist_parts && (hist_mask >= 512 || ((hist_mask + 1) & hist_mask) != 0 || hist_digits < 1 ||
                       hist_digits > kKeyDigitsMax || hist_shift + hist_digits * hist_bits > 64))
        return CSTONE_ERR_INVALID_ARG;
    double s[3];
    for (int d = 0; d < 3; ++d) s[d] = 2097152.0 / (box.hi[d] - box.lo[d]);
    auto aligned = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; };
    const bool paired = aligned(x) && aligned(y) && aligned(z) && aligned(keys);
    const size_t per_thread = paired ? 2 : 1;
    size_t blocks = (n + kKeysBlockPlain * per_thread - 1) / (kKeysBlockPlain * per_thread);
    if (blocks > kKeysMaxBlocks) blocks = kKeysMaxBlocks;  // grid-stride beyond that
    if (blocks_used) *blocks_used = static_cast<uint32_t>(blocks);
    if (curve == CSTONE_HILBERT) {
        if (paired)
            launch_keys_t<CSTONE_HILBERT, true>(blocks, stream, x, y, z, n, box, s, keys, flags, hist_parts, hist_mask,
                                                   hist_shift, bad_parts, hist_digits, hist_bits);
        else
            launch_keys_t<CSTONE_HILBERT, false>(blocks, stream, x, y, z, n, box, s, keys, flags, hist_parts, hist_mask,
                                                   hist_shift, bad_parts, hist_digits, hist_bits);
    } else {
        if (paired)
            launch_keys_t<CSTONE_MORTON, true>(blocks, stream, x, y, z, n, box, s, keys, flags, hist_parts, hist_mask,
                                                   hist_shift, bad_parts, hist_digits, hist_bits);
        else
            launch_keys_t<CSTONE_MORTON, false>(blocks, stream, x, y, z, n, box, s, keys, flags, hist_parts, hist_mask,
                                                   hist_shift, bad_parts, hist_digits, hist_bits);
    }
    CS_HIP(hipGetLastError());
    return CSTONE_OK;
}

}  // namespace cs
