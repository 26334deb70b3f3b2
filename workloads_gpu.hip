// Seeded synthetic particle coordinates drawn on the GPU: input data for the
// tests and the benchmark (the serving workload needs billions of particles,
// too many to draw on the host). Not part of the octree build.
//
// Random numbers: Philox4x32-10 (J. Salmon, M. Moraes, R. Dror, D. Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), key = (seed, set
// stream), counter = (particle index low word, high word, draw, 0). A particle
// takes two counter blocks: draw 0 gives its first two uniforms, draw 1 the
// third. A uniform is (64 bits >> 11) * 2^-53, an exact double in [0, 1).
//
// Recipes (the same as the host generator's):
//   kind 0, uniform cube: x, y, z = u0, u1, u2 in [0, 1)^3;
//   kind 1, Plummer sphere (scale radius 1, truncated at r_t = 20): radius from
//   the inverse cumulative mass r = (X^(-2/3) - 1)^(-1/2) with X = u0 * M(r_t),
//   M(r) = r^3 / (1 + r^2)^(3/2); direction cos(theta) = 2 u1 - 1, phi = 2 pi u2.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#define WL_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;  // round multipliers
constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;  // key increments
constexpr int kMaxSets = 32;                              // sets per launch (kernel arguments)

struct Set {
    uint64_t offset;
    uint64_t n;
    uint32_t kind;
    uint32_t seed;
    uint32_t stream;
    uint32_t pad;
};

struct Sets {
    Set s[kMaxSets];
    uint32_t count;
};

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t lo0 = kM0 * c.x, hi0 = __umulhi(kM0, c.x);
        const uint32_t lo1 = kM1 * c.z, hi1 = __umulhi(kM1, c.z);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += kW0;
        k1 += kW1;
    }
    return c;
}

__device__ __forceinline__ double unit(uint32_t lo, uint32_t hi) {
    return static_cast<double>(((static_cast<uint64_t>(hi) << 32) | lo) >> 11) * 0x1p-53;
}

__global__ __launch_bounds__(256) void generate_kernel(Sets sets, uint64_t total, double* __restrict__ x,
                                                       double* __restrict__ y, double* __restrict__ z) {
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
        // set of the t-th particle of this launch (sets are back to back);
        // unrolled selects keep the argument block out of scratch memory
        uint64_t before = 0, acc = 0, offset = 0;
        uint32_t kind = 0, seed = 0, sid = 0;
#pragma unroll
        for (int k = 0; k < kMaxSets; ++k) {
            if (static_cast<uint32_t>(k) < sets.count && t >= acc) {
                before = acc;
                offset = sets.s[k].offset;
                kind = sets.s[k].kind;
                seed = sets.s[k].seed;
                sid = sets.s[k].stream;
            }
            acc += static_cast<uint32_t>(k) < sets.count ? sets.s[k].n : 0;
        }
        const uint64_t i = t - before;
        const uint32_t ilo = static_cast<uint32_t>(i), ihi = static_cast<uint32_t>(i >> 32);
        const uint4 a = philox4x32_10(make_uint4(ilo, ihi, 0u, 0u), seed, sid);
        const uint4 b = philox4x32_10(make_uint4(ilo, ihi, 1u, 0u), seed, sid);
        const double u0 = unit(a.x, a.y), u1 = unit(a.z, a.w), u2 = unit(b.x, b.y);
        double px, py, pz;
        if (kind == 0) {
            px = u0;
            py = u1;
            pz = u2;
        } else {
            const double rt = 20.0;
            const double x_max = rt * rt * rt / pow(1.0 + rt * rt, 1.5);
            const double X = fmax(u0 * x_max, 1e-300);
            const double r = 1.0 / sqrt(pow(X, -2.0 / 3.0) - 1.0);
            const double cos_t = 2.0 * u1 - 1.0;
            const double sin_t = sqrt(fmax(0.0, 1.0 - cos_t * cos_t));
            const double phi = 2.0 * M_PI * u2;
            px = r * sin_t * cos(phi);
            py = r * sin_t * sin(phi);
            pz = r * cos_t;
        }
        const uint64_t o = offset + i;
        x[o] = px;
        y[o] = py;
        z[o] = pz;
    }
}

// Cumulative Gaussian displacement: every coordinate moves by sigma * N(0, 1),
// the normals drawn by the Box-Muller transform from two Philox blocks
// (counter (i, 2) and (i, 3)) under key (seed, stream).
__global__ __launch_bounds__(256) void displace_kernel(uint64_t n, double sigma, uint32_t seed, uint32_t stream,
                                                       double* __restrict__ x, double* __restrict__ y,
                                                       double* __restrict__ z) {
    const uint64_t step = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += step) {
        const uint32_t ilo = static_cast<uint32_t>(i), ihi = static_cast<uint32_t>(i >> 32);
        const uint4 a = philox4x32_10(make_uint4(ilo, ihi, 2u, 0u), seed, stream);
        const uint4 b = philox4x32_10(make_uint4(ilo, ihi, 3u, 0u), seed, stream);
        // 1 - u lies in (0, 1], so the logarithm is finite
        const double r0 = sqrt(-2.0 * log(1.0 - unit(a.x, a.y)));
        const double t0 = 2.0 * M_PI * unit(a.z, a.w);
        const double r1 = sqrt(-2.0 * log(1.0 - unit(b.x, b.y)));
        const double t1 = 2.0 * M_PI * unit(b.z, b.w);
        x[i] += sigma * (r0 * cos(t0));
        y[i] += sigma * (r0 * sin(t0));
        z[i] += sigma * (r1 * cos(t1));
    }
}

// Philox4x32-10 blocks for known-answer checks: out[4 i ..] = philox(ctr[4 i ..], key).
__global__ void philox_kernel(const uint32_t* ctr, uint32_t n, uint32_t k0, uint32_t k1, uint32_t* out) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 c = philox4x32_10(make_uint4(ctr[4 * i], ctr[4 * i + 1], ctr[4 * i + 2], ctr[4 * i + 3]), k0, k1);
    out[4 * i] = c.x;
    out[4 * i + 1] = c.y;
    out[4 * i + 2] = c.z;
    out[4 * i + 3] = c.w;
}

}  // namespace

// Draw sets[k] (n particles of `kind` 0 uniform / 1 Plummer, keyed by seed and
// stream) into x, y, z (device) at [offset, offset + n). Asynchronous on
// `stream`; returns 0, or 1 for an invalid argument or a launch error.
WL_API int wl_generate(const uint64_t* offsets, const uint64_t* counts, const uint32_t* kinds, const uint32_t* seeds,
                       const uint32_t* streams, uint32_t n_sets, double* x, double* y, double* z,
                       hipStream_t stream) {
    if (n_sets && (!offsets || !counts || !kinds || !seeds || !streams || !x || !y || !z)) return 1;
    for (uint32_t base = 0; base < n_sets; base += kMaxSets) {
        Sets s{};
        uint64_t total = 0;
        s.count = n_sets - base < static_cast<uint32_t>(kMaxSets) ? n_sets - base : kMaxSets;
        for (uint32_t k = 0; k < s.count; ++k) {
            const uint32_t j = base + k;
            if (kinds[j] > 1) return 1;
            s.s[k] = {offsets[j], counts[j], kinds[j], seeds[j], streams[j], 0};
            total += counts[j];
        }
        if (total == 0) continue;
        uint64_t blocks = (total + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL(generate_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, stream, s, total, x,
                           y, z);
        if (hipGetLastError() != hipSuccess) return 1;
    }
    return 0;
}

// Move n particles (device x, y, z) by independent N(0, sigma^2) offsets keyed by (seed, stream).
WL_API int wl_displace(double* x, double* y, double* z, uint64_t n, double sigma, uint32_t seed, uint32_t stream,
                       hipStream_t hs) {
    if (n == 0) return 0;
    if (!x || !y || !z) return 1;
    uint64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(displace_kernel, dim3(static_cast<uint32_t>(blocks)), dim3(256), 0, hs, n, sigma, seed, stream,
                       x, y, z);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}

WL_API int wl_philox(const uint32_t* ctr_dev, uint32_t n, uint32_t k0, uint32_t k1, uint32_t* out_dev,
                     hipStream_t stream) {
    if (n == 0) return 0;
    if (!ctr_dev || !out_dev) return 1;
    hipLaunchKernelGGL(philox_kernel, dim3((n + 255) / 256), dim3(256), 0, stream, ctr_dev, n, k0, k1, out_dev);
    return hipGetLastError() == hipSuccess ? 0 : 1;
}
