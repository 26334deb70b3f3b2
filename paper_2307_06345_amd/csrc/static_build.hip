// cstone_build_static: cstone_build with its workspace in a fixed device
// array of this library instead of a caller buffer, for callers that cannot
// allocate device memory. It calls no allocator: the array is part of the
// library's code object on every device that runs it, and its address is
// looked up once per device.
#include <mutex>

#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

constexpr size_t kStaticScratchBytes = size_t{64} << 20;  // CSTONE_STATIC_SCRATCH_BYTES
static_assert(kStaticScratchBytes == CSTONE_STATIC_SCRATCH_BYTES, "the header states the same size");

// Workspace of cstone_build_static. In host code this name is a host-side
// stand-in, not a device address: only the address from hipGetSymbolAddress
// may be handed to kernels or copies.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call there). NULL if it cannot be found.
void* scratch_on_current_device() {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_scratch[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

}  // namespace
}  // namespace cs

extern "C" {

CSTONE_API cstone_status cstone_build_static(const double* x, const double* y, const double* z, size_t n,
                                             const cstone_box* box, cstone_curve curve, uint32_t n_crit,
                                             uint64_t* sorted_keys, uint32_t* perm, uint64_t* leaves,
                                             size_t* n_leaves, size_t leaf_capacity, uint32_t* counts,
                                             uint64_t* node_keys, uint32_t* child, uint32_t* level_offsets,
                                             uint32_t max_iters, uint32_t* iters_done, hipStream_t stream) {
    if (cstone_build_workspace_bytes(n, leaf_capacity) > cs::kStaticScratchBytes) return CSTONE_ERR_INVALID_ARG;
    void* ws = cs::scratch_on_current_device();
    if (!ws) return CSTONE_ERR_DEVICE;
    // every stage clears the parts of its workspace it relies on, so the
    // previous call's contents need no clearing here
    return cstone_build(x, y, z, n, box, curve, n_crit, sorted_keys, perm, leaves, n_leaves, leaf_capacity, counts,
                        node_keys, child, level_offsets, max_iters, iters_done, ws, cs::kStaticScratchBytes, nullptr,
                        stream);
}

}  // extern "C"
