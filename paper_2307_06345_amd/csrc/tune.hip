// Autotune table of the sort shapes: which compiled shape (digit width, block
// size, keys per thread) a sort of a given size class runs on a given device.
//
// Entries are keyed by (kernel, size class, device): the kernel is the plain
// particle-key sort (cstone_sort, cstone_build) or the segmented sort of a
// batch; the size class is floor(log2(n)) of the keys sorted; the device is
// its architecture name and compute-unit count. The autotuners record into the
// table; every sort looks its shape up once, at its start, and falls back to
// the built-in shape when no entry matches. The table can be written to and
// read from a JSON file, one entry per line.
#include <cinttypes>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "internal.hpp"

namespace cs {
namespace {

struct TuneEntry {
    int kernel;
    int size_class;
    std::string device;
    int variant;
};

std::mutex g_mu;
std::vector<TuneEntry> g_entries;
std::vector<std::string> g_device_names;  // per device index, filled on first use

const char* kKernelNames[kTuneKernels] = {"sort", "batch_sort"};

int size_class_of(size_t n) {
    int c = 0;
    while (n > 1) {
        n >>= 1;
        ++c;
    }
    return c;
}

// "<arch>/<compute units>cu" of the current device (cached; g_mu held).
std::string current_device_locked() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return "unknown";
    if (static_cast<size_t>(dev) >= g_device_names.size()) g_device_names.resize(dev + 1);
    std::string& name = g_device_names[dev];
    if (name.empty()) {
        hipDeviceProp_t prop;
        if (hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
        std::string arch(prop.gcnArchName);
        const size_t colon = arch.find(':');  // drop feature suffixes such as ":sramecc+:xnack-"
        if (colon != std::string::npos) arch.resize(colon);
        name = arch + "/" + std::to_string(prop.multiProcessorCount) + "cu";
    }
    return name;
}

TuneEntry* find_locked(int kernel, int size_class, const std::string& device) {
    for (auto& e : g_entries)
        if (e.kernel == kernel && e.size_class == size_class && e.device == device) return &e;
    return nullptr;
}

void set_locked(int kernel, int size_class, const std::string& device, int variant) {
    if (TuneEntry* e = find_locked(kernel, size_class, device))
        e->variant = variant;
    else
        g_entries.push_back({kernel, size_class, device, variant});
}

}  // namespace

int tune_lookup(int kernel, size_t n) {
    if (kernel < 0 || kernel >= kTuneKernels) return -1;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_entries.empty()) return -1;
    const TuneEntry* e = find_locked(kernel, size_class_of(n), current_device_locked());
    return e && e->variant >= 0 && e->variant < sort_variant_count() ? e->variant : -1;
}

void tune_record(int kernel, size_t n, int variant) {
    if (kernel < 0 || kernel >= kTuneKernels || variant < 0 || variant >= sort_variant_count()) return;
    std::lock_guard<std::mutex> lock(g_mu);
    set_locked(kernel, size_class_of(n), current_device_locked(), variant);
}

int sort_resolve_variant(size_t n) {
    const int v = tune_lookup(kTuneSort, n);
    return v >= 0 ? v : sort_builtin_variant();
}

}  // namespace cs

extern "C" {

CSTONE_API void cstone_tune_clear(void) {
    std::lock_guard<std::mutex> lock(cs::g_mu);
    cs::g_entries.clear();
}

CSTONE_API size_t cstone_tune_entries(void) {
    std::lock_guard<std::mutex> lock(cs::g_mu);
    return cs::g_entries.size();
}

CSTONE_API cstone_status cstone_tune_set(int kernel, size_t n, int variant) {
    if (kernel < 0 || kernel >= cs::kTuneKernels || variant < -1 || variant >= cs::sort_variant_count())
        return CSTONE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(cs::g_mu);
    const std::string dev = cs::current_device_locked();
    if (variant >= 0) {
        cs::set_locked(kernel, cs::size_class_of(n), dev, variant);
    } else {  // -1: drop the entry
        const int c = cs::size_class_of(n);
        for (size_t i = 0; i < cs::g_entries.size(); ++i)
            if (cs::g_entries[i].kernel == kernel && cs::g_entries[i].size_class == c && cs::g_entries[i].device == dev) {
                cs::g_entries.erase(cs::g_entries.begin() + static_cast<std::ptrdiff_t>(i));
                break;
            }
    }
    return CSTONE_OK;
}

CSTONE_API int cstone_tune_get(int kernel, size_t n) { return cs::tune_lookup(kernel, n); }

CSTONE_API cstone_status cstone_tune_save(const char* path) {
    if (!path) return CSTONE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(cs::g_mu);
    FILE* f = std::fopen(path, "w");
    if (!f) return CSTONE_ERR_INVALID_ARG;
    std::fprintf(f, "{\"format\": \"cstone-tune-2\", \"entries\": [\n");
    for (size_t i = 0; i < cs::g_entries.size(); ++i) {
        const auto& e = cs::g_entries[i];
        const cs::SortVariantInfo v = cs::sort_variant_info(e.variant);
        std::fprintf(f,
                     "{\"kernel\": \"%s\", \"size_log2\": %d, \"device\": \"%s\", \"variant\": %d, "
                     "\"digit_bits\": %d, \"block\": %d, \"items\": %d, \"split\": %d}%s\n",
                     cs::kKernelNames[e.kernel], e.size_class, e.device.c_str(), e.variant, v.bits, v.block, v.items,
                     v.split, i + 1 < cs::g_entries.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    return ok ? CSTONE_OK : CSTONE_ERR_INVALID_ARG;
}

CSTONE_API cstone_status cstone_tune_load(const char* path) {
    if (!path) return CSTONE_ERR_INVALID_ARG;
    FILE* f = std::fopen(path, "r");
    if (!f) return CSTONE_ERR_INVALID_ARG;
    std::vector<cs::TuneEntry> read;
    char line[512];
    bool ok = true, header = false;
    while (std::fgets(line, sizeof line, f)) {
        if (std::strncmp(line, "{\"format\": \"cstone-tune-2\"", 26) == 0) {
            header = true;
            continue;
        }
        if (line[0] == ']' || line[0] == '\n') continue;
        char kernel[32], device[128];
        int size_class = 0, variant = 0, bits = 0, block = 0, items = 0, split = 0;
        if (std::sscanf(line,
                        "{\"kernel\": \"%31[^\"]\", \"size_log2\": %d, \"device\": \"%127[^\"]\", \"variant\": %d, "
                        "\"digit_bits\": %d, \"block\": %d, \"items\": %d, \"split\": %d}",
                        kernel, &size_class, device, &variant, &bits, &block, &items, &split) != 8) {
            ok = false;
            break;
        }
        int k = -1;
        for (int i = 0; i < cs::kTuneKernels; ++i)
            if (std::strcmp(kernel, cs::kKernelNames[i]) == 0) k = i;
        // a shape that this library does not have under that index is skipped
        if (k < 0 || variant < 0 || variant >= cs::sort_variant_count()) continue;
        const cs::SortVariantInfo v = cs::sort_variant_info(variant);
        if (v.bits != bits || v.block != block || v.items != items || v.split != split) continue;
        read.push_back({k, size_class, device, variant});
    }
    std::fclose(f);
    if (!ok || !header) return CSTONE_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(cs::g_mu);
    for (const auto& e : read) cs::set_locked(e.kernel, e.size_class, e.device, e.variant);
    return CSTONE_OK;
}

}  // extern "C"
