// Host side of the C ABI declared in include/goldi.h: argument checks,
// device-range checks of every buffer, level offsets, kernel launches and
// status reporting.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <cstring>
#include <string>
#include <vector>

#include "goldi.h"
#include "kernels.hpp"

using goldi::u64;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define GOLDI_HIP(expr)                                                                        \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(GOLDI_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

bool mul_overflows(size_t a, size_t b, size_t *out) { return __builtin_mul_overflow(a, b, out); }

// Checks that [p, p + bytes) lies inside one device allocation of the
// current device, so a kernel launched on it cannot touch memory outside.
int check_device_range(const void *p, size_t bytes, const char *what) {
    if (p == nullptr) return fail(GOLDI_EINVAL, "%s is null", what);
    hipPointerAttribute_t attr;
    hipError_t e = hipPointerGetAttributes(&attr, p);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(GOLDI_EINVAL, "%s is not a device pointer (%s)", what, hipGetErrorString(e));
    }
    if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged)
        return fail(GOLDI_EINVAL, "%s is not device memory", what);
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess && attr.device != dev)
        return fail(GOLDI_EINVAL, "%s lives on device %d, current device is %d", what, attr.device, dev);
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    e = hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)p);
    if (e == hipSuccess && base != nullptr) {
        const size_t off = (size_t)((const char *)p - (const char *)base);
        if (off > size || bytes > size - off)
            return fail(GOLDI_EINVAL, "%s: %zu bytes needed but the allocation holds %zu past it", what, bytes,
                        size - (off > size ? size : off));
    } else {
        (void)hipGetLastError();  // range query unsupported for this allocation kind
    }
    return GOLDI_OK;
}

bool overlaps(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

// Per-device status word for the synchronous calls, and a lock that
// serialises them (they share the word).
struct DeviceSlot {
    std::mutex mu;
    uint32_t *status = nullptr;
};
constexpr int kMaxDevices = 64;
DeviceSlot g_slots[kMaxDevices];

int acquire_slot(int *dev_out, DeviceSlot **slot) {
    int dev = 0;
    GOLDI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GOLDI_EDEVICE, "device index %d out of range", dev);
    *dev_out = dev;
    *slot = &g_slots[dev];
    return GOLDI_OK;
}

// ------------------------------------------------------------- profiling
// While enabled, every launch is bracketed by two HIP events recorded on the
// launch stream; goldi_profile_read() sums their elapsed times per kernel.
struct ProfRecord {
    const char *name;
    hipEvent_t start, stop;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRecord> g_prof;

template <class F>
int timed_launch(const char *name, hipStream_t st, F launch) {
    bool on;
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        on = g_prof_on;
    }
    if (!on) {
        launch();
        GOLDI_HIP(hipGetLastError());
        return GOLDI_OK;
    }
    ProfRecord r{name, nullptr, nullptr};
    GOLDI_HIP(hipEventCreate(&r.start));
    GOLDI_HIP(hipEventCreate(&r.stop));
    GOLDI_HIP(hipEventRecord(r.start, st));
    launch();
    GOLDI_HIP(hipGetLastError());
    GOLDI_HIP(hipEventRecord(r.stop, st));
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof.push_back(r);
    return GOLDI_OK;
}

unsigned grid_for(size_t n) { return (unsigned)((n + goldi::BLOCK - 1) / goldi::BLOCK); }

constexpr size_t kMaxGrid = (size_t)0x7FFFFFFF * goldi::BLOCK / 4;  // quad kernels use 4 lanes per item

// ---------------------------------------------------------------- launches

int launch_permute(uint64_t *states, size_t n, uint32_t *status, hipStream_t st) {
    return timed_launch("permute", st, [&] {
        hipLaunchKernelGGL(goldi::k_permute, dim3(grid_for(n)), dim3(goldi::BLOCK), 0, st, states, n, status);
    });
}

// Launches at or below these sizes use the 4-lanes-per-state kernels, whose
// permutation latency is about a third of the one-lane kernels'.  Initial
// values come from GOLDI_QUAD_MAX_ROWS / GOLDI_QUAD_MAX_PARENTS if set;
// goldi_tune_set() changes them at run time.
size_t env_size(const char *name, size_t dflt) {
    const char *v = getenv(name);
    if (v == nullptr || *v == 0) return dflt;
    return (size_t)strtoull(v, nullptr, 0);
}
std::atomic<size_t> g_quad_max_rows{env_size("GOLDI_QUAD_MAX_ROWS", (size_t)1 << 14)};
std::atomic<size_t> g_quad_max_parents{env_size("GOLDI_QUAD_MAX_PARENTS", (size_t)1 << 16)};
size_t quad_max_rows() { return g_quad_max_rows.load(std::memory_order_relaxed); }
size_t quad_max_parents() { return g_quad_max_parents.load(std::memory_order_relaxed); }

int launch_leaf_hash(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *digests, uint32_t *status,
                     hipStream_t st) {
    if (n_rows <= quad_max_rows()) {
        return timed_launch("leaf_hash_quad", st, [&] {
            hipLaunchKernelGGL(goldi::k_leaf_hash_quad, dim3(grid_for(4 * n_rows)), dim3(goldi::BLOCK), 0, st,
                               leaves, n_rows, n_cols, digests, status);
        });
    }
    return timed_launch("leaf_hash", st, [&] {
        hipLaunchKernelGGL(goldi::k_leaf_hash, dim3(grid_for(n_rows)), dim3(goldi::BLOCK), 0, st, leaves, n_rows,
                           n_cols, digests, status);
    });
}

int launch_level(const uint64_t *child, size_t n_child, uint64_t *parent, hipStream_t st) {
    const size_t n_par = (n_child + 1) / 2;
    if (n_par <= quad_max_parents()) {
        return timed_launch("level_quad", st, [&] {
            hipLaunchKernelGGL(goldi::k_level_quad, dim3(grid_for(4 * n_par)), dim3(goldi::BLOCK), 0, st, child,
                               n_child, parent);
        });
    }
    return timed_launch("level", st, [&] {
        hipLaunchKernelGGL(goldi::k_level, dim3(grid_for(n_par)), dim3(goldi::BLOCK), 0, st, child, n_child,
                           parent);
    });
}

int launch_tree(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *nodes, uint32_t *status,
                hipStream_t st) {
    int rc = launch_leaf_hash(leaves, n_rows, n_cols, nodes, status, st);
    if (rc) return rc;
    size_t off = 0, n = n_rows;
    while (n > 1) {
        rc = launch_level(nodes + off * goldi::DIGEST, n, nodes + (off + n) * goldi::DIGEST, st);
        if (rc) return rc;
        off += n;
        n = (n + 1) / 2;
    }
    return GOLDI_OK;
}

// ------------------------------------------------------------ validation

int validate_permute(const uint64_t *states, size_t n) {
    if (n == 0) return fail(GOLDI_EINVAL, "n must be >= 1");
    size_t bytes;
    if (mul_overflows(n, goldi::WIDTH * sizeof(u64), &bytes) || n > kMaxGrid)
        return fail(GOLDI_EINVAL, "n = %zu is too large", n);
    return check_device_range(states, bytes, "states");
}

int validate_tree(const uint64_t *leaves, size_t n_rows, size_t n_cols, const uint64_t *out, size_t out_nodes,
                  const char *out_name) {
    if (n_rows == 0 || n_cols == 0) return fail(GOLDI_EINVAL, "n_rows and n_cols must be >= 1");
    size_t cells, in_bytes, out_bytes;
    if (mul_overflows(n_rows, n_cols, &cells) || mul_overflows(cells, sizeof(u64), &in_bytes) ||
        mul_overflows(out_nodes, goldi::DIGEST * sizeof(u64), &out_bytes) || n_rows > kMaxGrid)
        return fail(GOLDI_EINVAL, "shape %zu x %zu is too large", n_rows, n_cols);
    int rc = check_device_range(leaves, in_bytes, "leaves");
    if (rc) return rc;
    rc = check_device_range(out, out_bytes, out_name);
    if (rc) return rc;
    if (overlaps(leaves, in_bytes, out, out_bytes)) return fail(GOLDI_EINVAL, "%s overlaps leaves", out_name);
    return GOLDI_OK;
}

size_t num_nodes(size_t n) {
    if (n == 0) return 0;
    size_t total = n;
    while (n > 1) {
        n = (n + 1) / 2;
        total += n;
    }
    return total;
}

// Runs `enqueue(status)` on the null stream with the device's status word,
// waits, and maps the word to a return code.
template <class F>
int run_sync(F enqueue) {
    int dev;
    DeviceSlot *slot;
    int rc = acquire_slot(&dev, &slot);
    if (rc) return rc;
    std::lock_guard<std::mutex> lock(slot->mu);
    if (slot->status == nullptr) {
        void *p = nullptr;
        hipError_t e = hipMalloc(&p, 256);
        if (e != hipSuccess) return fail(GOLDI_ENOMEM, "status word: %s", hipGetErrorString(e));
        slot->status = (uint32_t *)p;
    }
    GOLDI_HIP(hipMemsetAsync(slot->status, 0, sizeof(uint32_t), 0));
    rc = enqueue(slot->status);
    if (rc) {
        (void)hipStreamSynchronize(0);
        return rc;
    }
    uint32_t h = 0;
    GOLDI_HIP(hipMemcpyAsync(&h, slot->status, sizeof h, hipMemcpyDeviceToHost, 0));
    GOLDI_HIP(hipStreamSynchronize(0));
    if (h & goldi::STATUS_NONCANON) return fail(GOLDI_ENONCANON, "an input word is >= p");
    return GOLDI_OK;
}

}  // namespace

extern "C" {

const char *goldi_strerror(int code) {
    switch (code) {
        case GOLDI_OK: return "ok";
        case GOLDI_EINVAL: return "invalid argument";
        case GOLDI_ENONCANON: return "input word not canonical (>= p)";
        case GOLDI_EDEVICE: return "HIP device error";
        case GOLDI_ENOMEM: return "device allocation failed";
        default: return "unknown status";
    }
}

const char *goldi_last_error(void) { return g_last_error.c_str(); }

size_t goldi_merkle_num_nodes(size_t n_rows) { return num_nodes(n_rows); }

int goldi_tune_set(const char *key, size_t value) {
    if (key == nullptr) return fail(GOLDI_EINVAL, "goldi_tune_set: null key");
    if (strcmp(key, "quad_max_rows") == 0) {
        g_quad_max_rows.store(value);
    } else if (strcmp(key, "quad_max_parents") == 0) {
        g_quad_max_parents.store(value);
    } else {
        return fail(GOLDI_EINVAL, "goldi_tune_set: unknown key '%s'", key);
    }
    return GOLDI_OK;
}

int goldi_tune_get(const char *key, size_t *value) {
    if (key == nullptr || value == nullptr) return fail(GOLDI_EINVAL, "goldi_tune_get: null argument");
    if (strcmp(key, "quad_max_rows") == 0) {
        *value = quad_max_rows();
    } else if (strcmp(key, "quad_max_parents") == 0) {
        *value = quad_max_parents();
    } else {
        return fail(GOLDI_EINVAL, "goldi_tune_get: unknown key '%s'", key);
    }
    return GOLDI_OK;
}

int goldi_profile_enable(int on) {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof_on = on != 0;
    return GOLDI_OK;
}

int goldi_profile_read(const char *kernel, double *total_ms, size_t *count) {
    if (kernel == nullptr || total_ms == nullptr || count == nullptr)
        return fail(GOLDI_EINVAL, "goldi_profile_read: null argument");
    std::vector<ProfRecord> mine;
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        std::vector<ProfRecord> rest;
        for (auto &r : g_prof) (std::string(r.name) == kernel ? mine : rest).push_back(r);
        g_prof.swap(rest);
    }
    double sum = 0.0;
    int rc = GOLDI_OK;
    for (auto &r : mine) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess && rc == GOLDI_OK) rc = fail(GOLDI_EDEVICE, "profile event: %s", hipGetErrorString(e));
        sum += ms;
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    *total_ms = sum;
    *count = mine.size();
    return rc;
}

int goldi_poseidon_permute_async(uint64_t *states, size_t n, uint32_t *dev_status, void *stream) {
    int rc = validate_permute(states, n);
    if (rc) return rc;
    rc = check_device_range(dev_status, sizeof(uint32_t), "dev_status");
    if (rc) return rc;
    return launch_permute(states, n, dev_status, (hipStream_t)stream);
}

int goldi_poseidon_permute(uint64_t *states, size_t n) {
    int rc = validate_permute(states, n);
    if (rc) return rc;
    return run_sync([&](uint32_t *status) { return launch_permute(states, n, status, 0); });
}

int goldi_leaf_hash_async(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *digests,
                          uint32_t *dev_status, void *stream) {
    int rc = validate_tree(leaves, n_rows, n_cols, digests, n_rows, "digests");
    if (rc) return rc;
    rc = check_device_range(dev_status, sizeof(uint32_t), "dev_status");
    if (rc) return rc;
    return launch_leaf_hash(leaves, n_rows, n_cols, digests, dev_status, (hipStream_t)stream);
}

int goldi_leaf_hash(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *digests) {
    int rc = validate_tree(leaves, n_rows, n_cols, digests, n_rows, "digests");
    if (rc) return rc;
    return run_sync([&](uint32_t *status) { return launch_leaf_hash(leaves, n_rows, n_cols, digests, status, 0); });
}

int goldi_merkle_build_async(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *nodes_out,
                             uint32_t *dev_status, void *stream) {
    int rc = validate_tree(leaves, n_rows, n_cols, nodes_out, num_nodes(n_rows), "nodes_out");
    if (rc) return rc;
    rc = check_device_range(dev_status, sizeof(uint32_t), "dev_status");
    if (rc) return rc;
    return launch_tree(leaves, n_rows, n_cols, nodes_out, dev_status, (hipStream_t)stream);
}

int goldi_merkle_build(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *nodes_out) {
    int rc = validate_tree(leaves, n_rows, n_cols, nodes_out, num_nodes(n_rows), "nodes_out");
    if (rc) return rc;
    return run_sync([&](uint32_t *status) { return launch_tree(leaves, n_rows, n_cols, nodes_out, status, 0); });
}

static int validate_many(const goldi_tree_t *trees, size_t n_trees) {
    if (trees == nullptr || n_trees == 0) return fail(GOLDI_EINVAL, "need at least one tree");
    for (size_t t = 0; t < n_trees; t++) {
        int rc = validate_tree(trees[t].leaves, trees[t].n_rows, trees[t].n_cols, trees[t].nodes_out,
                               num_nodes(trees[t].n_rows), "nodes_out");
        if (rc) return fail(rc, "tree %zu: %s", t, g_last_error.c_str());
    }
    for (size_t a = 0; a < n_trees; a++)
        for (size_t b = 0; b < n_trees; b++) {
            const size_t out_a = num_nodes(trees[a].n_rows) * goldi::DIGEST * sizeof(u64);
            if (a != b &&
                overlaps(trees[a].nodes_out, out_a, trees[b].nodes_out,
                         num_nodes(trees[b].n_rows) * goldi::DIGEST * sizeof(u64)))
                return fail(GOLDI_EINVAL, "outputs of trees %zu and %zu overlap", a, b);
            if (overlaps(trees[a].nodes_out, out_a, trees[b].leaves,
                         trees[b].n_rows * trees[b].n_cols * sizeof(u64)))
                return fail(GOLDI_EINVAL, "output of tree %zu overlaps leaves of tree %zu", a, b);
        }
    return GOLDI_OK;
}

int goldi_merkle_build_many_async(const goldi_tree_t *trees, size_t n_trees, uint32_t *dev_status, void *stream) {
    int rc = validate_many(trees, n_trees);
    if (rc) return rc;
    rc = check_device_range(dev_status, sizeof(uint32_t), "dev_status");
    if (rc) return rc;
    for (size_t t = 0; t < n_trees; t++) {
        rc = launch_tree(trees[t].leaves, trees[t].n_rows, trees[t].n_cols, trees[t].nodes_out, dev_status,
                         (hipStream_t)stream);
        if (rc) return rc;
    }
    return GOLDI_OK;
}

int goldi_merkle_build_many(const goldi_tree_t *trees, size_t n_trees) {
    int rc = validate_many(trees, n_trees);
    if (rc) return rc;
    return run_sync([&](uint32_t *status) {
        for (size_t t = 0; t < n_trees; t++) {
            int r = launch_tree(trees[t].leaves, trees[t].n_rows, trees[t].n_cols, trees[t].nodes_out, status, 0);
            if (r) return r;
        }
        return (int)GOLDI_OK;
    });
}

}  // extern "C"
