// Host side of the C ABI declared in include/goldi.h: argument checks,
// device-range checks of every buffer, level offsets, kernel launches and
// status reporting.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "goldi.h"
#include "goldi_internal.hpp"
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
// While enabled, launches are timed with HIP events recorded on the launch
// stream; goldi_profile_read() sums the elapsed times per kernel kind.  A run
// of consecutive launches of one kind on one stream within one library call
// (the five largest tree levels, say) is timed as one span: two event records
// per run rather than per launch, so the timing disturbs the work less.  The
// span covers the launches and the gaps between them.  It is closed by the
// next launch of another kind or stream, and at the end of the library call.
struct ProfRecord {
    const char *name;
    hipEvent_t start, stop;
    size_t launches;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::string g_prof_only;  // empty: every kernel kind
std::vector<ProfRecord> g_prof;

struct OpenSpan {
    const char *name = nullptr;  // null: no span open
    hipStream_t st = nullptr;
    ProfRecord r{};
};
thread_local OpenSpan t_span;

void span_drop() {
    if (t_span.r.start) (void)hipEventDestroy(t_span.r.start);
    if (t_span.r.stop) (void)hipEventDestroy(t_span.r.stop);
    t_span = OpenSpan{};
}

int span_close() {
    if (t_span.name == nullptr) return GOLDI_OK;
    hipError_t e = hipEventRecord(t_span.r.stop, t_span.st);
    if (e != hipSuccess) {
        span_drop();
        return fail(GOLDI_EDEVICE, "hipEventRecord: %s", hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        g_prof.push_back(t_span.r);
    }
    t_span = OpenSpan{};
    return GOLDI_OK;
}

// Closes the calling thread's open span when a library call returns.
struct SpanScope {
    ~SpanScope() { (void)span_close(); }
};

template <class F>
int timed_launch(const char *name, hipStream_t st, F launch) {
    bool on;
    {
        std::lock_guard<std::mutex> lock(g_prof_mu);
        on = g_prof_on && (g_prof_only.empty() || g_prof_only == name);
    }
    if (on) {  // no event records inside a stream capture
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) on = false;
        (void)hipGetLastError();
    }
    if (t_span.name != nullptr && (!on || strcmp(t_span.name, name) != 0 || t_span.st != st)) {
        if (int rc = span_close()) return rc;
    }
    if (!on) {
        launch();
        GOLDI_HIP(hipGetLastError());
        return GOLDI_OK;
    }
    if (t_span.name == nullptr) {
        t_span.r = ProfRecord{name, nullptr, nullptr, 0};
        // No system-scope release at the records: the events only time device work.
        hipError_t e = hipEventCreateWithFlags(&t_span.r.start, hipEventDisableSystemFence);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&t_span.r.stop, hipEventDisableSystemFence);
        if (e == hipSuccess) e = hipEventRecord(t_span.r.start, st);
        if (e != hipSuccess) {
            span_drop();
            return fail(GOLDI_EDEVICE, "profiling event: %s", hipGetErrorString(e));
        }
        t_span.name = name;
        t_span.st = st;
    }
    launch();
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        span_drop();
        return fail(GOLDI_EDEVICE, "kernel launch: %s", hipGetErrorString(e));
    }
    t_span.r.launches++;
    return GOLDI_OK;
}

// One dispatch covers at most 2^32 - 1 work-items (the dispatch packet's
// grid size is 32-bit), so a launch beyond that is refused, never truncated.
constexpr size_t kMaxThreads = 0xFFFFFFFFull - (goldi::BLOCK - 1);

int blocks_for(size_t items, size_t lanes, unsigned *blocks) {
    size_t threads;
    if (mul_overflows(items, lanes, &threads) || threads > kMaxThreads)
        return fail(GOLDI_EINVAL, "a launch of %zu items x %zu lanes exceeds one dispatch (2^32 - 1 work-items)",
                    items, lanes);
    *blocks = (unsigned)((threads + goldi::BLOCK - 1) / goldi::BLOCK);
    return GOLDI_OK;
}

// ---------------------------------------------------------------- launches

int launch_permute(uint64_t *states, size_t n, uint32_t *status, hipStream_t st) {
    unsigned g;
    if (int rc = blocks_for(n, 1, &g)) return rc;
    return timed_launch("permute", st, [&] {
        hipLaunchKernelGGL(goldi::k_permute, dim3(g), dim3(goldi::BLOCK), 0, st, states, n, status);
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
// Batched builds: 1 = one launch per step across all trees (default), 0 = the
// plain per-tree schedule.  Graphs: 1 = capture the batched launch sequence
// into a hipGraph cached per batch description and replay it.
std::atomic<size_t> g_batch_mode{env_size("GOLDI_BATCH_MODE", 1)};
std::atomic<size_t> g_graph_mode{env_size("GOLDI_GRAPH_MODE", 0)};
// At or below these sizes the one-word-per-lane kernels run instead (lower
// latency still, more instructions in total).
std::atomic<size_t> g_l12_max_rows{env_size("GOLDI_LANE12_MAX_ROWS", (size_t)1 << 13)};
std::atomic<size_t> g_l12_max_parents{env_size("GOLDI_LANE12_MAX_PARENTS", (size_t)1 << 13)};
// Single-tree builds finish in one single-workgroup launch (k_levels_lane12)
// from the first level of at most this many parents (<= 64; the default 16
// keeps one wave per SIMD of the workgroup's CU); 0 disables.
std::atomic<size_t> g_top_max_parents{env_size("GOLDI_TOP_MAX_PARENTS", 16)};
size_t top_max_parents() { return g_top_max_parents.load(std::memory_order_relaxed); }
size_t l12_max_rows() { return g_l12_max_rows.load(std::memory_order_relaxed); }
size_t l12_max_parents() { return g_l12_max_parents.load(std::memory_order_relaxed); }
size_t quad_max_rows() { return g_quad_max_rows.load(std::memory_order_relaxed); }
size_t quad_max_parents() { return g_quad_max_parents.load(std::memory_order_relaxed); }

// Rows 0 .. n_rows-1 of a column-major leaf matrix whose columns are ld words
// apart (ld = n_rows for a whole matrix, larger for a range of its rows).
int launch_leaf_hash(const uint64_t *leaves, size_t n_rows, size_t ld, size_t n_cols, uint64_t *digests,
                     uint32_t *status, hipStream_t st) {
    unsigned g;
    if (n_rows <= l12_max_rows()) {
        if (int rc = blocks_for(n_rows, 16, &g)) return rc;
        return timed_launch("leaf_hash_lane12", st, [&] {
            hipLaunchKernelGGL(goldi::k_leaf_hash_lane12, dim3(g), dim3(goldi::BLOCK), 0, st, leaves, n_rows, ld,
                               n_cols, digests, status);
        });
    }
    if (n_rows <= quad_max_rows()) {
        if (int rc = blocks_for(n_rows, 4, &g)) return rc;
        return timed_launch("leaf_hash_quad", st, [&] {
            hipLaunchKernelGGL(goldi::k_leaf_hash_quad, dim3(g), dim3(goldi::BLOCK), 0, st, leaves, n_rows, ld,
                               n_cols, digests, status);
        });
    }
    if (int rc = blocks_for(n_rows, 1, &g)) return rc;
    return timed_launch("leaf_hash", st, [&] {
        if (n_cols <= goldi::RATE)
            hipLaunchKernelGGL(goldi::k_leaf_hash<true>, dim3(g), dim3(goldi::BLOCK), 0, st, leaves, n_rows, ld,
                               n_cols, digests, status);
        else
            hipLaunchKernelGGL(goldi::k_leaf_hash<false>, dim3(g), dim3(goldi::BLOCK), 0, st, leaves, n_rows, ld,
                               n_cols, digests, status);
    });
}

// One level, one lane (or four) per state; the one-word-per-lane layout runs
// several levels per launch instead (launch_levels_lane12).  The layout
// follows `width_par` parents (default: this launch's own), so that the
// ranges of a split level take the layout of the whole level.
int launch_level(const uint64_t *child, size_t n_child, uint64_t *parent, hipStream_t st, size_t width_par = 0) {
    const size_t n_par = (n_child + 1) / 2;
    unsigned g;
    if ((width_par ? width_par : n_par) <= quad_max_parents()) {
        if (int rc = blocks_for(n_par, 4, &g)) return rc;
        return timed_launch("level_quad", st, [&] {
            hipLaunchKernelGGL(goldi::k_level_quad, dim3(g), dim3(goldi::BLOCK), 0, st, child, n_child, parent);
        });
    }
    if (int rc = blocks_for(n_par, 1, &g)) return rc;
    return timed_launch("level", st, [&] {
        hipLaunchKernelGGL(goldi::k_level, dim3(g), dim3(goldi::BLOCK), 0, st, child, n_child, parent);
    });
}

// Levels of one word per lane: from the level at `off` (n nodes wide), its
// nodes [c0, c1), through `levels` <= kLevelsPerLaunch levels in one launch
// of 256-thread blocks (32 nodes per block: c0, and c1 unless it is n, must
// be multiples of 2^levels).
constexpr int kLevelsPerLaunch = 5;
int launch_levels_lane12(uint64_t *nodes, size_t off, size_t n, size_t c0, size_t c1, int levels, hipStream_t st) {
    unsigned g;
    if (int rc = blocks_for((c1 - c0 + 1) / 2, 16, &g)) return rc;
    return timed_launch("levels_lane12", st, [&] {
        hipLaunchKernelGGL(goldi::k_levels_lane12, dim3(g), dim3(goldi::BLOCK), 0, st, nodes, off, n, c0, c1, levels);
    });
}

// Every level from the one at `off` (n nodes, at most 2 TOP_STATES) to the
// root in one single-workgroup launch, sized to the first level's parents.
int launch_top(uint64_t *nodes, size_t off, size_t n, hipStream_t st) {
    const unsigned threads = (unsigned)(64 * (((n + 1) / 2 + 3) / 4));  // whole waves of 4 states
    return timed_launch("top_lane12", st, [&] {
        hipLaunchKernelGGL(goldi::k_levels_lane12, dim3(1), dim3(threads), 0, st, nodes, off, n, (size_t)0, n,
                           64);
    });
}

// Levels above `off`, `n` nodes wide, up to the root, on one stream.
int launch_upper(uint64_t *nodes, size_t off, size_t n, hipStream_t st) {
    while (n > 1) {
        const size_t n_par = (n + 1) / 2;
        if (n_par <= top_max_parents()) return launch_top(nodes, off, n, st);
        if (n_par <= l12_max_parents()) {
            if (int rc = launch_levels_lane12(nodes, off, n, 0, n, kLevelsPerLaunch, st)) return rc;
            for (int k = 0; k < kLevelsPerLaunch && n > 1; k++) {
                off += n;
                n = (n + 1) / 2;
            }
            continue;
        }
        if (int rc = launch_level(nodes + off * goldi::DIGEST, n, nodes + (off + n) * goldi::DIGEST, st)) return rc;
        off += n;
        n = (n + 1) / 2;
    }
    return GOLDI_OK;
}

// ---------------------------------------------------------- split builds
// A single tree's leaf hash and every level with more parents than the join
// width (default 16: all but the tree-top launch) run as `parts` ranges of
// rows, each on its own stream, and the streams join on the caller's stream
// before the rest.  Two effects, both measured on the 2^22 x 8 tree (2.97 ->
// 2.89 ms with two parts): each launch ends with a drain in which the SIMDs
// hold fewer and fewer waves, and the other stream's launch fills them; and
// a latency-bound level (a few thousand parents or fewer) costs about one
// permutation latency whatever its width, so two half-width launches side by
// side take the time of one.  Three and four parts, and unequal halves (the
// caller's part 1/64 .. 1/256 larger or smaller), measured slower.  Part k covers leaves [b_k, b_(k+1)); every boundary is a
// multiple of 2^depth, so at each of the first `depth` levels part k's nodes
// are [b_k >> L, b_(k+1) >> L) of level L and every part but the last has an
// even number of children.  The nodes written are the same as an unsplit
// build's, byte for byte.
std::atomic<size_t> g_split_parts{env_size("GOLDI_SPLIT_PARTS", 2)};
// Set while the calling thread runs a call that must not split (the
// allocation-free entry point).
thread_local bool t_no_split = false;
struct NoSplitScope {
    bool old = t_no_split;
    NoSplitScope() { t_no_split = true; }
    ~NoSplitScope() { t_no_split = old; }
};
std::atomic<size_t> g_split_min_rows{env_size("GOLDI_SPLIT_MIN_ROWS", (size_t)1 << 20)};
std::atomic<size_t> g_split_join_parents{env_size("GOLDI_SPLIT_JOIN_PARENTS", 4096)};
constexpr size_t kMaxSplit = 4;

// Library-owned streams (default priority, non-blocking) for parts 1.., one
// set per device, created on first use and kept for the process's life.
struct AuxStreams {
    std::mutex mu;
    hipStream_t s[kMaxSplit - 1] = {};
    std::vector<hipEvent_t> free_events;  // fork/join events, reusable once their waits are enqueued
};
AuxStreams g_aux[kMaxDevices];

int aux_setup(int dev, size_t parts, hipStream_t *streams, hipEvent_t *events, size_t n_events) {
    AuxStreams &a = g_aux[dev];
    std::lock_guard<std::mutex> lock(a.mu);
    for (size_t k = 0; k + 1 < parts; k++) {
        if (a.s[k] == nullptr) GOLDI_HIP(hipStreamCreateWithFlags(&a.s[k], hipStreamNonBlocking));
        streams[k] = a.s[k];
    }
    for (size_t i = 0; i < n_events; i++) {
        if (a.free_events.empty()) {
            GOLDI_HIP(hipEventCreateWithFlags(&events[i], hipEventDisableTiming));
        } else {
            events[i] = a.free_events.back();
            a.free_events.pop_back();
        }
    }
    return GOLDI_OK;
}

void aux_release(int dev, const hipEvent_t *events, size_t n_events) {
    AuxStreams &a = g_aux[dev];
    std::lock_guard<std::mutex> lock(a.mu);
    for (size_t i = 0; i < n_events; i++)
        if (events[i]) a.free_events.push_back(events[i]);
}

// Number of leading levels that run split: those with more parents than the
// join width (and than the tree-top launch takes).
size_t split_levels(size_t n) {
    const size_t cut = std::max(g_split_join_parents.load(), top_max_parents());
    size_t depth = 0;
    while ((n + 1) / 2 > cut) {
        depth++;
        n = (n + 1) / 2;
    }
    return depth;
}

int launch_split(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *nodes, uint32_t *status,
                 hipStream_t st, size_t parts, size_t depth) {
    int dev = 0;
    GOLDI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GOLDI_EDEVICE, "device index %d out of range", dev);
    hipStream_t aux[kMaxSplit - 1] = {};
    hipEvent_t ev[kMaxSplit] = {};  // ev[0]: fork; ev[k]: join of part k
    if (int rc = aux_setup(dev, parts, aux, ev, parts)) return rc;
    const size_t unit = (size_t)1 << depth;
    size_t b[kMaxSplit + 1];
    b[0] = 0;
    for (size_t k = 1; k < parts; k++) b[k] = (k * n_rows / parts + unit - 1) / unit * unit;
    b[parts] = n_rows;
    int rc = GOLDI_OK;
    hipError_t e = hipEventRecord(ev[0], st);
    for (size_t k = 1; k < parts && e == hipSuccess; k++) e = hipStreamWaitEvent(aux[k - 1], ev[0], 0);
    if (e != hipSuccess) rc = fail(GOLDI_EDEVICE, "split fork: %s", hipGetErrorString(e));
    size_t off_end = 0, n_end = n_rows;  // level `depth`: offset and width
    for (size_t k = 0; k < parts && rc == GOLDI_OK; k++) {
        hipStream_t sk = k == 0 ? st : aux[k - 1];
        rc = launch_leaf_hash(leaves + b[k], b[k + 1] - b[k], n_rows, n_cols, nodes + b[k] * goldi::DIGEST, status,
                              sk);
        size_t off = 0, n = n_rows;
        for (size_t L = 0; L < depth && rc == GOLDI_OK;) {
            const size_t c0 = b[k] >> L, c1 = k + 1 < parts ? b[k + 1] >> L : n;
            // Every layout choice follows the whole level's width: the parts'
            // launches run side by side and share the GPU like one launch.
            size_t done = 1;
            if ((n + 1) / 2 <= l12_max_parents()) {
                done = std::min((size_t)kLevelsPerLaunch, depth - L);  // c0, c1: multiples of 2^(depth - L)
                rc = launch_levels_lane12(nodes, off, n, c0, c1, (int)done, sk);
            } else {
                rc = launch_level(nodes + (off + c0) * goldi::DIGEST, c1 - c0,
                                  nodes + (off + n + c0 / 2) * goldi::DIGEST, sk, (n + 1) / 2);
            }
            for (size_t j = 0; j < done; j++, L++) {
                off += n;
                n = (n + 1) / 2;
            }
        }
        off_end = off;
        n_end = n;
    }
    // Join even after a failed launch, so that nothing of this call runs
    // behind the caller's stream.
    for (size_t k = 1; k < parts; k++) {
        e = hipEventRecord(ev[k], aux[k - 1]);
        if (e == hipSuccess) e = hipStreamWaitEvent(st, ev[k], 0);
        if (e != hipSuccess && rc == GOLDI_OK) rc = fail(GOLDI_EDEVICE, "split join: %s", hipGetErrorString(e));
    }
    aux_release(dev, ev, parts);
    if (rc) return rc;
    return launch_upper(nodes, off_end, n_end, st);
}

int launch_tree(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *nodes, uint32_t *status,
                hipStream_t st) {
    const size_t parts = std::min(g_split_parts.load(), kMaxSplit);
    if (parts >= 2 && n_rows >= g_split_min_rows.load() && !t_no_split) {
        const size_t depth = split_levels(n_rows);
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        const bool capturing = hipStreamIsCapturing(st, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone;
        (void)hipGetLastError();
        // Every part needs at least 2^depth rows; a captured sequence stays on one stream.
        if (!capturing && depth >= 1 && n_rows / parts >= ((size_t)1 << depth))
            return launch_split(leaves, n_rows, n_cols, nodes, status, st, parts, depth);
    }
    if (int rc = launch_leaf_hash(leaves, n_rows, n_rows, n_cols, nodes, status, st)) return rc;
    return launch_upper(nodes, 0, n_rows, st);
}

// ------------------------------------------------------- batched builds

size_t chunks_of(size_t n_cols) { return (n_cols + goldi::RATE - 1) / goldi::RATE; }

// Where tree t of a many-tree call reports a non-canonical word: base + t *
// stride (stride 0: one word shared by every tree).
struct StatusMap {
    uint32_t *base;
    size_t stride;
    uint32_t *of(size_t t) const { return base + t * stride; }
};

// Launches one step of a batch: fills block_begin from per-tree item counts
// (lanes_per_item = 1, 4 or 16) and launches `kernel`.
template <class K>
int launch_batch(const char *name, K kernel, goldi::Batch &b, const size_t *items, int lanes_per_item,
                 hipStream_t st) {
    size_t blocks = 0;
    for (uint32_t t = 0; t < b.n_trees; t++) {
        unsigned g;
        if (int rc = blocks_for(items[t], lanes_per_item, &g)) return rc;
        b.block_begin[t] = (uint32_t)blocks;
        blocks += g;
        if (blocks * goldi::BLOCK > kMaxThreads)
            return fail(GOLDI_EINVAL, "batched launch '%s' exceeds one dispatch (2^32 - 1 work-items)", name);
    }
    b.block_begin[b.n_trees] = (uint32_t)blocks;
    if (blocks == 0) return GOLDI_OK;
    return timed_launch(name, st, [&] {
        hipLaunchKernelGGL(kernel, dim3((unsigned)blocks), dim3(goldi::BLOCK), 0, st, b);
    });
}

// All trees of `order` (indices into trees, at most MAX_BATCH), one launch
// per step: the leaves of every tree, then level 1 of every tree that has
// one, and so on.  Trees are ordered by per-row cost, heaviest first, so the
// longest blocks are dispatched first.  Tree t reports into status.of(t).
int launch_group(const goldi_tree_t *trees, const std::vector<size_t> &order, StatusMap status, hipStream_t st) {
    const uint32_t nt = (uint32_t)order.size();
    goldi::Batch b;
    memset(&b, 0, sizeof b);
    b.n_trees = nt;
    size_t items[goldi::MAX_BATCH];
    size_t total = 0, max_cols = 0;
    for (uint32_t k = 0; k < nt; k++) {
        const goldi_tree_t &T = trees[order[k]];
        b.t[k] = {T.leaves, T.nodes_out, status.of(order[k]), (uint32_t)T.n_rows, (uint32_t)T.n_cols};
        items[k] = T.n_rows;
        total += T.n_rows;
        max_cols = std::max(max_cols, T.n_cols);
    }
    int rc = total <= l12_max_rows()
                 ? launch_batch("leaf_hash_lane12", goldi::k_leaf_hash_lane12_batch, b, items, 16, st)
             : total <= quad_max_rows()
                 ? launch_batch("leaf_hash_quad", goldi::k_leaf_hash_quad_batch, b, items, 4, st)
                 : max_cols <= goldi::RATE
                 ? launch_batch("leaf_hash", goldi::k_leaf_hash_batch<true>, b, items, 1, st)
                 : launch_batch("leaf_hash", goldi::k_leaf_hash_batch<false>, b, items, 1, st);
    if (rc) return rc;
    // Level loop: off[k] = first node of the current child level of tree k.
    std::vector<size_t> off(nt, 0), n(nt);
    for (uint32_t k = 0; k < nt; k++) n[k] = trees[order[k]].n_rows;
    for (;;) {
        goldi::Batch lb;
        memset(&lb, 0, sizeof lb);
        size_t parents = 0;
        uint32_t m = 0;
        for (uint32_t k = 0; k < nt; k++) {
            if (n[k] <= 1) continue;
            u64 *nodes = trees[order[k]].nodes_out;
            lb.t[m] = {nodes + off[k] * goldi::DIGEST, nodes + (off[k] + n[k]) * goldi::DIGEST, nullptr,
                       (uint32_t)n[k], 0};
            items[m] = (n[k] + 1) / 2;
            parents += items[m];
            m++;
        }
        if (m == 0) break;
        lb.n_trees = m;
        rc = parents <= l12_max_parents()
                 ? launch_batch("level_lane12", goldi::k_level_lane12_batch, lb, items, 16, st)
             : parents <= quad_max_parents()
                 ? launch_batch("level_quad", goldi::k_level_quad_batch, lb, items, 4, st)
                 : launch_batch("level", goldi::k_level_batch, lb, items, 1, st);
        if (rc) return rc;
        for (uint32_t k = 0; k < nt; k++) {
            if (n[k] <= 1) continue;
            off[k] += n[k];
            n[k] = (n[k] + 1) / 2;
        }
    }
    return GOLDI_OK;
}

int launch_many(const goldi_tree_t *trees, size_t n_trees, StatusMap status, hipStream_t st) {
    if (g_batch_mode.load() == 0) {
        for (size_t t = 0; t < n_trees; t++) {
            int rc = launch_tree(trees[t].leaves, trees[t].n_rows, trees[t].n_cols, trees[t].nodes_out,
                                 status.of(t), st);
            if (rc) return rc;
        }
        return GOLDI_OK;
    }
    // Trees too large for 32-bit batch descriptors take the plain path.
    std::vector<size_t> order;
    for (size_t t = 0; t < n_trees; t++) {
        if (trees[t].n_rows > 0xFFFFFFFFull || trees[t].n_cols > 0xFFFFFFFFull) {
            int rc = launch_tree(trees[t].leaves, trees[t].n_rows, trees[t].n_cols, trees[t].nodes_out,
                                 status.of(t), st);
            if (rc) return rc;
        } else {
            order.push_back(t);
        }
    }
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        const size_t ca = chunks_of(trees[a].n_cols), cb = chunks_of(trees[b].n_cols);
        return ca != cb ? ca > cb : trees[a].n_rows > trees[b].n_rows;
    });
    for (size_t g = 0; g < order.size(); g += goldi::MAX_BATCH) {
        std::vector<size_t> grp(order.begin() + g, order.begin() + std::min(order.size(), g + goldi::MAX_BATCH));
        int rc = launch_group(trees, grp, status, st);
        if (rc) return rc;
    }
    return GOLDI_OK;
}

// Graph cache: the launch sequence of a batch, captured once per distinct
// (device, status word, knobs, tree descriptors) and replayed afterwards.
struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::vector<GraphEntry> g_graphs;  // most recently used last
constexpr size_t kGraphCacheMax = 16;
hipStream_t g_capture_stream[kMaxDevices] = {};

int launch_many_graph(int dev, const goldi_tree_t *trees, size_t n_trees, StatusMap status, hipStream_t st) {
    std::vector<uint64_t> key = {(uint64_t)dev,      (uint64_t)(uintptr_t)status.base, status.stride,
                                 quad_max_rows(),    quad_max_parents(),               l12_max_rows(),
                                 l12_max_parents(),  top_max_parents(),                g_batch_mode.load()};
    for (size_t t = 0; t < n_trees; t++) {
        key.push_back((uint64_t)(uintptr_t)trees[t].leaves);
        key.push_back(trees[t].n_rows);
        key.push_back(trees[t].n_cols);
        key.push_back((uint64_t)(uintptr_t)trees[t].nodes_out);
    }
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (size_t i = 0; i < g_graphs.size(); i++) {
        if (g_graphs[i].key == key) {
            GraphEntry e = g_graphs[i];
            g_graphs.erase(g_graphs.begin() + i);
            g_graphs.push_back(e);
            GOLDI_HIP(hipGraphLaunch(e.exec, st));
            return GOLDI_OK;
        }
    }
    if (g_capture_stream[dev] == nullptr) GOLDI_HIP(hipStreamCreateWithFlags(&g_capture_stream[dev], hipStreamNonBlocking));
    hipStream_t cs = g_capture_stream[dev];
    GOLDI_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    int rc = launch_many(trees, n_trees, status, cs);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(GOLDI_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(GOLDI_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    if (g_graphs.size() >= kGraphCacheMax) {
        (void)hipGraphExecDestroy(g_graphs.front().exec);
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back({key, exec});
    GOLDI_HIP(hipGraphLaunch(exec, st));
    return GOLDI_OK;
}

int enqueue_many(const goldi_tree_t *trees, size_t n_trees, StatusMap status, hipStream_t st) {
    if (g_graph_mode.load() != 0 && g_batch_mode.load() != 0) {
        int dev = 0;
        GOLDI_HIP(hipGetDevice(&dev));
        if (dev < 0 || dev >= kMaxDevices) return fail(GOLDI_EDEVICE, "device index %d out of range", dev);
        return launch_many_graph(dev, trees, n_trees, status, st);
    }
    return launch_many(trees, n_trees, status, st);
}

// ------------------------------------------------------------ validation

int validate_permute(const uint64_t *states, size_t n) {
    if (n == 0) return fail(GOLDI_EINVAL, "n must be >= 1");
    size_t bytes;
    if (mul_overflows(n, goldi::WIDTH * sizeof(u64), &bytes) || n > kMaxThreads)
        return fail(GOLDI_EINVAL, "n = %zu is too large", n);
    return check_device_range(states, bytes, "states");
}

int validate_tree(const uint64_t *leaves, size_t n_rows, size_t n_cols, const uint64_t *out, size_t out_nodes,
                  const char *out_name) {
    if (n_rows == 0 || n_cols == 0) return fail(GOLDI_EINVAL, "n_rows and n_cols must be >= 1");
    size_t cells, in_bytes, out_bytes;
    if (mul_overflows(n_rows, n_cols, &cells) || mul_overflows(cells, sizeof(u64), &in_bytes) ||
        mul_overflows(out_nodes, goldi::DIGEST * sizeof(u64), &out_bytes) || n_rows > kMaxThreads)
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
    if (rc == GOLDI_OK) rc = span_close();
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

// ------------------------------------------------ allocation-free builds
// The per-tree status words of goldi_merkle_build_many_noalloc live in this
// file-scope device array instead of memory the library allocates.  Each GPU
// holds its own copy at its own address; host code never uses the array's
// name (a host-side stand-in), only the address hipGetSymbolAddress returns
// on that device.
constexpr size_t kNoallocMaxTrees = 4096;
static __device__ __align__(256) uint32_t scratch[kNoallocMaxTrees];

struct NoallocSlot {
    std::mutex mu;            // serialises the calls on one device
    uint32_t *ptr = nullptr;  // device address of `scratch` on that device
};
NoallocSlot g_noalloc[kMaxDevices];

// Clears n words (a kernel rather than a memset node, so that a captured
// launch sequence replays correctly).
__global__ void k_zero_words(uint32_t *p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

}  // namespace

int goldi_internal_enqueue_many(const goldi_tree_t *trees, size_t n_trees, uint32_t *dev_status_per_tree,
                                hipStream_t stream) {
    SpanScope span_scope;
    return launch_many(trees, n_trees, StatusMap{dev_status_per_tree, 1}, stream);
}

int goldi_internal_check_device_range(const void *p, size_t bytes, const char *what) {
    return check_device_range(p, bytes, what);
}

extern "C" {

const char *goldi_strerror(int code) {
    switch (code) {
        case GOLDI_OK: return "ok";
        case GOLDI_EINVAL: return "invalid argument";
        case GOLDI_ENONCANON: return "input word not canonical (>= p)";
        case GOLDI_EDEVICE: return "HIP device error";
        case GOLDI_ENOMEM: return "device allocation failed";
        case GOLDI_ECANCELED: return "request cancelled (server destroyed while it was queued)";
        case GOLDI_ETIMEDOUT: return "request timed out (watchdog)";
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
    } else if (strcmp(key, "lane12_max_rows") == 0) {
        g_l12_max_rows.store(value);
    } else if (strcmp(key, "lane12_max_parents") == 0) {
        g_l12_max_parents.store(value);
    } else if (strcmp(key, "top_max_parents") == 0) {
        if (value > (size_t)goldi::TOP_STATES)
            return fail(GOLDI_EINVAL, "top_max_parents must be at most %d", goldi::TOP_STATES);
        g_top_max_parents.store(value);
    } else if (strcmp(key, "split_parts") == 0) {
        if (value > kMaxSplit) return fail(GOLDI_EINVAL, "split_parts must be at most %zu", kMaxSplit);
        g_split_parts.store(value);
    } else if (strcmp(key, "split_min_rows") == 0) {
        g_split_min_rows.store(value);
    } else if (strcmp(key, "split_join_parents") == 0) {
        g_split_join_parents.store(value);
    } else if (strcmp(key, "batch_mode") == 0) {
        if (value > 1) return fail(GOLDI_EINVAL, "batch_mode must be 0 or 1");
        g_batch_mode.store(value);
    } else if (strcmp(key, "graph") == 0) {
        if (value > 1) return fail(GOLDI_EINVAL, "graph must be 0 or 1");
        g_graph_mode.store(value);
    } else if (strcmp(key, "partial_form") == 0 || strcmp(key, "mds_limb_bits") == 0) {
        return fail(GOLDI_EINVAL, "%s is fixed when the library is compiled", key);
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
    } else if (strcmp(key, "lane12_max_rows") == 0) {
        *value = l12_max_rows();
    } else if (strcmp(key, "lane12_max_parents") == 0) {
        *value = l12_max_parents();
    } else if (strcmp(key, "top_max_parents") == 0) {
        *value = top_max_parents();
    } else if (strcmp(key, "split_parts") == 0) {
        *value = g_split_parts.load();
    } else if (strcmp(key, "split_min_rows") == 0) {
        *value = g_split_min_rows.load();
    } else if (strcmp(key, "split_join_parents") == 0) {
        *value = g_split_join_parents.load();
    } else if (strcmp(key, "batch_mode") == 0) {
        *value = g_batch_mode.load();
    } else if (strcmp(key, "graph") == 0) {
        *value = g_graph_mode.load();
    } else if (strcmp(key, "partial_form") == 0) {
        *value = GOLDI_USE_BLOCKS ? 2 : GOLDI_USE_SPARSE ? 1 : 0;
    } else if (strcmp(key, "mds_limb_bits") == 0) {
        *value = GOLDI_MDS_LIMB24 ? 22 : 32;
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

int goldi_profile_select(const char *kernel) {
    std::lock_guard<std::mutex> lock(g_prof_mu);
    g_prof_only = kernel ? kernel : "";
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
    size_t launches = 0;
    int rc = GOLDI_OK;
    for (auto &r : mine) {
        launches += r.launches;
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.stop);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.start, r.stop);
        if (e != hipSuccess && rc == GOLDI_OK) rc = fail(GOLDI_EDEVICE, "profile event: %s", hipGetErrorString(e));
        sum += ms;
        (void)hipEventDestroy(r.start);
        (void)hipEventDestroy(r.stop);
    }
    *total_ms = sum;
    *count = launches;
    return rc;
}

int goldi_poseidon_permute_async(uint64_t *states, size_t n, uint32_t *dev_status, void *stream) {
    SpanScope span_scope;
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
    SpanScope span_scope;
    int rc = validate_tree(leaves, n_rows, n_cols, digests, n_rows, "digests");
    if (rc) return rc;
    rc = check_device_range(dev_status, sizeof(uint32_t), "dev_status");
    if (rc) return rc;
    return launch_leaf_hash(leaves, n_rows, n_rows, n_cols, digests, dev_status, (hipStream_t)stream);
}

int goldi_leaf_hash(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *digests) {
    int rc = validate_tree(leaves, n_rows, n_cols, digests, n_rows, "digests");
    if (rc) return rc;
    return run_sync(
        [&](uint32_t *status) { return launch_leaf_hash(leaves, n_rows, n_rows, n_cols, digests, status, 0); });
}

int goldi_merkle_build_async(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *nodes_out,
                             uint32_t *dev_status, void *stream) {
    SpanScope span_scope;
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
    SpanScope span_scope;
    int rc = validate_many(trees, n_trees);
    if (rc) return rc;
    rc = check_device_range(dev_status, sizeof(uint32_t), "dev_status");
    if (rc) return rc;
    return enqueue_many(trees, n_trees, StatusMap{dev_status, 0}, (hipStream_t)stream);
}

int goldi_merkle_build_many_status_async(const goldi_tree_t *trees, size_t n_trees, uint32_t *dev_status,
                                         void *stream) {
    SpanScope span_scope;
    int rc = validate_many(trees, n_trees);
    if (rc) return rc;
    size_t bytes;
    if (mul_overflows(n_trees, sizeof(uint32_t), &bytes)) return fail(GOLDI_EINVAL, "n_trees is too large");
    rc = check_device_range(dev_status, bytes, "dev_status");
    if (rc) return rc;
    return enqueue_many(trees, n_trees, StatusMap{dev_status, 1}, (hipStream_t)stream);
}

int goldi_merkle_build_many(const goldi_tree_t *trees, size_t n_trees) {
    int rc = validate_many(trees, n_trees);
    if (rc) return rc;
    return run_sync([&](uint32_t *status) { return enqueue_many(trees, n_trees, StatusMap{status, 0}, 0); });
}

int goldi_merkle_build_many_noalloc(const goldi_tree_t *trees, size_t n_trees, int *tree_status, void *stream) {
    if (n_trees > kNoallocMaxTrees)
        return fail(GOLDI_EINVAL, "goldi_merkle_build_many_noalloc: %zu trees, at most %zu (its status array is fixed)",
                    n_trees, kNoallocMaxTrees);
    int rc = validate_many(trees, n_trees);
    if (rc) return rc;
    int dev = 0;
    GOLDI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(GOLDI_EDEVICE, "device index %d out of range", dev);
    NoallocSlot &slot = g_noalloc[dev];
    std::lock_guard<std::mutex> lock(slot.mu);
    if (slot.ptr == nullptr) {  // first call on this device, which is current
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr)
            return fail(GOLDI_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        slot.ptr = (uint32_t *)p;
    }
    hipStream_t st = (hipStream_t)stream;
    const unsigned zero_blocks = (unsigned)((n_trees + 255) / 256);
    hipLaunchKernelGGL(k_zero_words, dim3(zero_blocks), dim3(256), 0, st, slot.ptr, n_trees);
    GOLDI_HIP(hipGetLastError());
    // Launched directly (never through the graph cache, which instantiates graphs).
    {
        NoSplitScope no_split;  // a split would create the library's stream and events on first use
        rc = launch_many(trees, n_trees, StatusMap{slot.ptr, 1}, st);
    }
    if (rc == GOLDI_OK) rc = span_close();
    if (rc) {
        (void)hipStreamSynchronize(st);
        return rc;
    }
    uint32_t words[kNoallocMaxTrees];
    GOLDI_HIP(hipMemcpyAsync(words, slot.ptr, n_trees * sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    GOLDI_HIP(hipStreamSynchronize(st));
    bool bad = false;
    for (size_t t = 0; t < n_trees; t++) {
        const bool b = (words[t] & goldi::STATUS_NONCANON) != 0;
        if (tree_status) tree_status[t] = b ? GOLDI_ENONCANON : GOLDI_OK;
        bad |= b;
    }
    return bad ? fail(GOLDI_ENONCANON, "an input word is >= p") : GOLDI_OK;
}

}  // extern "C"
