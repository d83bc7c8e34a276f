// Serving loop: continuous batching of Merkle-build requests on one GPU.
//
// Requests (a leaf matrix in host or device memory) are queued by
// goldi_server_submit.  A scheduler thread admits waiting requests whenever
// a slot (a HIP stream with its own status words and completion event) is
// free and the device bytes of all admitted requests stay within the HBM
// budget; requests admitted together form one batched build
// (goldi_merkle_build_many's schedule), each with a status word of its own.
// Several slots run at once, so requests that arrive while others are on the
// GPU overlap with them on the device.  Each request's input copy (when it
// comes from the host) and its nodes live in device memory taken from the
// stream-ordered allocator; the root comes back to the host; the nodes stay
// on the device until the request is released.
//
// Failures stay with the request that caused them: a non-canonical word marks
// only its own request; a batch that fails on the host side is taken apart
// and each request is built again alone; a batch that overruns the watchdog
// time is reported GOLDI_ETIMEDOUT while its memory is kept until the device
// work really ends.
#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "goldi.h"
#include "goldi_internal.hpp"

namespace {

constexpr unsigned kMaxGroup = 64;  // status words and root slots per slot

int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

struct Slot;

struct Request {
    uint64_t id = 0;
    const uint64_t *leaves_host = nullptr;
    const uint64_t *leaves_dev = nullptr;
    size_t n_rows = 0, n_cols = 0;
    size_t node_bytes = 0;           // device bytes of all nodes
    size_t in_bytes = 0;             // device bytes of the server's input copy (host inputs only)
    size_t held = 0;                 // bytes of this request counted against the budget now
    uint64_t *in_dev = nullptr;      // server copy of host leaves
    uint64_t *nodes_dev = nullptr;   // all nodes, server-owned
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
    int status = GOLDI_OK;
    bool done = false;
    bool solo = false;               // rebuild in a batch of its own (its batch failed)
    bool released = false;           // released while its batch still ran: freed when it ends
    Slot *running = nullptr;         // slot whose device work still uses this request's memory
    uint64_t root[4] = {0, 0, 0, 0};
    int group = 0;                   // requests built in the same batch
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint32_t *status_dev = nullptr;   // kMaxGroup words, one per request of the batch
    uint32_t *status_host = nullptr;  // pinned copy
    uint64_t *roots_host = nullptr;   // pinned, 4 words per request of the batch
    std::vector<Request *> reqs;
    bool busy = false;
    bool timed_out = false;           // its requests were reported GOLDI_ETIMEDOUT
    int64_t t_launch = 0;
};

}  // namespace

struct goldi_server {
    int device = 0;
    size_t budget = 0, inflight_bytes = 0, max_group = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> pending;
    std::unordered_map<uint64_t, Request *> reqs;
    uint64_t next_id = 1;
    bool stop = false;
    std::thread th;
    std::string error;
    size_t admitted = 0, groups = 0, peak_bytes = 0;
    int64_t watchdog_ns = 30ll * 1000 * 1000 * 1000;
    uint64_t fail_next_batches = 0;
};

namespace {

void drop_bytes(goldi_server *s, Request *r, size_t bytes) {
    r->held -= bytes;
    s->inflight_bytes -= bytes;
}

// Frees a request's device memory on `st` and takes all of it off the budget.
void free_request_memory(goldi_server *s, Request *r, hipStream_t st) {
    if (r->in_dev) (void)hipFreeAsync(r->in_dev, st);
    if (r->nodes_dev) (void)hipFreeAsync(r->nodes_dev, st);
    r->in_dev = nullptr;
    r->nodes_dev = nullptr;
    drop_bytes(s, r, r->held);
}

void finish(Request *r, int status, int64_t t) {
    r->status = status;
    r->done = true;
    r->t_done = t;
}

// Finishes every slot whose event has completed, and applies the watchdog to
// the others.  Called with s->mu held.
void reap(goldi_server *s) {
    const int64_t t = now_ns();
    for (auto &sl : s->slots) {
        if (!sl.busy) continue;
        hipError_t e = hipEventQuery(sl.done);
        if (e == hipErrorNotReady) {
            if (!sl.timed_out && s->watchdog_ns > 0 && t - sl.t_launch > s->watchdog_ns) {
                sl.timed_out = true;
                for (Request *r : sl.reqs)
                    if (!r->done) finish(r, GOLDI_ETIMEDOUT, t);
            }
            continue;
        }
        const bool dev_ok = e == hipSuccess;
        if (!dev_ok) (void)hipGetLastError();
        for (size_t k = 0; k < sl.reqs.size(); k++) {
            Request *r = sl.reqs[k];
            r->running = nullptr;
            if (r->in_dev) {
                (void)hipFreeAsync(r->in_dev, sl.stream);
                r->in_dev = nullptr;
                drop_bytes(s, r, r->in_bytes);
            }
            if (!r->done) {
                if (!dev_ok) {
                    finish(r, GOLDI_EDEVICE, t);
                } else if (sl.status_host[k] & 1u) {
                    finish(r, GOLDI_ENONCANON, t);
                } else {
                    memcpy(r->root, sl.roots_host + 4 * k, sizeof r->root);
                    finish(r, GOLDI_OK, t);
                }
            }
            if (r->released) {  // released by the client after a watchdog report
                free_request_memory(s, r, sl.stream);
                delete r;
            }
        }
        sl.reqs.clear();
        sl.busy = false;
        sl.timed_out = false;
    }
}

// A batch failed before it was launched: each of its requests is queued again
// at the head (in order) to be built alone; a request that was already alone
// fails.  Called with s->mu held, after the batch's memory was freed.
void requeue_alone(goldi_server *s, std::vector<Request *> &batch, int status) {
    const int64_t t = now_ns();
    for (size_t k = batch.size(); k-- > 0;) {
        Request *r = batch[k];
        r->running = nullptr;
        if (r->solo || batch.size() == 1) {
            finish(r, status, t);
        } else {
            r->solo = true;
            s->pending.push_front(r);
        }
    }
    batch.clear();
}

// Enqueues the batch of slot `sl` (its requests already admitted).  Returns
// false if any step failed; nothing of the batch is then left running.
bool launch_batch(goldi_server *s, Slot &sl) {
    hipStream_t st = sl.stream;
    const size_t take = sl.reqs.size();
    std::vector<goldi_tree_t> trees;
    bool ok = true;
    for (Request *r : sl.reqs) {
        if (hipMallocAsync((void **)&r->nodes_dev, r->node_bytes, st) != hipSuccess) {
            r->nodes_dev = nullptr;
            ok = false;
            break;
        }
        const uint64_t *src = r->leaves_dev;
        if (r->leaves_host) {
            if (hipMallocAsync((void **)&r->in_dev, r->in_bytes, st) != hipSuccess) {
                r->in_dev = nullptr;
                ok = false;
                break;
            }
            if (hipMemcpyAsync(r->in_dev, r->leaves_host, r->in_bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
                ok = false;
                break;
            }
            src = r->in_dev;
        }
        trees.push_back({src, r->n_rows, r->n_cols, r->nodes_dev});
    }
    if (ok) ok = hipMemsetAsync(sl.status_dev, 0, take * sizeof(uint32_t), st) == hipSuccess;
    if (ok) ok = goldi_internal_enqueue_many(trees.data(), trees.size(), sl.status_dev, st) == GOLDI_OK;
    for (size_t k = 0; ok && k < take; k++) {
        Request *r = sl.reqs[k];
        const size_t root_off = (goldi_merkle_num_nodes(r->n_rows) - 1) * 4;
        ok = hipMemcpyAsync(sl.roots_host + 4 * k, r->nodes_dev + root_off, 32, hipMemcpyDeviceToHost, st) ==
             hipSuccess;
    }
    if (ok)
        ok = hipMemcpyAsync(sl.status_host, sl.status_dev, take * sizeof(uint32_t), hipMemcpyDeviceToHost, st) ==
             hipSuccess;
    if (ok) ok = hipEventRecord(sl.done, st) == hipSuccess;
    if (!ok) {
        s->error = hipGetErrorString(hipGetLastError());
        (void)hipStreamSynchronize(st);
        for (Request *r : sl.reqs) free_request_memory(s, r, st);
    }
    return ok;
}

// Admits waiting requests into free slots.  Called with s->mu held.
void admit(goldi_server *s) {
    for (auto &sl : s->slots) {
        if (sl.busy || s->pending.empty()) continue;
        std::vector<size_t> bytes;
        for (auto *r : s->pending) bytes.push_back(r->node_bytes + r->in_bytes);
        size_t take = 0;
        goldi_admission_plan(bytes.data(), bytes.size(), s->budget, s->inflight_bytes, s->max_group, &take);
        if (take == 0) return;  // the head does not fit yet: wait for memory (FIFO, no overtaking)
        if (s->pending.front()->solo) take = 1;
        const int64_t t = now_ns();
        for (size_t k = 0; k < take; k++) {
            Request *r = s->pending.front();
            if (k > 0 && r->solo) break;  // a request to rebuild alone starts its own batch
            s->pending.pop_front();
            r->t_admit = t;
            r->held = r->node_bytes + r->in_bytes;
            s->inflight_bytes += r->held;
            r->running = &sl;
            sl.reqs.push_back(r);
        }
        take = sl.reqs.size();
        for (Request *r : sl.reqs) r->group = (int)take;
        s->peak_bytes = s->inflight_bytes > s->peak_bytes ? s->inflight_bytes : s->peak_bytes;
        s->admitted += take;
        s->groups += 1;
        bool ok;
        if (take >= 2 && s->fail_next_batches > 0) {  // injected failure: nothing was enqueued
            s->fail_next_batches--;
            for (Request *r : sl.reqs) drop_bytes(s, r, r->held);
            ok = false;
        } else {
            ok = launch_batch(s, sl);
        }
        if (!ok) {
            requeue_alone(s, sl.reqs, GOLDI_EDEVICE);
            continue;
        }
        sl.t_launch = now_ns();
        sl.busy = true;
    }
}

void scheduler(goldi_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lock(s->mu);
    while (true) {
        reap(s);
        if (s->stop) {  // queued requests are cancelled; admitted batches finish
            const int64_t t = now_ns();
            for (Request *r : s->pending) finish(r, GOLDI_ECANCELED, t);
            s->pending.clear();
        } else {
            admit(s);
        }
        s->cv_done.notify_all();
        bool busy = false;
        for (auto &sl : s->slots) busy |= sl.busy;
        if (s->stop && !busy) break;
        // Poll completions every 20 us while work is in flight; otherwise
        // sleep until a submission arrives.
        if (busy)
            s->cv_work.wait_for(lock, std::chrono::microseconds(20));
        else
            s->cv_work.wait_for(lock, std::chrono::milliseconds(5));
    }
}

}  // namespace

extern "C" {

int goldi_admission_plan(const size_t *pending_bytes, size_t n_pending, size_t budget, size_t inflight_bytes,
                         size_t max_group, size_t *take) {
    if (take == nullptr || (n_pending > 0 && pending_bytes == nullptr)) return GOLDI_EINVAL;
    size_t used = inflight_bytes, k = 0;
    while (k < n_pending && k < max_group && used <= budget && pending_bytes[k] <= budget - used) {
        used += pending_bytes[k];
        k++;
    }
    *take = k;
    return GOLDI_OK;
}

int goldi_server_create(size_t hbm_budget_bytes, unsigned n_slots, unsigned max_group, goldi_server **out) {
    if (out == nullptr || n_slots == 0 || n_slots > 64 || max_group == 0 || max_group > kMaxGroup ||
        hbm_budget_bytes == 0)
        return GOLDI_EINVAL;
    goldi_server *s = new goldi_server();
    s->budget = hbm_budget_bytes;
    s->max_group = max_group;
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return GOLDI_EDEVICE;
    }
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, s->device) == hipSuccess) {
        uint64_t keep = UINT64_MAX;  // keep freed blocks for reuse instead of returning them to the OS
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    s->slots.resize(n_slots);
    for (auto &sl : s->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipMalloc((void **)&sl.status_dev, kMaxGroup * sizeof(uint32_t)) != hipSuccess ||
            hipHostMalloc((void **)&sl.status_host, kMaxGroup * sizeof(uint32_t), 0) != hipSuccess ||
            hipHostMalloc((void **)&sl.roots_host, kMaxGroup * 4 * sizeof(uint64_t), 0) != hipSuccess) {
            goldi_server_destroy(s);
            return GOLDI_EDEVICE;
        }
    }
    s->th = std::thread(scheduler, s);
    *out = s;
    return GOLDI_OK;
}

int goldi_server_set(goldi_server *s, const char *key, uint64_t value) {
    if (s == nullptr || key == nullptr) return GOLDI_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    if (strcmp(key, "watchdog_us") == 0) {
        if (value > (uint64_t)INT64_MAX / 1000) return GOLDI_EINVAL;
        s->watchdog_ns = (int64_t)value * 1000;
    } else if (strcmp(key, "fail_next_batches") == 0) {
        s->fail_next_batches = value;
    } else {
        return GOLDI_EINVAL;
    }
    return GOLDI_OK;
}

int goldi_server_submit(goldi_server *s, const uint64_t *leaves_host, const uint64_t *leaves_dev, size_t n_rows,
                        size_t n_cols, uint64_t *request_id) {
    if (s == nullptr || request_id == nullptr || n_rows == 0 || n_cols == 0 || n_rows > 0xFFFFFFFFull ||
        n_cols > 0xFFFFFFFFull || ((leaves_host == nullptr) == (leaves_dev == nullptr)))
        return GOLDI_EINVAL;
    size_t cells;
    if (__builtin_mul_overflow(n_rows, n_cols, &cells) || cells > (SIZE_MAX / 16)) return GOLDI_EINVAL;
    if (leaves_dev != nullptr) {
        int rc = goldi_internal_check_device_range(leaves_dev, cells * sizeof(uint64_t), "leaves");
        if (rc) return rc;
    }
    Request *r = new Request();
    r->leaves_host = leaves_host;
    r->leaves_dev = leaves_dev;
    r->n_rows = n_rows;
    r->n_cols = n_cols;
    r->node_bytes = goldi_merkle_num_nodes(n_rows) * 4 * sizeof(uint64_t);
    r->in_bytes = leaves_host != nullptr ? cells * sizeof(uint64_t) : 0;
    if (r->node_bytes + r->in_bytes > s->budget) {
        delete r;
        return GOLDI_ENOMEM;
    }
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> lock(s->mu);
        if (s->stop) {
            delete r;
            return GOLDI_EINVAL;
        }
        r->id = s->next_id++;
        s->reqs[r->id] = r;
        s->pending.push_back(r);
        *request_id = r->id;
    }
    s->cv_work.notify_one();
    return GOLDI_OK;
}

int goldi_server_wait(goldi_server *s, uint64_t id, goldi_request_info *info) {
    if (s == nullptr || info == nullptr) return GOLDI_EINVAL;
    std::unique_lock<std::mutex> lock(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end()) return GOLDI_EINVAL;
    Request *r = it->second;
    s->cv_done.wait(lock, [&] { return r->done; });
    info->status = r->status;
    info->n_rows = r->n_rows;
    info->n_cols = r->n_cols;
    info->nodes = r->status == GOLDI_OK ? r->nodes_dev : nullptr;
    info->t_submit_ns = r->t_submit;
    info->t_admit_ns = r->t_admit;
    info->t_done_ns = r->t_done;
    info->group_size = r->group;
    memcpy(info->root, r->root, sizeof r->root);
    return GOLDI_OK;
}

int goldi_server_read_nodes(goldi_server *s, uint64_t id, uint64_t *dst, size_t dst_words) {
    if (s == nullptr || dst == nullptr) return GOLDI_EINVAL;
    uint64_t *src;
    size_t words;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        auto it = s->reqs.find(id);
        if (it == s->reqs.end() || !it->second->done || it->second->status != GOLDI_OK) return GOLDI_EINVAL;
        src = it->second->nodes_dev;
        words = goldi_merkle_num_nodes(it->second->n_rows) * 4;
    }
    if (dst_words < words) return GOLDI_EINVAL;
    return hipMemcpy(dst, src, words * sizeof(uint64_t), hipMemcpyDefault) == hipSuccess ? GOLDI_OK : GOLDI_EDEVICE;
}

int goldi_server_release(goldi_server *s, uint64_t id) {
    if (s == nullptr) return GOLDI_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || !it->second->done) return GOLDI_EINVAL;
    Request *r = it->second;
    s->reqs.erase(it);
    if (r->running) {  // reported by the watchdog, still on the device: freed when its batch ends
        r->released = true;
    } else {
        free_request_memory(s, r, s->slots[0].stream);
        delete r;
    }
    s->cv_work.notify_one();
    return GOLDI_OK;
}

int goldi_server_stats(goldi_server *s, size_t *admitted, size_t *groups, size_t *peak_bytes) {
    if (s == nullptr || admitted == nullptr || groups == nullptr || peak_bytes == nullptr) return GOLDI_EINVAL;
    std::lock_guard<std::mutex> lock(s->mu);
    *admitted = s->admitted;
    *groups = s->groups;
    *peak_bytes = s->peak_bytes;
    return GOLDI_OK;
}

int goldi_server_destroy(goldi_server *s) {
    if (s == nullptr) return GOLDI_EINVAL;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->th.joinable()) s->th.join();
    // The scheduler has ended: no batch is running and nothing is queued.
    for (auto &kv : s->reqs) {
        Request *r = kv.second;
        if (!s->slots.empty()) free_request_memory(s, r, s->slots[0].stream);
        delete r;
    }
    s->reqs.clear();
    for (auto &sl : s->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
    }
    for (auto &sl : s->slots) {
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.status_dev) (void)hipFree(sl.status_dev);
        if (sl.status_host) (void)hipHostFree(sl.status_host);
        if (sl.roots_host) (void)hipHostFree(sl.roots_host);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete s;
    return GOLDI_OK;
}

}  // extern "C"
