/*
 * goldi.h -- C ABI of the MI355X (gfx950) Poseidon-12 / Goldilocks Merkle
 * builder.
 *
 * What is computed (arXiv 2506.09505):
 *   - the Goldilocks field p = 2^64 - 2^32 + 1 (Sec. 2.4, Eq. 1); every word
 *     handed in or out is a canonical element, 0 <= x < p;
 *   - the Poseidon permutation of a 12-word state: 4 full, 22 partial, 4 full
 *     rounds with S-box x^7 and a 12 x 12 matrix (Sec. 2.4, Alg. 1);
 *   - the sponge "absorbing" rows in chunks of eight words (Sec. 2.4): state
 *     starts at zero, each chunk is added into words 0..7 (a short last chunk
 *     adds zeros), then the state is permuted; the digest is words 0..3;
 *   - the Merkle tree (Sec. 2.4 "Merkle Tree", Sec. 4.2): leaf digests first,
 *     then level by level each parent is the sponge of the 8-word
 *     concatenation left||right of its two children, until one root.  An
 *     unpaired last node of a level moves up unchanged.
 * The round constants and matrix are a seeded instance (the paper prints no
 * values); the library is compiled against that one instance.
 *
 * Layouts (all words are uint64_t):
 *   states    [n][12] row-major, permuted in place.
 *   leaves    column-major: element (row r, column c) at leaves[c*n_rows + r]
 *             (columns are polynomials, rows are the tree's leaves).
 *   nodes_out level-major, 4 words per node: level 0 (n_rows leaf digests),
 *             then level 1 (ceil(n_rows/2) nodes), ... ; the root is the last
 *             node.  Size: goldi_merkle_num_nodes(n_rows) nodes.
 *
 * Memory: every data pointer is DEVICE memory (hipMalloc, or a PyTorch
 * tensor's storage) on the current HIP device.  The caller owns and
 * allocates every buffer; the library keeps no pointer after a call returns
 * (synchronous calls) or after the stream work completes (asynchronous
 * calls).  nodes_out must not overlap leaves.
 *
 * Errors: every call returns a status code.  Inputs >= p are detected on the
 * device and give GOLDI_ENONCANON (output contents are then unspecified).
 * Null pointers, zero sizes or sizes whose byte counts overflow give
 * GOLDI_EINVAL before anything is launched; so do more than 2^32 - 256
 * states or rows, since one kernel dispatch covers at most 2^32 - 1
 * work-items.  A launch that would exceed that limit because the schedule
 * knobs (goldi_tune_set) put many lanes on each item is refused with
 * GOLDI_EINVAL when it is reached; kernels already enqueued by the same
 * call then leave the output incomplete.  HIP failures give GOLDI_EDEVICE;
 * goldi_last_error() returns a thread-local message for the last failure.
 * No C++ exception crosses this interface.
 *
 * Threads: calls are thread-safe.  Synchronous calls run on the legacy null
 * stream of the current device and return when the work is complete.
 */
#ifndef GOLDI_H
#define GOLDI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GOLDI_OK = 0,
    GOLDI_EINVAL = -1,    /* bad argument (null, zero size, overflow)        */
    GOLDI_ENONCANON = -2, /* an input word was >= p                          */
    GOLDI_EDEVICE = -3,   /* a HIP call failed; see goldi_last_error()       */
    GOLDI_ENOMEM = -4,    /* a device allocation failed                      */
    GOLDI_ECANCELED = -5, /* serving: the request was still queued when the
                             server was destroyed                            */
    GOLDI_ETIMEDOUT = -6  /* serving: the request's batch did not complete
                             within the server's watchdog time               */
};

/* Poseidon-12 permutation (Sec. 2.4, Alg. 1) of n states, in place.
 * states: device pointer to [n][12] words, each < p.  n >= 1.
 * Returns GOLDI_OK, GOLDI_EINVAL, GOLDI_ENONCANON or GOLDI_EDEVICE. */
int goldi_poseidon_permute(uint64_t *states, size_t n);

/* Number of nodes of a tree over n leaves: sum of the level sizes n_l with
 * n_0 = n and n_{l+1} = ceil(n_l / 2) down to 1 (2n - 1 when n is a power of
 * two).  Returns 0 for n = 0. */
size_t goldi_merkle_num_nodes(size_t n_rows);

/* Leaf linear hash (the sponge of Sec. 2.4 over each row, Sec. 4.2):
 * leaves column-major [n_cols][n_rows] -> digests [n_rows][4].
 * n_rows >= 1, n_cols >= 1.  Same error codes as the permutation. */
int goldi_leaf_hash(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *digests);

/* Whole Merkle tree (Sec. 2.4 "Merkle Tree", Sec. 4.2): writes every node of
 * the tree over the rows of `leaves` into nodes_out (level-major, see above).
 * n_rows >= 1, n_cols >= 1. */
int goldi_merkle_build(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *nodes_out);

/* One tree for goldi_merkle_build_many. */
typedef struct {
    const uint64_t *leaves; /* device, column-major [n_cols][n_rows]          */
    size_t n_rows;          /* >= 1                                           */
    size_t n_cols;          /* >= 1                                           */
    uint64_t *nodes_out;    /* device, goldi_merkle_num_nodes(n_rows) * 4 words */
} goldi_tree_t;

/* Many independent trees in one call (the trees of Sec. 4.2, built side by
 * side).  trees: HOST array of n_trees descriptors (n_trees >= 1); each
 * tree's output equals goldi_merkle_build on that tree alone.  Outputs of
 * different trees must not overlap each other or any input. */
int goldi_merkle_build_many(const goldi_tree_t *trees, size_t n_trees);

/* Asynchronous twins.  They enqueue on `stream` (a hipStream_t; 0 = null
 * stream) and return without waiting.  Argument checks happen before
 * anything is enqueued; device-side failures are reported by OR-ing a bit
 * into *dev_status (a device word the caller zeroes beforehand): bit 0 =
 * an input word was >= p.  The return value covers launch errors only. */
int goldi_poseidon_permute_async(uint64_t *states, size_t n, uint32_t *dev_status, void *stream);
int goldi_leaf_hash_async(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *digests,
                          uint32_t *dev_status, void *stream);
int goldi_merkle_build_async(const uint64_t *leaves, size_t n_rows, size_t n_cols, uint64_t *nodes_out,
                             uint32_t *dev_status, void *stream);
int goldi_merkle_build_many_async(const goldi_tree_t *trees, size_t n_trees, uint32_t *dev_status,
                                  void *stream);

/* goldi_merkle_build_many_async with one status word per tree: tree k
 * (in the order of `trees`) ORs its bits into dev_status[k], so a tree with
 * a non-canonical word is reported alone and every other tree of the call
 * is built exactly as goldi_merkle_build would build it alone.
 * dev_status: device array of n_trees words, zeroed by the caller. */
int goldi_merkle_build_many_status_async(const goldi_tree_t *trees, size_t n_trees, uint32_t *dev_status,
                                         void *stream);

/* goldi_merkle_build_many for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc): the same trees,
 * the same schedule and the same outputs, but the per-tree status words live
 * in a fixed array inside the library (one per GPU, kept until the process
 * ends) instead of memory allocated by the call; nothing is allocated.
 * n_trees: 1..4096 (GOLDI_EINVAL with a message beyond).  tree_status: NULL
 * or a HOST array of n_trees codes (GOLDI_OK or GOLDI_ENONCANON per tree).
 * The work is enqueued on `stream` (0 = null stream) and the call waits for
 * it.  Calls on one GPU share the array: the library serialises them, and
 * the array keeps the last call's words (each call clears its words first).
 * Returns GOLDI_OK, GOLDI_ENONCANON if any tree held a word >= p, or the
 * error codes of goldi_merkle_build_many. */
int goldi_merkle_build_many_noalloc(const goldi_tree_t *trees, size_t n_trees, int *tree_status, void *stream);

/* Schedule knobs (process-wide).  Every setting computes the same bytes;
 * only speed changes.  Keys:
 *   "quad_max_rows"    leaf hashing of at most this many rows runs 4 lanes per
 *                      row (default 2^14; lower latency, ~1.7x the
 *                      instructions per row);
 *   "quad_max_parents" tree levels of at most this many parents do the same
 *                      (default 2^16);
 *   "lane12_max_rows", "lane12_max_parents"
 *                      at or below these sizes (default 2^13 each) one
 *                      state word per lane (a 16-lane row per state) is used
 *                      instead: lower latency again, ~3x the instructions
 *                      per row;
 *   "top_max_parents"  single-tree builds run every level from the first one
 *                      of at most this many parents up to the root in one
 *                      single-workgroup launch (default 16, at most 64;
 *                      0 = one launch per level; GOLDI_EINVAL above 64);
 *   "split_parts"      single-tree builds of at least "split_min_rows" rows
 *                      (default 2^20) hash the leaves and build every level
 *                      with more than "split_join_parents" parents (default
 *                      4096) as this many ranges of rows (default 2, at most 4;
 *                      0 or 1 = no split), each on its own library-owned
 *                      stream (created on first use per device, default
 *                      priority), joined on the caller's stream before the
 *                      remaining levels: the call still orders all of its work
 *                      on `stream`.  No split while `stream` is being
 *                      captured into a graph;
 *   "split_min_rows", "split_join_parents"
 *                      see "split_parts";
 *   "batch_mode"       goldi_merkle_build_many: 1 (default) = one launch per
 *                      tree level across all trees (up to 64 trees per
 *                      launch, heaviest rows first), 0 = tree after tree;
 *   "graph"            goldi_merkle_build_many: 1 = capture the launch
 *                      sequence into a hipGraph, cached per batch description
 *                      (pointers, sizes, status word, knobs; 16 most recent),
 *                      and replay it; 0 (default) = launch directly.
 * goldi_tune_get also reads "partial_form", fixed when the library is
 * compiled: how the one-state-per-lane permutation evaluates the partial
 * rounds (2 = blocks of three rounds as one product with 32-bit entries,
 * 1 = the sparse form of Sec. 2.4 / Alg. 1, 0 = the dense matrix every
 * round), and "mds_limb_bits": the limb width of the full-round matrix
 * products (32 = 32 x 32 -> 64-bit multiply-adds, 22 = 24-bit multipliers on
 * 22-bit limbs, a test build); goldi_tune_set rejects both with GOLDI_EINVAL.
 * Returns GOLDI_EINVAL for an unknown key or a null pointer. */
int goldi_tune_set(const char *key, size_t value);
int goldi_tune_get(const char *key, size_t *value);

/* Per-kernel timing for measurement; off by default.  While enabled, the
 * kernels the library launches are timed with HIP events recorded on the
 * stream they are launched on: each run of consecutive launches of one kind
 * within one call (e.g. the largest levels of a tree) is bracketed by one
 * pair of events, which also covers the gaps between those launches.  Costs a
 * few microseconds per run.  In a split build (see "split_parts") the two
 * halves' launches run side by side on two streams, so their runs overlap in
 * time and a run's span includes the other stream's work; set "split_parts"
 * to 0 to time each launch alone. */
int goldi_profile_enable(int on);

/* Restricts the timing to one kernel kind (names as for goldi_profile_read);
 * NULL or "" times every kind again. */
int goldi_profile_select(const char *kernel);

/* Sums the elapsed times of the recorded runs of one kernel kind
 * ("permute", "leaf_hash", "leaf_hash_quad", "leaf_hash_lane12", "level",
 * "level_quad", "level_lane12", "top_lane12"), waiting for them to finish,
 * and forgets them; *count receives the number of launches they covered.
 * total_ms and count are host pointers; returns GOLDI_EINVAL for nulls and
 * GOLDI_EDEVICE if an event query fails. */
int goldi_profile_read(const char *kernel, double *total_ms, size_t *count);

/* ---------------------------------------------------------------- serving
 * A serving loop with continuous batching.  Requests are tree builds (the
 * tree of goldi_merkle_build).  A scheduler thread admits waiting requests in
 * arrival order whenever one of `n_slots` slots (each a HIP stream) is free
 * and the device bytes of all admitted, unreleased requests stay within
 * `hbm_budget_bytes`; up to `max_group` requests admitted together are built
 * as one batch.  Slots run concurrently, so newly admitted requests overlap
 * on the device with those already running.  Per request the server holds,
 * in device memory from the stream-ordered allocator, a copy of host leaves
 * (freed when the build completes) and all nodes (kept until released).
 * The root is returned to the host.  All server calls are thread-safe.
 *
 * Failure isolation: every request of a batch has its own device status word,
 * so a request holding a word >= p fails alone (GOLDI_ENONCANON) and its
 * batch-mates complete normally.  If a whole batch fails on the host side
 * (an allocation or launch error), each of its requests is queued again at
 * the head of the queue and rebuilt in a batch of its own; only a request
 * that fails alone too is reported failed.  A watchdog marks the requests of
 * a batch that has not completed within the watchdog time GOLDI_ETIMEDOUT
 * and wakes their waiters; the batch's device memory is kept until the GPU
 * work really completes (a release in the meantime is deferred until then). */
typedef struct goldi_server goldi_server;

typedef struct {
    int status;            /* GOLDI_OK, GOLDI_ENONCANON, GOLDI_EDEVICE,
                              GOLDI_ETIMEDOUT or GOLDI_ECANCELED               */
    size_t n_rows, n_cols;
    uint64_t *nodes;       /* device, level-major nodes; valid until release  */
    int64_t t_submit_ns;   /* steady-clock times of submission, admission and */
    int64_t t_admit_ns;    /* completion (completion is observed by polling   */
    int64_t t_done_ns;     /* every ~20 us)                                    */
    int group_size;        /* requests built in the same batch                 */
    uint64_t root[4];      /* canonical root digest                            */
} goldi_request_info;

/* Creates a server on the current device.  n_slots in 1..64, max_group in
 * 1..64, budget > 0.  Returns GOLDI_EINVAL or GOLDI_EDEVICE on failure. */
int goldi_server_create(size_t hbm_budget_bytes, unsigned n_slots, unsigned max_group, goldi_server **out);

/* Queues one request.  Exactly one of leaves_host (host memory, preferably
 * pinned; it must stay valid until the request completes) and leaves_dev
 * (device memory on the server's device, valid until completion) is non-null;
 * both are column-major [n_cols][n_rows].  n_rows, n_cols in 1..2^32-1.
 * Returns GOLDI_ENOMEM if the request alone exceeds the budget. */
int goldi_server_submit(goldi_server *s, const uint64_t *leaves_host, const uint64_t *leaves_dev, size_t n_rows,
                        size_t n_cols, uint64_t *request_id);

/* Blocks until the request completes and fills *info (host pointer). */
int goldi_server_wait(goldi_server *s, uint64_t id, goldi_request_info *info);

/* Copies a completed, unreleased request's nodes (goldi_merkle_num_nodes(n_rows)
 * * 4 words) to dst (device or host memory of at least dst_words words).
 * Blocks until the copy is done. */
int goldi_server_read_nodes(goldi_server *s, uint64_t id, uint64_t *dst, size_t dst_words);

/* Frees a completed request's nodes and forgets it. */
int goldi_server_release(goldi_server *s, uint64_t id);

/* Requests admitted, batches formed and the peak of admitted device bytes. */
int goldi_server_stats(goldi_server *s, size_t *admitted, size_t *groups, size_t *peak_bytes);

/* Server settings (keys):
 *   "watchdog_us"        time a batch may run before its requests are marked
 *                        GOLDI_ETIMEDOUT (default 30 s; 0 disables);
 *   "fail_next_batches"  a fault-injection hook for tests: the next `value`
 *                        batches of two or more requests are treated as if
 *                        their launch had failed, before anything is
 *                        enqueued for them (so their requests take the
 *                        rebuild-alone path).
 * Returns GOLDI_EINVAL for an unknown key. */
int goldi_server_set(goldi_server *s, const char *key, uint64_t value);

/* Stops the server: requests still queued (not admitted) are completed with
 * GOLDI_ECANCELED, admitted batches are waited for, then the server and all
 * unreleased nodes are freed.  No call on `s` may run concurrently with or
 * after it. */
int goldi_server_destroy(goldi_server *s);

/* The admission rule, exposed so it can be checked without a GPU: with
 * `inflight_bytes` already admitted, how many requests from the head of the
 * queue (device bytes pending_bytes[0..n_pending)) are admitted together:
 * the longest prefix, at most max_group long, whose bytes fit the budget. */
int goldi_admission_plan(const size_t *pending_bytes, size_t n_pending, size_t budget, size_t inflight_bytes,
                         size_t max_group, size_t *take);

/* Static text for a status code. */
const char *goldi_strerror(int code);

/* Thread-local detail of the last failing call on this thread ("" if none). */
const char *goldi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* GOLDI_H */
