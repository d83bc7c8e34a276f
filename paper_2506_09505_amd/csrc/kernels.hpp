// Device kernels of the Merkle builder: permutation, leaf linear hash and
// level reduce, each in three layouts of one permutation (poseidon.hpp: one
// state per lane, the state's 12 words in 24 VGPRs; poseidon_quad.hpp: four
// lanes per state; poseidon_lane12.hpp: one word per lane), the tree top in
// one single-workgroup launch, and the batched variants that cover up to 64
// trees per launch.
#pragma once
#include <hip/hip_runtime.h>

#include "poseidon.hpp"
#include "poseidon_quad.hpp"
#include "poseidon_lane12.hpp"

namespace goldi {

static constexpr uint32_t STATUS_NONCANON = 1u;
static constexpr int BLOCK = 256;

// Minimum waves per SIMD the register allocator must allow (VGPR budget
// 512 / waves): the permutation has enough instruction-level parallelism
// that 4 resident waves already keep the VALU busy (measured: 4 to 8
// waves per SIMD change the permutation rate by under 1%).
#ifndef GOLDI_WAVES_PER_EU
#define GOLDI_WAVES_PER_EU 4
#endif
// The interleaved product blocks (field_asm.inc) use v110..v127 as scratch,
// which lies inside the kernel's register budget only up to four waves per
// SIMD (128 VGPRs each).
static_assert(GOLDI_WAVES_PER_EU <= 4, "field_asm.inc scratch registers v110..v127 need a 128-VGPR budget");
#define GOLDI_KERNEL_ATTRS __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(GOLDI_WAVES_PER_EU)))

__device__ __forceinline__ void report(uint32_t *status, bool bad) {
    if (bad) atomicOr(status, STATUS_NONCANON);
}

// Stores the canonical digest state[0..3] (Sec. 2.4: digest = words 0..3).
__device__ __forceinline__ void store_digest(u64 *dst, const u64 s[WIDTH]) {
#pragma unroll
    for (int k = 0; k < DIGEST; k++) dst[k] = canon(s[k]);
}

// ---------------------------------------------------------------------------
// Per-item bodies, shared by the single-tree and the batched kernels.

// Leaf linear hash of row r (Sec. 2.4 sponge, Sec. 4.2 leaves): the row of
// the column-major matrix is absorbed in chunks of 8 words; lane r reads
// leaves[c*ld + r] (ld: the column stride, the matrix's full row count), so a
// wave's loads of one column are contiguous.
// SINGLE: the caller guarantees n_cols <= 8, so the row is one absorption of
// a zero-capacity state and only the digest is kept (the permutation skips
// the constant S-boxes of round 0 and rows 4..11 of the last matrix).
template <bool SINGLE>
__device__ __forceinline__ void leaf_row(const u64 *__restrict__ leaves, size_t ld, size_t n_cols,
                                         u64 *__restrict__ digests, uint32_t *status, size_t r) {
    u64 s[WIDTH];
#pragma unroll
    for (int k = 0; k < WIDTH; k++) s[k] = 0;
    bool bad = false;
    if constexpr (SINGLE) {
#pragma unroll
        for (int k = 0; k < RATE; k++) {
            if (k < (int)n_cols) {
                const u64 w = leaves[(size_t)k * ld + r];
                bad |= w >= P;
                s[k] = w;
            }
        }
        permute(s, true, true);
    } else {
        for (size_t c0 = 0; c0 < n_cols; c0 += RATE) {
#pragma unroll
            for (int k = 0; k < RATE; k++) {
                if (c0 + k < n_cols) {
                    const u64 w = leaves[(c0 + k) * ld + r];
                    bad |= w >= P;
                    s[k] = add_weak(s[k], w);
                }
            }
            permute(s);
        }
    }
    report(status, bad);
    store_digest(digests + r * DIGEST, s);
}

// Parent i of a level: sponge(child 2i || child 2i+1); an unpaired last child
// moves up unchanged (Sec. 2.4 "Merkle Tree", Sec. 4.2).  Children are
// canonical digests written by this library.
__device__ __forceinline__ void level_node(const u64 *__restrict__ child, size_t n_child, u64 *__restrict__ parent,
                                           size_t i) {
    const u64 *c = child + 2 * i * DIGEST;
    if (2 * i + 1 < n_child) {
        u64 s[WIDTH];
#pragma unroll
        for (int k = 0; k < 2 * DIGEST; k++) s[k] = c[k];
#pragma unroll
        for (int k = 2 * DIGEST; k < WIDTH; k++) s[k] = 0;
        permute(s, true, true);
        store_digest(parent + i * DIGEST, s);
    } else {
#pragma unroll
        for (int k = 0; k < DIGEST; k++) parent[i * DIGEST + k] = c[k];
    }
}

// Quad bodies (4 lanes per state, poseidon_quad.hpp).  A quad is either
// entirely in range or entirely out of range, so callers may return early
// per quad; the LDS constant table must be loaded before that.

// Stores the digest from a quad: words 0..2 live in lane 0, word 3 in lane 1.
__device__ __forceinline__ void store_digest_quad(u64 *d, const u64 w[3], int q) {
    if (q == 0) {
        d[0] = canon(w[0]);
        d[1] = canon(w[1]);
        d[2] = canon(w[2]);
    } else if (q == 1) {
        d[3] = canon(w[0]);
    }
}

__device__ __forceinline__ void leaf_row_quad(const u64 *__restrict__ leaves, size_t ld, size_t n_cols,
                                              u64 *__restrict__ digests, uint32_t *status, size_t r, int q,
                                              const QuadTab &tbl) {
    u64 w[3] = {0, 0, 0};
    bool bad = false;
    for (size_t c0 = 0; c0 < n_cols; c0 += RATE) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int idx = 3 * q + k;
            if (idx < RATE && c0 + idx < n_cols) {
                const u64 v = leaves[(c0 + idx) * ld + r];
                bad |= v >= P;
                w[k] = add_weak(w[k], v);
            }
        }
        permute_quad(w, q, tbl);
    }
    report(status, bad);
    store_digest_quad(digests + r * DIGEST, w, q);
}

__device__ __forceinline__ void level_node_quad(const u64 *__restrict__ child, size_t n_child,
                                                u64 *__restrict__ parent, size_t i, int q, const QuadTab &tbl) {
    const u64 *c = child + 2 * i * DIGEST;
    if (2 * i + 1 < n_child) {
        u64 w[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int idx = 3 * q + k;
            w[k] = idx < 2 * DIGEST ? c[idx] : 0;
        }
        permute_quad(w, q, tbl);
        store_digest_quad(parent + i * DIGEST, w, q);
    } else {
        parent[i * DIGEST + q] = c[q];
    }
}

// One-word-per-lane bodies (poseidon_lane12.hpp): a 16-lane row per state.
// Every lane must reach the permutation (it reads other lanes), so range
// checks guard only loads and stores.

__device__ __forceinline__ void leaf_row_lane12(const u64 *__restrict__ leaves, size_t ld, size_t n_cols,
                                                u64 *__restrict__ digests, uint32_t *status, size_t r, bool valid,
                                                const Lane12 &L, const QuadRc &tbl) {
    u64 x = 0;
    bool bad = false;
    for (size_t c0 = 0; c0 < n_cols; c0 += RATE) {
        if (valid && L.i < RATE && c0 + L.i < n_cols) {
            const u64 v = leaves[(c0 + L.i) * ld + r];
            bad |= v >= P;
            x = add_weak(x, v);
        }
        x = permute_lane12(x, L, tbl);
    }
    report(status, bad);
    if (valid && L.i < DIGEST) digests[r * DIGEST + L.i] = canon(x);
}

__device__ __forceinline__ void level_node_lane12(const u64 *__restrict__ child, size_t n_child,
                                                  u64 *__restrict__ parent, size_t i, bool valid, const Lane12 &L,
                                                  const QuadRc &tbl) {
    const bool pair = valid && 2 * i + 1 < n_child;
    u64 x = (pair && L.i < 2 * DIGEST) ? child[2 * i * DIGEST + L.i] : 0;
    x = permute_lane12(x, L, tbl);
    if (L.i < DIGEST) {
        if (pair) parent[i * DIGEST + L.i] = canon(x);
        else if (valid) parent[i * DIGEST + L.i] = child[2 * i * DIGEST + L.i];
    }
}

// ---------------------------------------------------------------------------
// Single-tree kernels.

// Poseidon permutation of n states [n][12], in place.
__global__ void GOLDI_KERNEL_ATTRS k_permute(u64 *states, size_t n, uint32_t *status) {
    const size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    u64 *p = states + i * WIDTH;
    u64 s[WIDTH];
    bool bad = false;
#pragma unroll
    for (int k = 0; k < WIDTH; k++) {
        s[k] = p[k];
        bad |= s[k] >= P;
    }
    report(status, bad);
    permute(s);
#pragma unroll
    for (int k = 0; k < WIDTH; k++) p[k] = canon(s[k]);
}

// Rows 0 .. n_rows-1 of a column-major matrix whose columns are ld words
// apart (ld >= n_rows: a range of rows of a taller matrix).
template <bool SINGLE>
__global__ void GOLDI_KERNEL_ATTRS k_leaf_hash(const u64 *__restrict__ leaves, size_t n_rows, size_t ld,
                                               size_t n_cols, u64 *__restrict__ digests, uint32_t *status) {
    const size_t r = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r < n_rows) leaf_row<SINGLE>(leaves, ld, n_cols, digests, status, r);
}

__global__ void GOLDI_KERNEL_ATTRS k_level(const u64 *__restrict__ child, size_t n_child, u64 *__restrict__ parent) {
    const size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (i < (n_child + 1) / 2) level_node(child, n_child, parent, i);
}

__global__ void GOLDI_KERNEL_ATTRS k_leaf_hash_quad(const u64 *__restrict__ leaves, size_t n_rows, size_t ld,
                                                    size_t n_cols, u64 *__restrict__ digests, uint32_t *status) {
    __shared__ QuadTab tbl;
    quad_tab_load(tbl);
    const size_t r = ((size_t)blockIdx.x * BLOCK + threadIdx.x) >> 2;
    if (r < n_rows) leaf_row_quad(leaves, ld, n_cols, digests, status, r, threadIdx.x & 3, tbl);
}

__global__ void GOLDI_KERNEL_ATTRS k_level_quad(const u64 *__restrict__ child, size_t n_child,
                                                u64 *__restrict__ parent) {
    __shared__ QuadTab tbl;
    quad_tab_load(tbl);
    const size_t i = ((size_t)blockIdx.x * BLOCK + threadIdx.x) >> 2;
    if (i < (n_child + 1) / 2) level_node_quad(child, n_child, parent, i, threadIdx.x & 3, tbl);
}

static constexpr int LANE12_PER_BLOCK = BLOCK / 16;  // states per block

// Several levels of a tree in one launch, one word per lane.  The level read
// first has n nodes at `off` of the level-major node array; the launch covers
// its nodes [c0, c1).  Block b takes the 2S nodes [c0 + 2S b, ...) (S =
// blockDim.x / 16 states, one per parent) and reduces them through up to
// `levels` levels, or to the root: a level's nodes pass to the next through
// LDS (and are written to the node array), a workgroup barrier separates
// levels, and waves with no parent skip the permutation.  Blocks never read
// each other's nodes, so they need no synchronisation: c0 and, unless it is
// n, c1 must be multiples of 2^levels, and 2S >= 2^levels, so that every
// parent's children lie in its own block.  Each level costs one permutation
// latency, with one launch and one global round trip for all of them.
// Used with 256-thread blocks and up to 5 levels for the narrow levels of a
// tree, and as one block of up to TOP_THREADS threads for its top, from a
// level of at most 2 TOP_STATES nodes to the root (the host sizes that
// workgroup to the level's parents, so that few waves share a SIMD).
static constexpr int TOP_THREADS = 1024;
static constexpr int TOP_STATES = TOP_THREADS / 16;

__global__ void __launch_bounds__(TOP_THREADS) k_levels_lane12(u64 *nodes, size_t off, size_t n, size_t c0,
                                                               size_t c1, int levels) {
    __shared__ QuadRc tbl;
    __shared__ u64 buf[2][2 * TOP_STATES * DIGEST];
    quad_rc_load(tbl);
    const Lane12 L = lane12_setup(tbl);
    const size_t S = blockDim.x >> 4;
    const int p = threadIdx.x >> 4;             // the state (parent) this lane works on
    const int p_wave = (threadIdx.x >> 6) * 4;  // first state of this wave
    size_t lo = c0 + (size_t)blockIdx.x * 2 * S;
    size_t hi = lo + 2 * S < c1 ? lo + 2 * S : c1;
    for (size_t k = threadIdx.x; k < (hi - lo) * DIGEST; k += blockDim.x) buf[0][k] = nodes[(off + lo) * DIGEST + k];
    __syncthreads();
    int cur = 0;
    // n, lo and hi are the same in every thread of the block: all reach each barrier.
    for (int lev = 0; lev < levels && n > 1; lev++) {
        const size_t plo = lo / 2, phi = (hi + 1) / 2;  // this block's parents; lo is even
        const size_t cnt = phi - plo;
        const bool valid = (size_t)p < cnt && L.i < WIDTH;
        const bool pair = valid && 2 * (plo + p) + 1 < n;
        const u64 *child = buf[cur];  // parent plo + p reads local children 2p, 2p + 1
        u64 x = (pair && L.i < 2 * DIGEST) ? child[2 * p * DIGEST + L.i] : 0;
        if ((size_t)p_wave < cnt) x = permute_lane12(x, L, tbl);  // whole waves only
        if (valid && L.i < DIGEST) {
            const u64 d = pair ? canon(x) : child[2 * p * DIGEST + L.i];
            buf[cur ^ 1][p * DIGEST + L.i] = d;
            nodes[(off + n + plo + p) * DIGEST + L.i] = d;
        }
        __syncthreads();
        off += n;
        n = (n + 1) / 2;
        lo = plo;
        hi = phi;
        cur ^= 1;
    }
}

__global__ void GOLDI_KERNEL_ATTRS k_leaf_hash_lane12(const u64 *__restrict__ leaves, size_t n_rows, size_t ld,
                                                      size_t n_cols, u64 *__restrict__ digests, uint32_t *status) {
    __shared__ QuadRc tbl;
    quad_rc_load(tbl);
    const Lane12 L = lane12_setup(tbl);
    const size_t r = (size_t)blockIdx.x * LANE12_PER_BLOCK + (threadIdx.x >> 4);
    leaf_row_lane12(leaves, ld, n_cols, digests, status, r, r < n_rows && L.i < WIDTH, L, tbl);
}


// ---------------------------------------------------------------------------
// Batched launches: one launch covers one step (the leaves, or one level) of
// up to MAX_BATCH independent trees.  The trees are described by value in the
// kernel arguments; block b belongs to the tree t with
// block_begin[t] <= b < block_begin[t + 1] (binary search over the uniform
// kernel-argument array, i.e. scalar loads).

static constexpr int MAX_BATCH = 64;

struct BatchTree {
    const u64 *src;    // leaves (column-major) or the child level
    u64 *dst;          // digests (level 0) or the parent level
    uint32_t *status;  // this tree's status word (leaf launches); unused for levels
    uint32_t n;        // rows, or children
    uint32_t w;        // columns (leaf launches); unused for levels
};

struct Batch {
    BatchTree t[MAX_BATCH];
    uint32_t block_begin[MAX_BATCH + 1];
    uint32_t n_trees;
};

__device__ __forceinline__ int batch_tree_of(const Batch &b, uint32_t blk) {
    int lo = 0, hi = (int)b.n_trees - 1;
    while (lo < hi) {  // last t with block_begin[t] <= blk
        const int mid = (lo + hi + 1) >> 1;
        if (b.block_begin[mid] <= blk) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Leaf launches report a non-canonical word into the status word of the tree
// it belongs to, so one bad tree does not mark the others of its batch.
template <bool SINGLE>
__global__ void GOLDI_KERNEL_ATTRS k_leaf_hash_batch(const Batch b) {
    const int t = batch_tree_of(b, blockIdx.x);
    const size_t r = (size_t)(blockIdx.x - b.block_begin[t]) * BLOCK + threadIdx.x;
    if (r < b.t[t].n) leaf_row<SINGLE>(b.t[t].src, b.t[t].n, b.t[t].w, b.t[t].dst, b.t[t].status, r);
}

__global__ void GOLDI_KERNEL_ATTRS k_leaf_hash_quad_batch(const Batch b) {
    __shared__ QuadTab tbl;
    quad_tab_load(tbl);
    const int t = batch_tree_of(b, blockIdx.x);
    const size_t r = ((size_t)(blockIdx.x - b.block_begin[t]) * BLOCK + threadIdx.x) >> 2;
    if (r < b.t[t].n)
        leaf_row_quad(b.t[t].src, b.t[t].n, b.t[t].w, b.t[t].dst, b.t[t].status, r, threadIdx.x & 3, tbl);
}

__global__ void GOLDI_KERNEL_ATTRS k_level_batch(const Batch b) {
    const int t = batch_tree_of(b, blockIdx.x);
    const size_t i = (size_t)(blockIdx.x - b.block_begin[t]) * BLOCK + threadIdx.x;
    if (i < ((size_t)b.t[t].n + 1) / 2) level_node(b.t[t].src, b.t[t].n, b.t[t].dst, i);
}

__global__ void GOLDI_KERNEL_ATTRS k_level_quad_batch(const Batch b) {
    __shared__ QuadTab tbl;
    quad_tab_load(tbl);
    const int t = batch_tree_of(b, blockIdx.x);
    const size_t i = ((size_t)(blockIdx.x - b.block_begin[t]) * BLOCK + threadIdx.x) >> 2;
    if (i < ((size_t)b.t[t].n + 1) / 2) level_node_quad(b.t[t].src, b.t[t].n, b.t[t].dst, i, threadIdx.x & 3, tbl);
}

__global__ void GOLDI_KERNEL_ATTRS k_leaf_hash_lane12_batch(const Batch b) {
    __shared__ QuadRc tbl;
    quad_rc_load(tbl);
    const Lane12 L = lane12_setup(tbl);
    const int t = batch_tree_of(b, blockIdx.x);
    const size_t r = (size_t)(blockIdx.x - b.block_begin[t]) * LANE12_PER_BLOCK + (threadIdx.x >> 4);
    leaf_row_lane12(b.t[t].src, b.t[t].n, b.t[t].w, b.t[t].dst, b.t[t].status, r, r < b.t[t].n && L.i < WIDTH,
                    L, tbl);
}

__global__ void GOLDI_KERNEL_ATTRS k_level_lane12_batch(const Batch b) {
    __shared__ QuadRc tbl;
    quad_rc_load(tbl);
    const Lane12 L = lane12_setup(tbl);
    const int t = batch_tree_of(b, blockIdx.x);
    const size_t i = (size_t)(blockIdx.x - b.block_begin[t]) * LANE12_PER_BLOCK + (threadIdx.x >> 4);
    level_node_lane12(b.t[t].src, b.t[t].n, b.t[t].dst, i, i < ((size_t)b.t[t].n + 1) / 2 && L.i < WIDTH, L, tbl);
}

}  // namespace goldi
