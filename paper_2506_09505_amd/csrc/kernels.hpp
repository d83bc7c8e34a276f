// Device kernels of the Merkle builder: permutation, leaf linear hash and
// level reduce.  One state per lane throughout (Sec. 2.4's state of 12
// words in 24 VGPRs); see poseidon.hpp for the permutation itself.
#pragma once
#include <hip/hip_runtime.h>

#include "poseidon.hpp"
#include "poseidon_quad.hpp"

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
#define GOLDI_KERNEL_ATTRS __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(GOLDI_WAVES_PER_EU)))

__device__ __forceinline__ void report(uint32_t *status, bool bad) {
    if (bad) atomicOr(status, STATUS_NONCANON);
}

// Stores the canonical digest state[0..3] (Sec. 2.4: digest = words 0..3).
__device__ __forceinline__ void store_digest(u64 *dst, const u64 s[WIDTH]) {
#pragma unroll
    for (int k = 0; k < DIGEST; k++) dst[k] = canon(s[k]);
}

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

// Leaf linear hash (Sec. 2.4 sponge): row r of the column-major matrix is
// absorbed in chunks of 8 words; lane r reads leaves[c*n_rows + r], so a
// wave's loads of one column are contiguous.
__global__ void GOLDI_KERNEL_ATTRS k_leaf_hash(const u64 *__restrict__ leaves, size_t n_rows,
                                                     size_t n_cols, u64 *__restrict__ digests,
                                                     uint32_t *status) {
    const size_t r = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    if (r >= n_rows) return;
    u64 s[WIDTH];
#pragma unroll
    for (int k = 0; k < WIDTH; k++) s[k] = 0;
    bool bad = false;
    for (size_t c0 = 0; c0 < n_cols; c0 += RATE) {
#pragma unroll
        for (int k = 0; k < RATE; k++) {
            if (c0 + k < n_cols) {
                const u64 w = leaves[(c0 + k) * n_rows + r];
                bad |= w >= P;
                s[k] = add_weak(s[k], w);
            }
        }
        permute(s);
    }
    report(status, bad);
    store_digest(digests + r * DIGEST, s);
}

// One tree level: parent i = sponge(child 2i || child 2i+1); an unpaired last
// child moves up unchanged (Sec. 2.4 "Merkle Tree", Sec. 4.2).  Children are
// canonical digests written by this library.
__global__ void GOLDI_KERNEL_ATTRS k_level(const u64 *__restrict__ child, size_t n_child,
                                                 u64 *__restrict__ parent) {
    const size_t i = (size_t)blockIdx.x * BLOCK + threadIdx.x;
    const size_t n_par = (n_child + 1) / 2;
    if (i >= n_par) return;
    const u64 *c = child + 2 * i * DIGEST;
    if (2 * i + 1 < n_child) {
        u64 s[WIDTH];
#pragma unroll
        for (int k = 0; k < 2 * DIGEST; k++) s[k] = c[k];
#pragma unroll
        for (int k = 2 * DIGEST; k < WIDTH; k++) s[k] = 0;
        permute(s);
        store_digest(parent + i * DIGEST, s);
    } else {
#pragma unroll
        for (int k = 0; k < DIGEST; k++) parent[i * DIGEST + k] = c[k];
    }
}

// ---------------------------------------------------------------------------
// Quad variants (4 lanes per state, poseidon_quad.hpp) for latency-bound
// launches: few rows or few parents.  Whole quads share one state, so a quad
// is either entirely in range or entirely out of range.

// Leaf hash, 4 lanes per row: lane q absorbs words 3q..3q+2 of each chunk.
__global__ void GOLDI_KERNEL_ATTRS k_leaf_hash_quad(const u64 *__restrict__ leaves, size_t n_rows,
                                                    size_t n_cols, u64 *__restrict__ digests,
                                                    uint32_t *status) {
    __shared__ QuadRc tbl;
    quad_rc_load(tbl);
    const size_t r = ((size_t)blockIdx.x * BLOCK + threadIdx.x) >> 2;
    const int q = threadIdx.x & 3;
    if (r >= n_rows) return;
    u64 w[3] = {0, 0, 0};
    bool bad = false;
    for (size_t c0 = 0; c0 < n_cols; c0 += RATE) {
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int idx = 3 * q + k;
            if (idx < RATE && c0 + idx < n_cols) {
                const u64 v = leaves[(c0 + idx) * n_rows + r];
                bad |= v >= P;
                w[k] = add_weak(w[k], v);
            }
        }
        permute_quad(w, q, tbl);
    }
    report(status, bad);
    u64 *d = digests + r * DIGEST;
    if (q == 0) {
        d[0] = canon(w[0]);
        d[1] = canon(w[1]);
        d[2] = canon(w[2]);
    } else if (q == 1) {
        d[3] = canon(w[0]);
    }
}

// One tree level, 4 lanes per parent.
__global__ void GOLDI_KERNEL_ATTRS k_level_quad(const u64 *__restrict__ child, size_t n_child,
                                                u64 *__restrict__ parent) {
    __shared__ QuadRc tbl;
    quad_rc_load(tbl);
    const size_t i = ((size_t)blockIdx.x * BLOCK + threadIdx.x) >> 2;
    const int q = threadIdx.x & 3;
    const size_t n_par = (n_child + 1) / 2;
    if (i >= n_par) return;
    const u64 *c = child + 2 * i * DIGEST;
    if (2 * i + 1 < n_child) {
        u64 w[3];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            const int idx = 3 * q + k;
            w[k] = idx < 2 * DIGEST ? c[idx] : 0;
        }
        permute_quad(w, q, tbl);
        u64 *d = parent + i * DIGEST;
        if (q == 0) {
            d[0] = canon(w[0]);
            d[1] = canon(w[1]);
            d[2] = canon(w[2]);
        } else if (q == 1) {
            d[3] = canon(w[0]);
        }
    } else {
        parent[i * DIGEST + q] = c[q];
    }
}

}  // namespace goldi
