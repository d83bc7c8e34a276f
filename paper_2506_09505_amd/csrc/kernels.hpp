// Device kernels of the Merkle builder: permutation, leaf linear hash and
// level reduce.  One state per lane throughout (Sec. 2.4's state of 12
// words in 24 VGPRs); see poseidon.hpp for the permutation itself.
#pragma once
#include <hip/hip_runtime.h>

#include "poseidon.hpp"

namespace goldi {

static constexpr uint32_t STATUS_NONCANON = 1u;
static constexpr int BLOCK = 256;

__device__ __forceinline__ void report(uint32_t *status, bool bad) {
    if (bad) atomicOr(status, STATUS_NONCANON);
}

// Stores the canonical digest state[0..3] (Sec. 2.4: digest = words 0..3).
__device__ __forceinline__ void store_digest(u64 *dst, const u64 s[WIDTH]) {
#pragma unroll
    for (int k = 0; k < DIGEST; k++) dst[k] = canon(s[k]);
}

// Poseidon permutation of n states [n][12], in place.
__global__ void __launch_bounds__(BLOCK) k_permute(u64 *states, size_t n, uint32_t *status) {
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
__global__ void __launch_bounds__(BLOCK) k_leaf_hash(const u64 *__restrict__ leaves, size_t n_rows,
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
__global__ void __launch_bounds__(BLOCK) k_level(const u64 *__restrict__ child, size_t n_child,
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

}  // namespace goldi
