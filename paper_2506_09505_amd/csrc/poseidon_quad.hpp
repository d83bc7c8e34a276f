// Poseidon-12 permutation spread over the 4 lanes of a quad, for the
// latency-bound parts of a tree (its small top levels, small trees).
//
// One state per lane (poseidon.hpp) is the throughput layout: a wave runs 64
// permutations, but one permutation takes ~20k dependent-ish instructions, so
// a level with few nodes costs a whole permutation latency.  Here lane q of a
// quad holds words 3q, 3q+1, 3q+2 of the 12-word state (Sec. 2.4); a round
// runs its S-boxes on 3 words per lane and each lane computes 3 rows of the
// matrix product after fetching the other 9 words from its quad neighbours
// with DPP quad permutations.  A permutation then takes about a third of the
// instructions per lane.
//
// Because M is circulant (M[i][j] = m[(j - i) mod 12]) and 12 = 3 x 4, the
// entry multiplying word k of the quad neighbour at distance d in output row
// r of lane q is m[(3d + k - r) mod 12], independent of q: all lanes run the
// same code with the same inline constants.  Round constants differ per lane
// (words 3q..3q+2), so they are read from a copy of the table in LDS.
#pragma once
#include "poseidon.hpp"

namespace goldi {

// Value of `v` in lane (q + D) mod 4 of this lane's quad.
template <int D>
__device__ __forceinline__ u32 quad_fetch(u32 v) {
    constexpr int ctrl = ((0 + D) & 3) | (((1 + D) & 3) << 2) | (((2 + D) & 3) << 4) | (((3 + D) & 3) << 6);
    return (u32)__builtin_amdgcn_mov_dpp((int)v, ctrl, 0xF, 0xF, false);
}

template <int D>
__device__ __forceinline__ u64 quad_fetch64(u64 v) {
    return mk64(quad_fetch<D>(lo32(v)), quad_fetch<D>(hi32(v)));
}

// Row r of this lane's 3 rows: sum over quad distance d and word k.
template <int R, int D, int K>
__device__ __forceinline__ void quad_row_terms(const u64 (&x)[4][3], u64 &a_lo, u64 &a_hi) {
    constexpr unsigned m = GOLDI_MDS[0][(3 * D + K - R + 12) % 12];
    a_lo = mad_small<m>(lo32(x[D][K]), a_lo);
    a_hi = mad_small<m>(hi32(x[D][K]), a_hi);
    if constexpr (K < 2) {
        quad_row_terms<R, D, K + 1>(x, a_lo, a_hi);
    } else if constexpr (D < 3) {
        quad_row_terms<R, D + 1, 0>(x, a_lo, a_hi);
    }
}

// rc_lane: this lane's 3 round-constant words for round r1, split halves.
__device__ __forceinline__ void quad_mds_add_rc(u64 w[3], const u64 (*rc_lane)[2]) {
    u64 x[4][3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        x[0][k] = w[k];
        x[1][k] = quad_fetch64<1>(w[k]);
        x[2][k] = quad_fetch64<2>(w[k]);
        x[3][k] = quad_fetch64<3>(w[k]);
    }
    u64 a_lo, a_hi;
    a_lo = rc_lane[0][0];
    a_hi = rc_lane[0][1];
    quad_row_terms<0, 0, 0>(x, a_lo, a_hi);
    w[0] = reduce_split(a_lo, a_hi);
    a_lo = rc_lane[1][0];
    a_hi = rc_lane[1][1];
    quad_row_terms<1, 0, 0>(x, a_lo, a_hi);
    w[1] = reduce_split(a_lo, a_hi);
    a_lo = rc_lane[2][0];
    a_hi = rc_lane[2][1];
    quad_row_terms<2, 0, 0>(x, a_lo, a_hi);
    w[2] = reduce_split(a_lo, a_hi);
}

// The round-constant table in LDS: rc[r][i][half], rows 0..ROUNDS.
struct QuadRc {
    u64 rc[ROUNDS + 1][WIDTH][2];
};

// Fills the LDS copy of the table; every thread of the block must call it.
__device__ __forceinline__ void quad_rc_load(QuadRc &t) {
    const u64 *src = &RC_SPLIT[0][0][0];
    u64 *dst = &t.rc[0][0][0];
    constexpr int n = (ROUNDS + 1) * WIDTH * 2;
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
    __syncthreads();
}

// Permutes the state spread over the quad; q = lane index in the quad.
// All 4 lanes of the quad must be active.
__device__ __forceinline__ void permute_quad(u64 w[3], int q, const QuadRc &t) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const u64 *c = t.rc[0][3 * q + k];
        w[k] = add_weak(w[k], mk64(lo32(c[0]), lo32(c[1])));
    }
#pragma nounroll
    for (int r = 0; r < HALF_FULL; r++) {
#pragma unroll
        for (int k = 0; k < 3; k++) w[k] = sbox(w[k]);
        quad_mds_add_rc(w, t.rc[r + 1] + 3 * q);
    }
#pragma nounroll
    for (int r = HALF_FULL; r < HALF_FULL + PARTIAL; r++) {
        if (q == 0) w[0] = sbox(w[0]);
        quad_mds_add_rc(w, t.rc[r + 1] + 3 * q);
    }
#pragma nounroll
    for (int r = HALF_FULL + PARTIAL; r < ROUNDS; r++) {
#pragma unroll
        for (int k = 0; k < 3; k++) w[k] = sbox(w[k]);
        quad_mds_add_rc(w, t.rc[r + 1] + 3 * q);
    }
}

}  // namespace goldi
