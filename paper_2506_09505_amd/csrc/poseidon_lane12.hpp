// Poseidon-12 permutation with one state word per lane, for the most
// latency-bound launches (the top levels of a tree, tiny trees).
//
// A 64-lane wave holds four states, one per 16-lane row: word i of a state is
// in lane 16s + i (i < 12; the last four lanes of each row only follow along).
// A round then costs each lane one S-box and one row of the matrix product:
// row i = sum_k m[k] x[(i + k) mod 12] for the circulant M[i][j] =
// m[(j - i) mod 12], so the coefficient of the word fetched at rotation k is
// m[k] in every lane.  The eleven rotated words come from ds_bpermute
// (any-lane reads through the LDS crossbar, no LDS storage) at per-lane
// addresses computed once.  A permutation is then ~5k instructions per lane
// with most of a round's latency in its S-box chain.
#pragma once
#include "poseidon_quad.hpp"

namespace goldi {

struct Lane12 {
    int i;             // word index held by this lane (0..15; >= 12 idle)
    int addr[WIDTH];   // byte addresses for ds_bpermute: lane of word (i + k) mod 12
    int addr_w0;       // lane of word 0 of this row
    u32 m0;            // M[i][0] = m[(12 - i) mod 12], the coefficient of word 0
    u32 nz;            // all-ones except in the lane of word 0
};

__device__ __forceinline__ Lane12 lane12_setup(const QuadRc &t) {
    Lane12 L;
    const int lane = threadIdx.x & 63;
    const int base = lane & ~15;
    L.i = lane & 15;
    const int i = L.i < WIDTH ? L.i : 0;
#pragma unroll
    for (int k = 0; k < WIDTH; k++) L.addr[k] = (base + (i + k) % WIDTH) * 4;
    L.addr_w0 = base * 4;
    L.m0 = t.col0[i];
    L.nz = (L.i == 0) ? 0u : 0xFFFFFFFFu;
    return L;
}

__device__ __forceinline__ u64 bperm64(int addr, u64 v) {
    return mk64((u32)__builtin_amdgcn_ds_bpermute(addr, (int)lo32(v)),
                (u32)__builtin_amdgcn_ds_bpermute(addr, (int)hi32(v)));
}

// Row accumulation over the rotated words y[k] = x[(i + k) mod 12].
template <int K>
__device__ __forceinline__ void lane12_terms(const u64 (&y)[WIDTH], u64 &a_lo, u64 &a_hi) {
    a_lo = mad_small<GOLDI_MDS[0][K]>(lo32(y[K]), a_lo);
    a_hi = mad_small<GOLDI_MDS[0][K]>(hi32(y[K]), a_hi);
    if constexpr (K + 1 < WIDTH) lane12_terms<K + 1>(y, a_lo, a_hi);
}

// x <- row i of (M x) + C[r1][i]; `src` is the word each lane publishes.
__device__ __forceinline__ void lane12_rows(const Lane12 &L, u64 src, const u64 *rc_word, u64 &a_lo, u64 &a_hi) {
    u64 y[WIDTH];
    y[0] = src;
#pragma unroll
    for (int k = 1; k < WIDTH; k++) y[k] = bperm64(L.addr[k], src);
    a_lo = rc_word[0];
    a_hi = rc_word[1];
    lane12_terms<0>(y, a_lo, a_hi);
}

// Permutes the four states of the wave; every lane of the wave must be
// active (ds_bpermute reads other lanes).
__device__ __forceinline__ u64 permute_lane12(u64 x, const Lane12 &L, const QuadRc &t) {
    const int i = L.i < WIDTH ? L.i : 0;
    x = add_weak(x, mk64(lo32(t.rc[0][i][0]), lo32(t.rc[0][i][1])));
    u64 a_lo, a_hi;
#pragma nounroll
    for (int r = 0; r < HALF_FULL; r++) {
        lane12_rows(L, sbox(x), t.rc[r + 1][i], a_lo, a_hi);
        x = reduce_split(a_lo, a_hi);
    }
#pragma nounroll
    for (int r = HALF_FULL; r < HALF_FULL + PARTIAL; r++) {
        // Word 0 is published as zero while its S-box runs; the S-box result
        // of the row's word-0 lane is then broadcast and added with M[i][0].
        lane12_rows(L, mk64(lo32(x) & L.nz, hi32(x) & L.nz), t.rc[r + 1][i], a_lo, a_hi);
        const u64 sb = bperm64(L.addr_w0, sbox(x));
        a_lo = mad32(L.m0, lo32(sb), a_lo);
        a_hi = mad32(L.m0, hi32(sb), a_hi);
        x = reduce_split(a_lo, a_hi);
    }
#pragma nounroll
    for (int r = HALF_FULL + PARTIAL; r < ROUNDS; r++) {
        lane12_rows(L, sbox(x), t.rc[r + 1][i], a_lo, a_hi);
        x = reduce_split(a_lo, a_hi);
    }
    return x;
}

}  // namespace goldi
