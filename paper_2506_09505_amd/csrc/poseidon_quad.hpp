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
// (words 3q..3q+2), so they are read from a copy of the table in LDS, as are
// the entries of the partial rounds' block form (quad_block), whose matrix
// is not circulant.
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
    a_lo = mad_small_c<m>(lo32(x[D][K]), a_lo);
    a_hi = mad_small_c<m>(hi32(x[D][K]), a_hi);
    if constexpr (K < 2) {
        quad_row_terms<R, D, K + 1>(x, a_lo, a_hi);
    } else if constexpr (D < 3) {
        quad_row_terms<R, D + 1, 0>(x, a_lo, a_hi);
    }
}

// Accumulates the 3 rows of this lane (unreduced, split halves) from the
// quad's 12 words; rc_lane: this lane's 3 round-constant words, split halves.
__device__ __forceinline__ void quad_mds_accumulate(const u64 w[3], const u64 (*rc_lane)[2], u64 a_lo[3],
                                                    u64 a_hi[3]) {
    u64 x[4][3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        x[0][k] = w[k];
        x[1][k] = quad_fetch64<1>(w[k]);
        x[2][k] = quad_fetch64<2>(w[k]);
        x[3][k] = quad_fetch64<3>(w[k]);
    }
#pragma unroll
    for (int r = 0; r < 3; r++) {
        a_lo[r] = rc_lane[r][0];
        a_hi[r] = rc_lane[r][1];
    }
    quad_row_terms<0, 0, 0>(x, a_lo[0], a_hi[0]);
    quad_row_terms<1, 0, 0>(x, a_lo[1], a_hi[1]);
    quad_row_terms<2, 0, 0>(x, a_lo[2], a_hi[2]);
}

__device__ __forceinline__ void quad_mds_add_rc(u64 w[3], const u64 (*rc_lane)[2]) {
    u64 a_lo[3], a_hi[3];
    quad_mds_accumulate(w, rc_lane, a_lo, a_hi);
#pragma unroll
    for (int r = 0; r < 3; r++) w[r] = reduce_split_c(a_lo[r], a_hi[r]);
}

// Partial round, arranged so the matrix product does not wait for the S-box:
// the product is accumulated with word 0 of the state (held by lane 0) read
// as zero, while every lane runs the S-box on its own word 0; lane 0's result
// is then broadcast to the quad and added with this lane's column-0 entries
// m0[r] = M[3q + r][0].  nz is all-ones in lanes 1..3 and zero in lane 0.
__device__ __forceinline__ void quad_partial_round(u64 w[3], const u64 (*rc_lane)[2], u32 nz, const u32 m0[3]) {
    const u64 w0 = w[0];
    u64 masked[3] = {mk64(lo32(w0) & nz, hi32(w0) & nz), w[1], w[2]};
    u64 a_lo[3], a_hi[3];
    quad_mds_accumulate(masked, rc_lane, a_lo, a_hi);
    const u64 sb = sbox_blocks(w0);
    const u32 s_lo = (u32)__builtin_amdgcn_mov_dpp((int)lo32(sb), 0x00, 0xF, 0xF, false);  // quad_perm [0,0,0,0]
    const u32 s_hi = (u32)__builtin_amdgcn_mov_dpp((int)hi32(sb), 0x00, 0xF, 0xF, false);
#pragma unroll
    for (int r = 0; r < 3; r++) {
        a_lo[r] = mad32(m0[r], s_lo, a_lo[r]);
        a_hi[r] = mad32(m0[r], s_hi, a_hi[r]);
        w[r] = reduce_split_c(a_lo[r], a_hi[r]);
    }
}

// The round-constant table in LDS: rc[r][i][half], rows 0..ROUNDS.
struct QuadRc {
    u64 rc[ROUNDS + 1][WIDTH][2];
    u32 col0[WIDTH];  // column 0 of M: col0[i] = M[i][0]
};

__device__ __forceinline__ void quad_rc_copy(QuadRc &t) {
    const u64 *src = &RC_SPLIT[0][0][0];
    u64 *dst = &t.rc[0][0][0];
    constexpr int n = (ROUNDS + 1) * WIDTH * 2;
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
    if (threadIdx.x < WIDTH) t.col0[threadIdx.x] = GOLDI_MDS[threadIdx.x][0];
}

// Fills the LDS copy of the table; every thread of the block must call it.
__device__ __forceinline__ void quad_rc_load(QuadRc &t) {
    quad_rc_copy(t);
    __syncthreads();
}

#if GOLDI_USE_BLOCKS
// Partial rounds three at a time (the block form of poseidon.hpp: A_m =
// (M P)^m, f_m the S-box columns, K_m the constants).  Lane q computes rows
// 3q .. 3q+2 of the state after the block from the quad's 12 words; A_3 is
// not circulant, so its entries differ per lane and come from LDS.  The two
// chained S-box inputs are row 0 of A_1 and A_2 (plus S-box terms): each
// lane takes its own three words' share, and two DPP steps sum the shares
// over the quad, so every lane ends up with the same S-box outputs and no
// broadcast is needed after the first.
struct QuadBlk {
    u32 a[4][3][WIDTH];             // [q][R][3D + K] = A_3[3q + R][3((q + D) mod 4) + K]
    u32 c[4][GOLDI_BLK - 1][3];     // [q][m - 1][K] = A_m[0][3q + K]
    u32 f[4][3][GOLDI_BLK];         // [q][R][m] = f_3[3q + R][m]
    u64 k[GOLDI_BLK_N][4][3 + GOLDI_BLK - 1][2];  // rows 3q + R, then the chain's (in lane 0; zero elsewhere)
};

constexpr QuadBlk make_quad_blk() {
    QuadBlk t{};
    constexpr u64 blk_k[GOLDI_BLK_N][GOLDI_BLK - 1 + WIDTH][2] = GOLDI_BLK_K_INIT;
    for (int q = 0; q < 4; q++) {
        for (int r = 0; r < 3; r++) {
            for (int d = 0; d < 4; d++)
                for (int k = 0; k < 3; k++) t.a[q][r][3 * d + k] = GOLDI_BLK_A[GOLDI_BLK - 1][3 * q + r][3 * ((q + d) % 4) + k];
            for (int m = 0; m < GOLDI_BLK; m++) t.f[q][r][m] = GOLDI_BLK_F[GOLDI_BLK - 1][3 * q + r][m];
        }
        for (int m = 1; m < GOLDI_BLK; m++)
            for (int k = 0; k < 3; k++) t.c[q][m - 1][k] = GOLDI_BLK_A[m - 1][0][3 * q + k];
        for (int b = 0; b < GOLDI_BLK_N; b++)
            for (int h = 0; h < 2; h++) {
                for (int r = 0; r < 3; r++) t.k[b][q][r][h] = blk_k[b][GOLDI_BLK - 1 + 3 * q + r][h];
                for (int m = 1; m < GOLDI_BLK; m++) t.k[b][q][2 + m][h] = q == 0 ? blk_k[b][m - 1][h] : 0;
            }
    }
    return t;
}

__constant__ QuadBlk QUAD_BLK_C = make_quad_blk();

__device__ __forceinline__ u64 quad_bcast0(u64 v) {  // lane 0 of the quad, quad_perm [0,0,0,0]
    return mk64((u32)__builtin_amdgcn_mov_dpp((int)lo32(v), 0x00, 0xF, 0xF, false),
                (u32)__builtin_amdgcn_mov_dpp((int)hi32(v), 0x00, 0xF, 0xF, false));
}

// a += sum over j < M of f_M[0][j] S_j (uniform entries).
template <int M, int J = 0>
__device__ __forceinline__ void quad_chain_sterms(const u64 (&s)[GOLDI_BLK], u64 &a_lo, u64 &a_hi) {
    if constexpr (J < M) {
        constexpr unsigned C = GOLDI_BLK_F[M - 1][0][J];
        a_lo = mad_coef<C>(lo32(s[J]), a_lo);
        a_hi = mad_coef<C>(hi32(s[J]), a_hi);
        quad_chain_sterms<M, J + 1>(s, a_lo, a_hi);
    }
}

// S-box outputs M .. GOLDI_BLK-1 of the block from the quad sums p of the
// chain rows.
template <int M>
__device__ __forceinline__ void quad_chain(u64 (&s)[GOLDI_BLK], const u64 (&p_lo)[GOLDI_BLK - 1],
                                           const u64 (&p_hi)[GOLDI_BLK - 1]) {
    if constexpr (M < GOLDI_BLK) {
        u64 a_lo = p_lo[M - 1], a_hi = p_hi[M - 1];
        quad_chain_sterms<M>(s, a_lo, a_hi);
        s[M] = sbox_blocks(reduce_split_c(a_lo, a_hi));
        quad_chain<M + 1>(s, p_lo, p_hi);
    }
}

// GOLDI_BLK partial rounds from a state holding its round constant.
__device__ __forceinline__ void quad_block(u64 w[3], int q, const QuadBlk &qb, int b) {
    u64 x[4][3];
#pragma unroll
    for (int k = 0; k < 3; k++) {
        x[0][k] = w[k];
        x[1][k] = quad_fetch64<1>(w[k]);
        x[2][k] = quad_fetch64<2>(w[k]);
        x[3][k] = quad_fetch64<3>(w[k]);
    }
    u64 s[GOLDI_BLK];
    s[0] = sbox_blocks(w[0]);  // the block's first S-box (lane 0's word 0)
    // This lane's share of the chain rows, then the sum over the quad.
    u64 p_lo[GOLDI_BLK - 1], p_hi[GOLDI_BLK - 1];
#pragma unroll
    for (int m = 0; m < GOLDI_BLK - 1; m++) {
        p_lo[m] = qb.k[b][q][3 + m][0];
        p_hi[m] = qb.k[b][q][3 + m][1];
#pragma unroll
        for (int k = 0; k < 3; k++) {
            p_lo[m] = mad32(qb.c[q][m][k], lo32(w[k]), p_lo[m]);
            p_hi[m] = mad32(qb.c[q][m][k], hi32(w[k]), p_hi[m]);
        }
    }
#pragma unroll
    for (int m = 0; m < GOLDI_BLK - 1; m++) {
        p_lo[m] += quad_fetch64<1>(p_lo[m]);
        p_hi[m] += quad_fetch64<1>(p_hi[m]);
        p_lo[m] += quad_fetch64<2>(p_lo[m]);
        p_hi[m] += quad_fetch64<2>(p_hi[m]);
    }
    u64 a_lo[3], a_hi[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        a_lo[r] = qb.k[b][q][r][0];
        a_hi[r] = qb.k[b][q][r][1];
#pragma unroll
        for (int d = 0; d < 4; d++)
#pragma unroll
            for (int k = 0; k < 3; k++) {
                a_lo[r] = mad32(qb.a[q][r][3 * d + k], lo32(x[d][k]), a_lo[r]);
                a_hi[r] = mad32(qb.a[q][r][3 * d + k], hi32(x[d][k]), a_hi[r]);
            }
    }
    s[0] = quad_bcast0(s[0]);
    quad_chain<1>(s, p_lo, p_hi);
#pragma unroll
    for (int r = 0; r < 3; r++) {
#pragma unroll
        for (int m = 0; m < GOLDI_BLK; m++) {
            a_lo[r] = mad32(qb.f[q][r][m], lo32(s[m]), a_lo[r]);
            a_hi[r] = mad32(qb.f[q][r][m], hi32(s[m]), a_hi[r]);
        }
        w[r] = reduce_split_c(a_lo[r], a_hi[r]);
    }
}
#endif

// The quad kernels' LDS table: round constants and, with blocks, the
// per-lane block entries.
struct QuadTab : QuadRc {
#if GOLDI_USE_BLOCKS
    QuadBlk blk;
#endif
};

__device__ __forceinline__ void quad_tab_load(QuadTab &t) {
    quad_rc_copy(t);
#if GOLDI_USE_BLOCKS
    static_assert(sizeof(QuadBlk) % 8 == 0, "copied as 64-bit words");
    const u64 *src = reinterpret_cast<const u64 *>(&QUAD_BLK_C);
    u64 *dst = reinterpret_cast<u64 *>(&t.blk);
    constexpr int n = sizeof(QuadBlk) / 8;
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = src[i];
#endif
    __syncthreads();
}

// Permutes the state spread over the quad; q = lane index in the quad.
// All 4 lanes of the quad must be active.
__device__ __forceinline__ void permute_quad(u64 w[3], int q, const QuadTab &t) {
#pragma unroll
    for (int k = 0; k < 3; k++) {
        const u64 *c = t.rc[0][3 * q + k];
        w[k] = add_weak(w[k], mk64(lo32(c[0]), lo32(c[1])));
    }
#pragma nounroll
    for (int r = 0; r < HALF_FULL; r++) {
        sbox3_blocks(w[0], w[1], w[2]);
        quad_mds_add_rc(w, t.rc[r + 1] + 3 * q);
    }
    const u32 nz = q == 0 ? 0u : 0xFFFFFFFFu;
    u32 m0[3];
#pragma unroll
    for (int r = 0; r < 3; r++) m0[r] = t.col0[3 * q + r];
#if GOLDI_USE_BLOCKS
    // The first partial round alone, then the blocks (the block constants
    // start from the round after it).
    quad_partial_round(w, t.rc[HALF_FULL + 1] + 3 * q, nz, m0);
#pragma nounroll
    for (int b = 0; b < GOLDI_BLK_N; b++) quad_block(w, q, t.blk, b);
    constexpr int FIRST_SINGLE = GOLDI_BLK_FIRST_TAIL;
#else
    constexpr int FIRST_SINGLE = HALF_FULL;
#endif
#pragma nounroll
    for (int r = FIRST_SINGLE; r < HALF_FULL + PARTIAL; r++) quad_partial_round(w, t.rc[r + 1] + 3 * q, nz, m0);
#pragma nounroll
    for (int r = HALF_FULL + PARTIAL; r < ROUNDS; r++) {
        sbox3_blocks(w[0], w[1], w[2]);
        quad_mds_add_rc(w, t.rc[r + 1] + 3 * q);
    }
}

}  // namespace goldi
