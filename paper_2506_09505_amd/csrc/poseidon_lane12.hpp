// Poseidon-12 permutation with one state word per lane, for the most
// latency-bound launches (the top levels of a tree, tiny trees).
//
// A 64-lane wave holds four states, one per 16-lane row: word i of a state is
// in lane 16s + i (i < 12).  A round costs each lane one S-box and one row of
// the matrix product, row i = sum_j M[i][j] x_j, over the row's words
// broadcast one at a time with the DPP row broadcast (v_mov_b64_dpp
// row_newbcast:j copies lane j of each row to the whole row: one VALU
// instruction, no LDS round trip); each lane holds its own row of
// coefficients in registers.
//
// Partial rounds go three at a time in the block form of the one-lane
// permutation (A_m = (M P)^m, f_m the S-box columns): lanes 0..11 take row i
// of A_3 and f_3, and the idle lanes 12 and 13 of each row take row 0 of A_1
// and A_2, so the block's two chained S-box inputs come out of the same
// multiply-adds as the state after it.  A block is then one pass over the
// words plus three S-boxes, each broadcast from the lane that computed it
// (0, 12, 13) and added in with the lane's f coefficient.  The first partial
// round rides on the last opening round: lanes 0..11 take the rows of M P M,
// lane 12 row 0 of M, whose result is that partial round's S-box input.
// Lanes 14 and 15 only follow along: their rows copy a helper lane's, and
// nothing reads their results.
#pragma once
#include "poseidon_quad.hpp"

namespace goldi {

// Per-lane coefficient rows and constants, indexed by the lane in its
// 16-lane row, built at compile time from the instance's matrices.
struct Lane12Const {
    u32 m[16][WIDTH];  // row i of M (lanes >= 12: row 0)
#if GOLDI_USE_BLOCKS
    u32 lead[16][WIDTH];  // row i of M P M (lanes < 12), row 0 of M (other lanes)
    u32 f_lead[16];       // M[i][0]: the lead's S-box term (lanes < 12)
    u32 blk[16][WIDTH];   // row i of A_3 (lanes < 12), row 0 of A_m (lane 11 + m)
    u32 f[16][GOLDI_BLK];  // the S-box columns of the same rows
    u64 k_lead[16][2];    // constants, split as RC_SPLIT
    u64 k_blk[GOLDI_BLK_N][16][2];
#endif
};

#if GOLDI_USE_BLOCKS
static_assert(WIDTH + GOLDI_BLK - 1 <= 16, "the chain rows need a free lane each");
#endif

constexpr Lane12Const make_lane12_const() {
    Lane12Const c{};
#if GOLDI_USE_BLOCKS
    constexpr u64 rc[ROUNDS + 1][WIDTH][2] = GOLDI_RC_SPLIT_INIT;
    constexpr u64 lead_k[WIDTH][2] = GOLDI_BLK_LEAD_K_INIT;
    constexpr u64 blk_k[GOLDI_BLK_N][GOLDI_BLK - 1 + WIDTH][2] = GOLDI_BLK_K_INIT;
#endif
    for (int l = 0; l < 16; l++) {
        const int i = l < WIDTH ? l : 0;
        for (int j = 0; j < WIDTH; j++) c.m[l][j] = GOLDI_MDS[i][j];
#if GOLDI_USE_BLOCKS
        // Block rows: lanes < 12 the state after the block (m = GOLDI_BLK),
        // lane 11 + m the S-box input of the block's round m; lanes past the
        // chain repeat lane 12's row.
        const int m = l < WIDTH ? GOLDI_BLK : (l - WIDTH + 1 < GOLDI_BLK ? l - WIDTH + 1 : 1);
        const int row = l < WIDTH ? l : 0;
        const int kidx = l < WIDTH ? GOLDI_BLK - 1 + l : m - 1;
        for (int j = 0; j < WIDTH; j++) {
            c.lead[l][j] = l < WIDTH ? GOLDI_BLK_LEAD_B[l][j] : GOLDI_MDS[0][j];
            c.blk[l][j] = GOLDI_BLK_A[m - 1][row][j];
        }
        for (int k = 0; k < GOLDI_BLK; k++) c.f[l][k] = GOLDI_BLK_F[m - 1][row][k];
        c.f_lead[l] = l < WIDTH ? GOLDI_MDS[l][0] : 0;
        for (int h = 0; h < 2; h++) {
            c.k_lead[l][h] = l < WIDTH ? lead_k[l][h] : rc[HALF_FULL][0][h];
            for (int b = 0; b < GOLDI_BLK_N; b++) c.k_blk[b][l][h] = blk_k[b][kidx][h];
        }
#endif
    }
    return c;
}

__constant__ Lane12Const LANE12_C = make_lane12_const();

struct Lane12 {
    int i;          // lane in the 16-lane row: word i for i < 12, a helper lane above
    int w;          // the word whose round constants the lane takes (i, or 0)
    u32 m[WIDTH];   // this lane's row of M
#if GOLDI_USE_BLOCKS
    u32 b[WIDTH];   // this lane's block row (column 0 is zero)
    u32 f[GOLDI_BLK];
    u32 f_lead;     // M[i][0] (lanes < 12): the lead's S-box term
#endif
};

__device__ __forceinline__ Lane12 lane12_setup(const QuadRc &) {
    Lane12 L;
    L.i = threadIdx.x & 15;
    L.w = L.i < WIDTH ? L.i : 0;
#pragma unroll
    for (int j = 0; j < WIDTH; j++) L.m[j] = LANE12_C.m[L.i][j];
#if GOLDI_USE_BLOCKS
#pragma unroll
    for (int j = 0; j < WIDTH; j++) L.b[j] = LANE12_C.blk[L.i][j];
#pragma unroll
    for (int k = 0; k < GOLDI_BLK; k++) L.f[k] = LANE12_C.f[L.i][k];
    L.f_lead = LANE12_C.f_lead[L.i];
#endif
    return L;
}

// Word J of this lane's 16-lane row, in every lane of the row.
template <int J>
__device__ __forceinline__ u64 row_bcast(u64 v) {
    static_assert(J >= 0 && J < 16, "a lane of the row");
    return __builtin_amdgcn_mov_dpp(v, 0x150 + J, 0xf, 0xf, false);
}

// a += sum_(j = J..J1-1) c[j] x_j over the words x_j of the row of v.
template <int J, int J1>
__device__ __forceinline__ void row_terms(u64 v, const u32 (&c)[WIDTH], u64 &a_lo, u64 &a_hi) {
    const u64 y = row_bcast<J>(v);
    a_lo = mad32(c[J], lo32(y), a_lo);
    a_hi = mad32(c[J], hi32(y), a_hi);
    if constexpr (J + 1 < J1) row_terms<J + 1, J1>(v, c, a_lo, a_hi);
}

// Full round: x <- row i of M S(x) + C[r + 1][i].
__device__ __forceinline__ u64 lane12_full(u64 x, const u32 (&c)[WIDTH], const u64 *k) {
    const u64 s = sbox_blocks(x);
    u64 a_lo = k[0], a_hi = k[1];
    row_terms<0, WIDTH>(s, c, a_lo, a_hi);
    return reduce_split_c(a_lo, a_hi);
}

// Partial round: word 0's S-box runs while the other words' terms add up;
// its output is broadcast from lane 0 and added last.
__device__ __forceinline__ u64 lane12_partial(u64 x, const u32 (&c)[WIDTH], const u64 *k) {
    const u64 s = sbox_blocks(x);
    u64 a_lo = k[0], a_hi = k[1];
    row_terms<1, WIDTH>(x, c, a_lo, a_hi);
    const u64 sb = row_bcast<0>(s);
    a_lo = mad32(c[0], lo32(sb), a_lo);
    a_hi = mad32(c[0], hi32(sb), a_hi);
    return reduce_split_c(a_lo, a_hi);
}

#if GOLDI_USE_BLOCKS
// The last opening full round with the first partial round: lane 12 takes
// row 0 of M, that round's S-box input u; lanes < 12 take the rows of
// M P M and then add M[i][0] S(u).  c and k: this lane's lead row and
// constant.
__device__ __forceinline__ u64 lane12_lead(u64 x, const Lane12 &L, const u32 (&c)[WIDTH], const u64 (&k)[2]) {
    const u64 s = sbox_blocks(x);
    u64 a_lo = k[0], a_hi = k[1];
    row_terms<0, WIDTH>(s, c, a_lo, a_hi);
    const u64 su = row_bcast<WIDTH>(sbox_blocks(reduce_split_c(a_lo, a_hi)));
    a_lo = mad32(L.f_lead, lo32(su), a_lo);
    a_hi = mad32(L.f_lead, hi32(su), a_hi);
    return reduce_split_c(a_lo, a_hi);
}

// S-box outputs M .. GOLDI_BLK-1 of the block: the S-box input of round M
// is lane 11 + M's row reduced; its output is broadcast from there.
template <int M>
__device__ __forceinline__ void lane12_chain(const Lane12 &L, u64 &a_lo, u64 &a_hi) {
    if constexpr (M < GOLDI_BLK) {
        const u64 sb = row_bcast<WIDTH + M - 1>(sbox_blocks(reduce_split_c(a_lo, a_hi)));
        a_lo = mad32(L.f[M], lo32(sb), a_lo);
        a_hi = mad32(L.f[M], hi32(sb), a_hi);
        lane12_chain<M + 1>(L, a_lo, a_hi);
    }
}

// GOLDI_BLK partial rounds from a state holding its round constant; k is
// this lane's constant of the block.
__device__ __forceinline__ u64 lane12_block(u64 x, const Lane12 &L, const u64 (&k)[2]) {
    const u64 s = sbox_blocks(x);
    u64 a_lo = k[0], a_hi = k[1];
    row_terms<1, WIDTH>(x, L.b, a_lo, a_hi);
    const u64 sb = row_bcast<0>(s);
    a_lo = mad32(L.f[0], lo32(sb), a_lo);
    a_hi = mad32(L.f[0], hi32(sb), a_hi);
    lane12_chain<1>(L, a_lo, a_hi);
    return reduce_split_c(a_lo, a_hi);
}
#endif

// Permutes the four states of the wave; every lane of the wave must be
// active (the row broadcasts read other lanes).
__device__ __forceinline__ u64 permute_lane12(u64 x, const Lane12 &L, const QuadRc &t) {
    x = add_weak(x, mk64(lo32(t.rc[0][L.w][0]), lo32(t.rc[0][L.w][1])));
#if GOLDI_USE_BLOCKS
    // The last opening round carries the first partial round.  Every
    // constant a lane reads from global memory is loaded a round or a block
    // before its use, so that no multiply-add waits for memory.
    constexpr int OPEN = HALF_FULL - 1;
#pragma nounroll
    for (int r = 0; r < OPEN - 1; r++) x = lane12_full(x, L.m, t.rc[r + 1][L.w]);
    u32 c[WIDTH];
#pragma unroll
    for (int j = 0; j < WIDTH; j++) c[j] = LANE12_C.lead[L.i][j];
    const u64 k[2] = {LANE12_C.k_lead[L.i][0], LANE12_C.k_lead[L.i][1]};
    x = lane12_full(x, L.m, t.rc[OPEN][L.w]);
    u64 kb[2] = {LANE12_C.k_blk[0][L.i][0], LANE12_C.k_blk[0][L.i][1]};
    x = lane12_lead(x, L, c, k);
#pragma nounroll
    for (int b = 0; b < GOLDI_BLK_N; b++) {
        const int bn = b + 1 < GOLDI_BLK_N ? b + 1 : b;
        const u64 kn[2] = {LANE12_C.k_blk[bn][L.i][0], LANE12_C.k_blk[bn][L.i][1]};
        x = lane12_block(x, L, kb);
        kb[0] = kn[0];
        kb[1] = kn[1];
    }
    constexpr int FIRST_SINGLE = GOLDI_BLK_FIRST_TAIL;
#else
#pragma nounroll
    for (int r = 0; r < HALF_FULL; r++) x = lane12_full(x, L.m, t.rc[r + 1][L.w]);
    constexpr int FIRST_SINGLE = HALF_FULL;
#endif
#pragma nounroll
    for (int r = FIRST_SINGLE; r < HALF_FULL + PARTIAL; r++) x = lane12_partial(x, L.m, t.rc[r + 1][L.w]);
#pragma nounroll
    for (int r = HALF_FULL + PARTIAL; r < ROUNDS; r++) x = lane12_full(x, L.m, t.rc[r + 1][L.w]);
    return x;
}

}  // namespace goldi
