// Poseidon-12 permutation over Goldilocks, one state per lane, on gfx950.
//
// Structure (Sec. 2.4, Alg. 1): a 12-word state, HALF_FULL_ROUNDS = 4 full
// rounds, PARTIAL_ROUNDS = 22 partial rounds, 4 full rounds; S-box x^7; a
// 12 x 12 matrix with small entries (Table 1's 8-bit mult_72 / mmult_4x12_8).
// Round r adds C[r], applies the S-box (to all words in a full round, to word
// 0 in a partial round) and multiplies by M.  The constant of round r + 1 is
// folded into the matrix product of round r, so each round costs one pass.
//
// Layout: the state lives in 24 VGPRs (12 x (lo, hi)); the matrix entries
// are inline constants of the multiply-adds; the round constants are read
// per round with scalar loads from a small constant table (wave-uniform, so
// they land in SGPRs).  The round loops are not unrolled: one full-round body
// and one partial-round body keep the code small enough for the instruction
// cache, which a fully unrolled permutation (~17k instructions) would not.
//
// Partial rounds use the dense matrix too.  Alg. 1 instead multiplies by a
// sparse matrix (MDSPartial) with full-size 64-bit entries.  On gfx950 the
// 32x32 multiply-add issues at the full VALU rate, and a dense product with
// 6-bit entries costs 2 multiply-adds per term, so the dense form costs about
// as much as the sparse one while needing no derived constants.
#pragma once
#include "field.hpp"
#ifdef GOLDI_CONSTANTS_INC
#include GOLDI_CONSTANTS_INC  // a special instance for closed-form tests
#else
#include "poseidon12_constants.inc"
#endif

namespace goldi {

static constexpr int WIDTH = 12;
static constexpr int RATE = 8;
static constexpr int DIGEST = 4;
static constexpr int HALF_FULL = 4;
static constexpr int PARTIAL = 22;
static constexpr int ROUNDS = 2 * HALF_FULL + PARTIAL;

// Round constants, split into 32-bit halves held in 64-bit words (see the
// generator); row ROUNDS is zero.
__constant__ u64 RC_SPLIT[ROUNDS + 1][WIDTH][2] = GOLDI_RC_SPLIT_INIT;

__device__ __forceinline__ u64 sbox(u64 x) {
    const u64 x2 = sqr(x);
    const u64 x3 = mul(x2, x);
    const u64 x4 = sqr(x2);
    return mul(x4, x3);
}

// V = a_lo + a_hi 2^32 with a_lo, a_hi < 2^43, reduced to a weak word:
// V = w2 2^64 + (w1 2^32 + lo32(a_lo)) with w1 = hi32(a_lo) + lo32(a_hi)
// and w2 = hi32(a_hi) + carry, then 2^64 = 2^32 - 1.
__device__ __forceinline__ u64 reduce_split(u64 a_lo, u64 a_hi) {
    u32 c, junk;
    const u32 w1 = __builtin_addc(hi32(a_lo), lo32(a_hi), 0u, &c);
    const u32 w2 = __builtin_addc(hi32(a_hi), 0u, c, &junk);
    return mad_eps_fold(w2, mk64(lo32(a_lo), w1));
}

// m * x + acc for a matrix entry m (an inline constant, 1..64) as exactly
// one v_mad_u64_u32; left to itself the compiler turns some entries (powers
// of two) into longer shift-and-mask sequences on the 64-bit pair.
#ifndef GOLDI_MDS_ASM
#define GOLDI_MDS_ASM 1  // 0: plain C++ for non-powers of two, 2: always plain C++
#endif
template <unsigned M>
__device__ __forceinline__ u64 mad_small(u32 x, u64 acc) {
    static_assert(M <= 64, "matrix entries are inline constants");
    if constexpr (M == 0) {
        return acc;
    } else if constexpr (GOLDI_MDS_ASM == 2 || (GOLDI_MDS_ASM == 0 && (M & (M - 1)) != 0)) {
        return mad32(x, M, acc);
    } else {
        u64 r;
        asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(r) : "v"(x), "i"(M), "v"(acc) : "vcc");
        return r;
    }
}

// The same with the accumulator in a scalar register pair: the first term of
// a row adds the round constant straight from the SGPRs it was loaded into
// (a VOP3 operand may be scalar), instead of copying it to VGPRs first.
template <unsigned M>
__device__ __forceinline__ u64 mad_small_sacc(u32 x, u64 acc) {
    static_assert(M <= 64, "matrix entries are inline constants");
    if constexpr (M == 0 || GOLDI_MDS_ASM != 1) {
        return mad_small<M>(x, acc);
    } else {
        u64 r;
        asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(r) : "v"(x), "i"(M), "s"(acc) : "vcc");
        return r;
    }
}

// Terms are accumulated for words 1..11 first and word 0 last: in a partial
// round only word 0 went through the S-box, so the other eleven products can
// issue while its S-box chain is still running.
template <int I, int K>
__device__ __forceinline__ void mds_term(const u64 s[WIDTH], u64 &a_lo, u64 &a_hi) {
    constexpr int J = (K + 1) % WIDTH;
    a_lo = mad_small<GOLDI_MDS[I][J]>(lo32(s[J]), a_lo);
    a_hi = mad_small<GOLDI_MDS[I][J]>(hi32(s[J]), a_hi);
    if constexpr (K + 1 < WIDTH) mds_term<I, K + 1>(s, a_lo, a_hi);
}

template <int I, int END>
__device__ __forceinline__ void mds_rows(const u64 s[WIDTH], u64 out[WIDTH], const u64 (*rc)[2]) {
    constexpr int J = 1;  // the first word of mds_term's order
    u64 a_lo = mad_small_sacc<GOLDI_MDS[I][J]>(lo32(s[J]), rc[I][0]);
    u64 a_hi = mad_small_sacc<GOLDI_MDS[I][J]>(hi32(s[J]), rc[I][1]);
    mds_term<I, 1>(s, a_lo, a_hi);
    out[I] = reduce_split(a_lo, a_hi);
    if constexpr (I + 1 < END) mds_rows<I + 1, END>(s, out, rc);
}

#ifndef GOLDI_RC_GROUP
#define GOLDI_RC_GROUP 6  // rows per batch of round-constant loads
#endif

template <int I0>
__device__ __forceinline__ void mds_row_group(const u64 s[WIDTH], u64 out[WIDTH], int r1) {
    constexpr int I1 = I0 + GOLDI_RC_GROUP < WIDTH ? I0 + GOLDI_RC_GROUP : WIDTH;
    u64 rc[WIDTH][2];
#pragma unroll
    for (int i = I0; i < I1; i++) {
        rc[i][0] = RC_SPLIT[r1][i][0];
        rc[i][1] = RC_SPLIT[r1][i][1];
    }
    mds_rows<I0, I1>(s, out, rc);
    if constexpr (I1 < WIDTH) mds_row_group<I1>(s, out, r1);
}

// s <- M s + C[r1]  (C[ROUNDS] = 0).  The constants of a group of rows are
// read together (wave-uniform scalar loads), so one wait covers the group.
__device__ __forceinline__ void mds_add_rc(u64 s[WIDTH], int r1) {
    u64 out[WIDTH];
    mds_row_group<0>(s, out, r1);
#pragma unroll
    for (int i = 0; i < WIDTH; i++) s[i] = out[i];
}

__device__ __forceinline__ void full_round(u64 s[WIDTH], int r) {
#pragma unroll
    for (int i = 0; i < WIDTH; i++) s[i] = sbox(s[i]);
    mds_add_rc(s, r + 1);
}

__device__ __forceinline__ void partial_round(u64 s[WIDTH], int r) {
    s[0] = sbox(s[0]);
    mds_add_rc(s, r + 1);
}

// In place; input words must be < 2^64 (any word), output words are weak.
__device__ __forceinline__ void permute(u64 s[WIDTH]) {
#pragma unroll
    for (int i = 0; i < WIDTH; i++) s[i] = add_weak(s[i], mk64(lo32(RC_SPLIT[0][i][0]), lo32(RC_SPLIT[0][i][1])));
#pragma nounroll
    for (int r = 0; r < HALF_FULL; r++) full_round(s, r);
#ifndef GOLDI_PARTIAL_UNROLL
#define GOLDI_PARTIAL_UNROLL 2
#endif
#pragma unroll GOLDI_PARTIAL_UNROLL
    for (int r = HALF_FULL; r < HALF_FULL + PARTIAL; r++) partial_round(s, r);
#pragma nounroll
    for (int r = HALF_FULL + PARTIAL; r < ROUNDS; r++) full_round(s, r);
}

}  // namespace goldi
