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
// Partial rounds: by default three at a time, as one product with the
// 32-bit integer matrix (M P)^3 (P zeroes word 0) plus the block's S-box
// outputs times integer columns, the first partial round riding on the last
// opening round's matrix.  A v_mad_u64_u32 costs the same for a 26-bit entry
// as for a 6-bit one, so a block of three costs about 1.3 dense rounds.  The
// sparse form of Alg. 1 (MDSPartial: one pre-matrix, then per round the
// identity apart from a full first row and column with 64-bit entries) and
// the dense form (the textbook matrix every round) stay selectable with
// GOLDI_PARTIAL_FORM=1 and 0; they measured slower on MI355X.
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
// For a state whose words 8..11 are zero (a sponge's first absorption, a tree
// node): those words enter round 0 as C[0][8..11], so their S-box outputs
// and matrix terms are constants; row i's constant becomes
// C[1][i] + sum_k M[i][8+k] C[0][8+k]^7 (mod p), split like RC_SPLIT.
__constant__ u64 CAP0_RC1[WIDTH][2] = GOLDI_CAP0_RC1_INIT;

// S-box x^7 = x^4 x^3 with x^2 = x x, x^3 = x^2 x, x^4 = x^2 x^2 (Alg. 1).
// Each product is a few small statements, so the compiler can interleave the
// S-box with independent work (the matrix terms of the other words).
__device__ __forceinline__ u64 sbox(u64 x) {
    const u64 x2 = sqr(x);
    const u64 x3 = mul(x2, x);
    const u64 x4 = sqr(x2);
    return mul(x4, x3);
}

// One S-box with its four products as asm blocks (field_asm.inc): x^2
// alone, x^3 and x^4 interleaved, x^7 alone.  Where few waves share a SIMD
// (the narrow layouts' single S-boxes) this spends only the wait states each
// carry read needs: 2 per block, against about 7 per statement-level product,
// whose asm statements the compiler pads.
__device__ __forceinline__ u64 sbox_blocks(u64 x) {
    u64 x2, x3, x4, x7;
    sqr1_asm(x, x2);
    mul2_asm(x2, x, x2, x2, x3, x4);
    mul1_asm(x4, x3, x7);
    return x7;
}

// Three independent S-boxes, each stage as one block of three interleaved
// products (field_asm.inc): no wait state is spent on a carry.  Measured on
// MI355X this helps where a lane holds three words and few waves share a
// SIMD (the four-lanes-per-state layout) and costs 1-1.5% in the one-lane
// layout, whose other waves already hide the wait states.
__device__ __forceinline__ void sbox3_blocks(u64 &x, u64 &y, u64 &z) {
    u64 x2, y2, z2, x3, y3, z3, x4, y4, z4;
    sqr3_asm(x, y, z, x2, y2, z2);
    mul3_asm(x2, x, y2, y, z2, z, x3, y3, z3);
    sqr3_asm(x2, y2, z2, x4, y4, z4);
    mul3_asm(x4, x3, y4, y3, z4, z3, x, y, z);
}

// V = a_lo + a_hi 2^32 with a_lo, a_hi < 2^63 (every row accumulator of
// this library stays below 2^58), reduced to a weak word.  With
// a_hi = h1 2^32 + h0 and 2^64 = 2^32 - 1 (mod p):
//     V = (a_lo + h1 (2^32 - 1)) + h0 2^32.
// The bracket is one multiply-add and cannot overflow (h1 < 2^31).  Adding
// h0 into its high word may carry out of 64 bits; the wrapped word is then
// below 2^64 - 2^32, so the carry's 2^32 - 1 is added back with a
// multiply-add that cannot overflow.  Four instructions.
__device__ __forceinline__ u64 reduce_split(u64 a_lo, u64 a_hi) {
    u64 r;
    asm("v_mad_u64_u32 %0, vcc, %1, -1, %2" : "=v"(r) : "v"(hi32(a_hi)), "v"(a_lo) : "vcc");
    u32 s_hi, c;
    asm("v_add_co_u32 %0, vcc, %2, %3\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32 %1, vcc, 0, 0, vcc"
        : "=v"(s_hi), "=v"(c)
        : "v"(hi32(r)), "v"(lo32(a_hi))
        : "vcc");
    u64 out;
    asm("v_mad_u64_u32 %0, vcc, %1, -1, %2" : "=v"(out) : "v"(c), "v"(mk64(lo32(r), s_hi)) : "vcc");
    return out;
}

// reduce_split as compiler-visible code, for the narrow layouts (see
// mad_small_c: no padding after asm statements).
__device__ __forceinline__ u64 reduce_split_c(u64 a_lo, u64 a_hi) {
    const u64 r = mad32(hi32(a_hi), 0xFFFFFFFFu, a_lo);
    const u64 s_hi = (u64)hi32(r) + lo32(a_hi);
    return mad32((u32)(s_hi >> 32), 0xFFFFFFFFu, mk64(lo32(r), (u32)s_hi));
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

// m * x + acc as compiler-visible code, for the narrow layouts: the compiler
// pads each inline-asm statement before a dependent read (it cannot rule out
// a transcendental instruction inside), which costs where few waves share a
// SIMD.  A power-of-two entry goes through an opaque scalar register, so that
// it stays one v_mad_u64_u32 instead of a shift sequence.
template <unsigned M>
__device__ __forceinline__ u64 mad_small_c(u32 x, u64 acc) {
    static_assert(M <= 64, "matrix entries are inline constants");
    if constexpr (M == 0) {
        return acc;
    } else if constexpr ((M & (M - 1)) != 0) {
        return mad32(x, M, acc);
    } else {
        u32 m;
        asm("" : "=s"(m) : "0"(M));
        return mad32(x, m, acc);
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
// Row I over the words 1 .. NW-1 and then 0 (NW = 12: all words; NW = 8:
// the words of a state whose words 8..11 enter as a constant instead).
template <int I, int K, int NW = WIDTH>
__device__ __forceinline__ void mds_term(const u64 s[WIDTH], u64 &a_lo, u64 &a_hi) {
    constexpr int J = (K + 1) % NW;
    a_lo = mad_small<GOLDI_MDS[I][J]>(lo32(s[J]), a_lo);
    a_hi = mad_small<GOLDI_MDS[I][J]>(hi32(s[J]), a_hi);
    if constexpr (K + 1 < NW) mds_term<I, K + 1, NW>(s, a_lo, a_hi);
}

#ifndef GOLDI_MDS_LIMB24
#define GOLDI_MDS_LIMB24 0
#endif

#if GOLDI_MDS_LIMB24
// The full-round matrix on 24-bit multipliers (a test build, measured against
// the 32 x 32 -> 64-bit form below): each word is cut into 22-bit limbs
// l0 = bits 0..21, l1 = bits 22..43, l2 = bits 44..63, and a row's three limb
// sums are 32-bit multiply-adds with 24-bit operands (v_mad_u32_u24); with
// entries of at most 64 a dozen terms stay below 12 * 64 * 2^22 < 2^32.  The
// row is then a0 + a1 2^22 + a2 2^44 = (a0 + a1 2^22) + (a2 2^12) 2^32, reduced
// like the other rows, plus the round constant.
__device__ __forceinline__ void limbs22(u64 x, u32 &l0, u32 &l1, u32 &l2) {
    l0 = lo32(x) & 0x3FFFFFu;
    l1 = __builtin_amdgcn_alignbit(hi32(x), lo32(x), 22) & 0x3FFFFFu;
    l2 = hi32(x) >> 12;
}

template <int I, int END, int NW = WIDTH>
__device__ __forceinline__ void mds_rows(const u64 s[WIDTH], u64 out[WIDTH], const u64 (*rc)[2]) {
    u32 l[WIDTH][3];
#pragma unroll
    for (int j = 0; j < NW; j++) limbs22(s[j], l[j][0], l[j][1], l[j][2]);
    u32 a[3] = {0, 0, 0};
#pragma unroll
    for (int j = 0; j < NW; j++) {
#pragma unroll
        for (int k = 0; k < 3; k++) a[k] = l[j][k] * GOLDI_MDS[I][j] + a[k];  // operands below 2^24: v_mad_u32_u24
    }
    const u64 a_lo = (u64)a[0] + ((u64)a[1] << 22);
    const u64 a_hi = (u64)a[2] << 12;
    out[I] = add_weak(reduce_split(a_lo, a_hi), mk64(lo32(rc[I][0]), lo32(rc[I][1])));
    if constexpr (I + 1 < END) mds_rows<I + 1, END, NW>(s, out, rc);
}
#else
template <int I, int END, int NW = WIDTH>
__device__ __forceinline__ void mds_rows(const u64 s[WIDTH], u64 out[WIDTH], const u64 (*rc)[2]) {
    constexpr int J = 1;  // the first word of mds_term's order
    u64 a_lo = mad_small_sacc<GOLDI_MDS[I][J]>(lo32(s[J]), rc[I][0]);
    u64 a_hi = mad_small_sacc<GOLDI_MDS[I][J]>(hi32(s[J]), rc[I][1]);
    mds_term<I, 1, NW>(s, a_lo, a_hi);
    out[I] = reduce_split(a_lo, a_hi);
    if constexpr (I + 1 < END) mds_rows<I + 1, END, NW>(s, out, rc);
}
#endif

#ifndef GOLDI_RC_GROUP
#define GOLDI_RC_GROUP 4  // rows per batch of round-constant loads (2, 3, 4, 6, 12 measured; 4 best)
#endif

// Rows I0..11 with the per-row constants tbl[i] (split as in RC_SPLIT).
template <int I0, int NW = WIDTH>
__device__ __forceinline__ void mds_row_group(const u64 s[WIDTH], u64 out[WIDTH], const u64 (*tbl)[2]) {
    constexpr int I1 = I0 + GOLDI_RC_GROUP < WIDTH ? I0 + GOLDI_RC_GROUP : WIDTH;
    u64 rc[WIDTH][2];
#pragma unroll
    for (int i = I0; i < I1; i++) {
        rc[i][0] = tbl[i][0];
        rc[i][1] = tbl[i][1];
    }
    mds_rows<I0, I1, NW>(s, out, rc);
    if constexpr (I1 < WIDTH) mds_row_group<I1, NW>(s, out, tbl);
}

// s <- M s + C[r1]  (C[ROUNDS] = 0).  The constants of a group of rows are
// read together (wave-uniform scalar loads), so one wait covers the group.
__device__ __forceinline__ void mds_add_rc(u64 s[WIDTH], int r1) {
    u64 out[WIDTH];
    mds_row_group<0>(s, out, RC_SPLIT[r1]);
#pragma unroll
    for (int i = 0; i < WIDTH; i++) s[i] = out[i];
}

__device__ __forceinline__ void full_round(u64 s[WIDTH], int r) {
#pragma unroll
    for (int i = 0; i < WIDTH; i++) s[i] = sbox(s[i]);
    mds_add_rc(s, r + 1);
}

// ---------------------------------------------------------------------------
// Partial rounds in sparse form (Sec. 2.4, Alg. 1): the 11 x 11 block of M
// is conjugated away, so that after one pre-matrix each partial round
// multiplies by a matrix whose first row and first column are full and whose
// rest is the identity, and only word 0 receives a round constant.  The
// constants are derived from C and M by the generator (sparse_form).
//   new x0 = m00 s + sum_i row[i] x_i + k     (s = the S-box output)
//   x_i   += col[i] s                         (i = 1..11)
// Full-width entries come as three 22-bit limbs, so each 32 x 22-bit product
// is below 2^54 and the dozen terms of a dot product add up in six 64-bit
// accumulators without carries; they are combined once.  Rounds go in
// groups: a later round's dot product reads the words from the start of the
// group (plus precomputed scalars times the group's earlier S-box outputs),
// so each word takes all the group's column terms in one reduction, from the
// constant limbs times s, s 2^22 and s 2^44 (mod p).
// GOLDI_PARTIAL_FORM: 2 = blocks of partial rounds (below; the default),
// 1 = the sparse form, 0 = dense.  An instance without the chosen form falls
// back to the next one down.
#ifndef GOLDI_PARTIAL_FORM
#define GOLDI_PARTIAL_FORM 2
#endif
#if GOLDI_PARTIAL_FORM >= 2 && GOLDI_BLOCK_OK
#define GOLDI_USE_BLOCKS 1
#define GOLDI_USE_SPARSE 0
#else
#define GOLDI_USE_BLOCKS 0
#endif
#if !GOLDI_USE_BLOCKS && GOLDI_PARTIAL_FORM >= 1 && GOLDI_SPARSE_OK
#define GOLDI_USE_SPARSE 1
__constant__ u32 SP_K[PARTIAL + 1][3] = GOLDI_SP_K_INIT;
__constant__ u32 SP_CEND[WIDTH - 1][2] = GOLDI_SP_CEND_INIT;
__constant__ u32 SP_ROW[PARTIAL][WIDTH - 1][3] = GOLDI_SP_ROW_INIT;
__constant__ u32 SP_COL22[PARTIAL][WIDTH - 1][3] = GOLDI_SP_COL22_INIT;
__constant__ u32 SP_LAG[PARTIAL][3][3] = GOLDI_SP_LAG_INIT;
__constant__ u32 SP_PRE_M[WIDTH - 1][WIDTH][3] = GOLDI_SP_PRE_M_INIT;
#elif !GOLDI_USE_BLOCKS
#define GOLDI_USE_SPARSE 0
#endif

#if GOLDI_USE_SPARSE
// sum_i x_i c_i with c_i = c_i0 + c_i1 2^22 + c_i2 2^44: a0[j] = sum of
// lo32(x_i) c_ij, a1[j] = sum of hi32(x_i) c_ij.
struct Dot6 {
    u64 a0[3], a1[3];
};

__device__ __forceinline__ void dot_init(Dot6 &d, const u32 (&k)[3]) {
#pragma unroll
    for (int j = 0; j < 3; j++) {
        d.a0[j] = k[j];
        d.a1[j] = 0;
    }
}

__device__ __forceinline__ void dot_term(Dot6 &d, u64 x, const u32 (&c)[3]) {
#pragma unroll
    for (int j = 0; j < 3; j++) {
        d.a0[j] = mad32(lo32(x), c[j], d.a0[j]);
        d.a1[j] = mad32(hi32(x), c[j], d.a1[j]);
    }
}

// (r 2^22 + x) mod p as a weak word, for any words r and x.
__device__ __forceinline__ u64 shl22_add(u64 r, u64 x) {
    u64 lo;
    const bool c = __builtin_add_overflow(r << 22, x, &lo);
    return mad_eps_fold((hi32(r) >> 10) + (u32)c, lo);
}

__device__ __forceinline__ u64 dot_finish(const Dot6 &d) {
    const u64 r0 = reduce_split(d.a0[0], d.a1[0]);
    const u64 r1 = reduce_split(d.a0[1], d.a1[1]);
    const u64 r2 = reduce_split(d.a0[2], d.a1[2]);
    return shl22_add(shl22_add(r2, r1), r0);
}

// r 2^22 mod p as a weak word.
__device__ __forceinline__ u64 shl22(u64 r) { return mad_eps_fold(hi32(r) >> 10, r << 22); }

// z + sum_g c_g x_g (mod p) for G constants c_g (22-bit limbs of the
// first-column entries of partial rounds j .. j+G-1 for word i) and
// sh[g] = {x_g, x_g 2^22, x_g 2^44} (mod p): 6 G products of 32 x 22 bits
// into a low and a high accumulator (each below 3 G 2^54 + 2^32), then one
// split reduction.
template <int G>
__device__ __forceinline__ u64 col_update(u64 z, const u64 (&sh)[G][3], int j, int i) {
    u64 a_lo = mad32(lo32(sh[0][0]), SP_COL22[j][i][0], (u64)lo32(z));
    u64 a_hi = mad32(hi32(sh[0][0]), SP_COL22[j][i][0], (u64)hi32(z));
#pragma unroll
    for (int g = 0; g < G; g++) {
#pragma unroll
        for (int l = (g == 0 ? 1 : 0); l < 3; l++) {
            a_lo = mad32(lo32(sh[g][l]), SP_COL22[j + g][i][l], a_lo);
            a_hi = mad32(hi32(sh[g][l]), SP_COL22[j + g][i][l], a_hi);
        }
    }
    return reduce_split(a_lo, a_hi);
}

// The last opening full round's matrix with the pre-matrix folded in:
// row 0 is M's (plus the scalar k_4), rows 1..11 are diag(1, Mh^22) M.
__device__ __forceinline__ void pre_matrix(const u64 s[WIDTH], u64 out[WIDTH]) {
    const u64 k4[1][2] = {GOLDI_SP_K4_SPLIT};
    mds_rows<0, 1>(s, out, k4);
    // Rows 1..11 one per iteration of a rolled loop (the scalar registers
    // hold one row's 36 constant limbs at a time); each new row enters a
    // shift register, so after the last iteration out[i] holds row i.
#pragma nounroll
    for (int i = 1; i < WIDTH; i++) {
        Dot6 d;
        const u32 zero[3] = {0, 0, 0};
        dot_init(d, zero);
#pragma unroll
        for (int j = 0; j < WIDTH; j++) dot_term(d, s[j], SP_PRE_M[i - 1][j]);
#pragma unroll
        for (int k = 1; k < WIDTH - 1; k++) out[k] = out[k + 1];
        out[WIDTH - 1] = dot_finish(d);
    }
}

// Partial rounds HALF_FULL + j .. HALF_FULL + j + G - 1.  With x_g the
// S-box output of round g of the group, round g's dot product reads the words
// from the start of the group plus sum_h lag * x_h over the group's earlier
// rounds, and each word takes all G column terms in one reduction:
//   x_i += sum_g col_(j+g)[i] x_g.
template <int G>
__device__ __forceinline__ void sparse_group(u64 s[WIDTH], int j) {
    u64 x[G];
    x[0] = sbox(s[0]);
#pragma unroll
    for (int g = 0; g < G; g++) {
        Dot6 d;
        dot_init(d, SP_K[j + g + 1]);
        d.a0[0] = mad_small<GOLDI_MDS[0][0]>(lo32(x[g]), d.a0[0]);
        d.a1[0] = mad_small<GOLDI_MDS[0][0]>(hi32(x[g]), d.a1[0]);
#pragma unroll
        for (int i = 1; i < WIDTH; i++) dot_term(d, s[i], SP_ROW[j + g][i - 1]);
#pragma unroll
        for (int h = 0; h < g; h++) dot_term(d, x[h], SP_LAG[j + g][g - 1 - h]);
        if (g + 1 < G)
            x[g + 1] = sbox(dot_finish(d));
        else
            s[0] = dot_finish(d);
    }
    u64 sh[G][3];
#pragma unroll
    for (int g = 0; g < G; g++) {
        sh[g][0] = x[g];
        sh[g][1] = shl22(x[g]);
        sh[g][2] = shl22(sh[g][1]);
    }
#pragma unroll
    for (int i = 1; i < WIDTH; i++) s[i] = col_update<G>(s[i], sh, j, i - 1);
}
#endif

#if GOLDI_USE_BLOCKS
// ---------------------------------------------------------------------------
// Partial rounds GOLDI_BLK at a time.  With P the projection that zeroes word
// 0 and c0 the first column of M, a partial round maps a state b that holds
// its round constant to M P b + c0 S(b_0) + C[r + 1]; m rounds map it to
//   A_m b + sum_(j<m) f_m[j] S_j + K_m,   A_m = (M P)^m, f_m[j] = A_(m-1-j) c0,
// with S_j the S-box output of round j of the block.  A_m and f_m do not
// depend on the block and, with the instance's 6-bit entries, are integers
// whose rows sum to below 2^26 (the generator checks a bound on every row), so:
//   * the S-box inputs of rounds 1 .. GOLDI_BLK-1 of the block are row 0 of
//     A_m b plus the earlier S-box terms: one dot product each;
//   * the state after the block is one dense product with 32-bit entries,
//     whose dozen-odd 32 x 32-bit products per accumulator stay below 2^58.
// Each product is one v_mad_u64_u32 like the full rounds' 6-bit entries, so a
// block of three rounds costs about as much as 1.3 dense rounds.  Entries
// above 64 are not inline constants; they go into scalar registers (a VOP3
// instruction reads one), and each row's first term, the newest S-box output
// times c0[i] (an inline constant), takes the row's constant as its addend
// straight from the scalar registers it was loaded into.
__constant__ u64 BLK_K[GOLDI_BLK_N][GOLDI_BLK - 1 + WIDTH][2] = GOLDI_BLK_K_INIT;
__constant__ u64 BLK_LEAD_K[WIDTH][2] = GOLDI_BLK_LEAD_K_INIT;

template <unsigned C>
__device__ __forceinline__ u64 mad_coef(u32 x, u64 acc) {
    if constexpr (C <= 64) {
        return mad_small<C>(x, acc);
    } else {
        u64 r;
        asm("v_mad_u64_u32 %0, vcc, %1, %2, %3" : "=v"(r) : "v"(x), "s"(C), "v"(acc) : "vcc");
        return r;
    }
}

// Terms j = J .. 11 of row I of A_M (column 0 is zero).
template <int M, int I, int J = 1>
__device__ __forceinline__ void blk_words(const u64 s[WIDTH], u64 &a_lo, u64 &a_hi) {
    constexpr unsigned C = GOLDI_BLK_A[M - 1][I][J];
    a_lo = mad_coef<C>(lo32(s[J]), a_lo);
    a_hi = mad_coef<C>(hi32(s[J]), a_hi);
    if constexpr (J + 1 < WIDTH) blk_words<M, I, J + 1>(s, a_lo, a_hi);
}

// Terms of the S-box outputs x[J] .. x[0] of row I of f_M.
template <int M, int I, int J>
__device__ __forceinline__ void blk_sterms(const u64 x[GOLDI_BLK], u64 &a_lo, u64 &a_hi) {
    if constexpr (J >= 0) {
        constexpr unsigned C = GOLDI_BLK_F[M - 1][I][J];
        a_lo = mad_coef<C>(lo32(x[J]), a_lo);
        a_hi = mad_coef<C>(hi32(x[J]), a_hi);
        blk_sterms<M, I, J - 1>(x, a_lo, a_hi);
    }
}

// Word I of the state M rounds into the block, as a weak word; k = its
// constant K_M[I] split as RC_SPLIT.
template <int M, int I>
__device__ __forceinline__ u64 blk_row(const u64 s[WIDTH], const u64 x[GOLDI_BLK], const u64 (&k)[2]) {
    static_assert(GOLDI_BLK_F[M - 1][I][M - 1] == GOLDI_MDS[I][0], "newest S-box term is c0");
    u64 a_lo = mad_small_sacc<GOLDI_MDS[I][0]>(lo32(x[M - 1]), k[0]);
    u64 a_hi = mad_small_sacc<GOLDI_MDS[I][0]>(hi32(x[M - 1]), k[1]);
    blk_sterms<M, I, M - 2>(x, a_lo, a_hi);
    blk_words<M, I>(s, a_lo, a_hi);
    return reduce_split(a_lo, a_hi);
}

// S-box outputs of rounds 1 .. GOLDI_BLK-1 of the block.
template <int M>
__device__ __forceinline__ void blk_chain(const u64 s[WIDTH], u64 x[GOLDI_BLK], const u64 (*kc)[2]) {
    if constexpr (M < GOLDI_BLK) {
        const u64 k[2] = {kc[M - 1][0], kc[M - 1][1]};
        x[M] = sbox(blk_row<M, 0>(s, x, k));
        blk_chain<M + 1>(s, x, kc);
    }
}

template <int I, int I1>
__device__ __forceinline__ void blk_rows_range(const u64 s[WIDTH], const u64 x[GOLDI_BLK], u64 out[WIDTH],
                                               const u64 (&k)[WIDTH][2]) {
    out[I] = blk_row<GOLDI_BLK, I>(s, x, k[I]);
    if constexpr (I + 1 < I1) blk_rows_range<I + 1, I1>(s, x, out, k);
}

// Rows I0 .. 11 of the state after the block, a group of rows' constants
// read together.
template <int I0>
__device__ __forceinline__ void blk_rows(const u64 s[WIDTH], const u64 x[GOLDI_BLK], u64 out[WIDTH],
                                         const u64 (*kc)[2]) {
    constexpr int I1 = I0 + GOLDI_RC_GROUP < WIDTH ? I0 + GOLDI_RC_GROUP : WIDTH;
    u64 k[WIDTH][2];
#pragma unroll
    for (int i = I0; i < I1; i++) {
        k[i][0] = kc[i][0];
        k[i][1] = kc[i][1];
    }
    blk_rows_range<I0, I1>(s, x, out, k);
    if constexpr (I1 < WIDTH) blk_rows<I1>(s, x, out, kc);
}

// The first partial round rides on the last opening full round's matrix:
// from that round's S-box outputs y, the partial round's S-box input is
// u = row 0 of M y + C[HALF_FULL][0], and the state after it is
// (M P M) y + c0 S(u) + M P C[HALF_FULL] + C[HALF_FULL + 1].
template <int I, int J = 0>
__device__ __forceinline__ void lead_words(const u64 y[WIDTH], u64 &a_lo, u64 &a_hi) {
    constexpr unsigned C = GOLDI_BLK_LEAD_B[I][J];
    a_lo = mad_coef<C>(lo32(y[J]), a_lo);
    a_hi = mad_coef<C>(hi32(y[J]), a_hi);
    if constexpr (J + 1 < WIDTH) lead_words<I, J + 1>(y, a_lo, a_hi);
}

template <int I, int I1>
__device__ __forceinline__ void lead_rows_range(const u64 y[WIDTH], u64 x, u64 out[WIDTH], const u64 (&k)[WIDTH][2]) {
    u64 a_lo = mad_small_sacc<GOLDI_MDS[I][0]>(lo32(x), k[I][0]);
    u64 a_hi = mad_small_sacc<GOLDI_MDS[I][0]>(hi32(x), k[I][1]);
    lead_words<I>(y, a_lo, a_hi);
    out[I] = reduce_split(a_lo, a_hi);
    if constexpr (I + 1 < I1) lead_rows_range<I + 1, I1>(y, x, out, k);
}

template <int I0>
__device__ __forceinline__ void lead_rows(const u64 y[WIDTH], u64 x, u64 out[WIDTH]) {
    constexpr int I1 = I0 + GOLDI_RC_GROUP < WIDTH ? I0 + GOLDI_RC_GROUP : WIDTH;
    u64 k[WIDTH][2];
#pragma unroll
    for (int i = I0; i < I1; i++) {
        k[i][0] = BLK_LEAD_K[i][0];
        k[i][1] = BLK_LEAD_K[i][1];
    }
    lead_rows_range<I0, I1>(y, x, out, k);
    if constexpr (I1 < WIDTH) lead_rows<I1>(y, x, out);
}

__device__ __forceinline__ void lead_matrix(const u64 y[WIDTH], u64 out[WIDTH]) {
    u64 u[WIDTH];
    mds_rows<0, 1>(y, u, RC_SPLIT[HALF_FULL]);
    lead_rows<0>(y, sbox(u[0]), out);
}

// Block b from state s into out (every row reads all of s, so the two
// cannot share registers).
__device__ __forceinline__ void partial_block_to(const u64 s[WIDTH], u64 out[WIDTH], int b) {
    const u64 (*kc)[2] = BLK_K[b];
    u64 x[GOLDI_BLK];
    x[0] = sbox(s[0]);
    blk_chain<1>(s, x, kc);
    blk_rows<0>(s, x, out, kc + GOLDI_BLK - 1);
}

// All blocks, in place.  Two blocks per loop step, the second writing back
// into s, so the state is not copied between blocks: with one block per
// step, the loop-carried outputs cannot take the inputs' registers and each
// step ends with a 12-word copy (measured: -1% on the 2^22 x 8 tree).
__device__ __forceinline__ void partial_blocks(u64 s[WIDTH]) {
    u64 t[WIDTH];
#pragma nounroll
    for (int b = 0; b + 1 < GOLDI_BLK_N; b += 2) {
        partial_block_to(s, t, b);
        partial_block_to(t, s, b + 1);
    }
    if constexpr (GOLDI_BLK_N % 2 == 1) {
        partial_block_to(s, t, GOLDI_BLK_N - 1);
#pragma unroll
        for (int i = 0; i < WIDTH; i++) s[i] = t[i];
    }
}
#endif

__device__ __forceinline__ void partial_round(u64 s[WIDTH], int r) {
    s[0] = sbox(s[0]);
    mds_add_rc(s, r + 1);
}

// In place; input words must be < 2^64 (any word), output words are weak.
// cap0: the caller guarantees words 8..11 are zero (they are not read);
// digest_only: only words 0..3 of the output are used (4..11 are left stale).
// Both are wave-uniform; call sites with constant flags compile to one path.
__device__ __forceinline__ void permute(u64 s[WIDTH], bool cap0 = false, bool digest_only = false) {
    const int n_in = cap0 ? 2 * DIGEST : WIDTH;
#pragma unroll
    for (int i = 0; i < WIDTH; i++)
        if (i < n_in) s[i] = add_weak(s[i], mk64(lo32(RC_SPLIT[0][i][0]), lo32(RC_SPLIT[0][i][1])));
#ifndef GOLDI_PARTIAL_UNROLL
#define GOLDI_PARTIAL_UNROLL 2
#endif
    // Opening full rounds.  Round 0 of a zero-capacity state: S-boxes of
    // words 0..7 only, and the matrix over those words with CAP0_RC1.
#pragma nounroll
    for (int r = 0; r < HALF_FULL; r++) {
        const bool short0 = cap0 && r == 0;
#pragma unroll
        for (int i = 0; i < WIDTH; i++)
            if (i < 2 * DIGEST || !short0) s[i] = sbox(s[i]);
        u64 out[WIDTH];
        if (short0)
            mds_row_group<0, 2 * DIGEST>(s, out, CAP0_RC1);
#if GOLDI_USE_SPARSE
        else if (r + 1 == HALF_FULL)
            pre_matrix(s, out);
#elif GOLDI_USE_BLOCKS
        else if (r + 1 == HALF_FULL)
            lead_matrix(s, out);
#endif
        else
            mds_row_group<0>(s, out, RC_SPLIT[r + 1]);
#pragma unroll
        for (int i = 0; i < WIDTH; i++) s[i] = out[i];
    }
#if GOLDI_USE_BLOCKS
    partial_blocks(s);
#pragma unroll
    for (int r = GOLDI_BLK_FIRST_TAIL; r < HALF_FULL + PARTIAL; r++) partial_round(s, r);
#elif GOLDI_USE_SPARSE
    // Pairs: larger groups measured slower (their constants no longer fit the
    // scalar registers of one group).
#pragma nounroll
    for (int j = 0; j < PARTIAL; j += 2) sparse_group<2>(s, j);
#pragma unroll
    for (int i = 1; i < WIDTH; i++) s[i] = add_weak(s[i], mk64(SP_CEND[i - 1][0], SP_CEND[i - 1][1]));
#else
#pragma unroll GOLDI_PARTIAL_UNROLL
    for (int r = HALF_FULL; r < HALF_FULL + PARTIAL; r++) partial_round(s, r);
#endif
    // Closing full rounds; with digest_only the last matrix computes rows
    // 0..3 only.
#pragma nounroll
    for (int r = HALF_FULL + PARTIAL; r < ROUNDS; r++) {
#pragma unroll
        for (int i = 0; i < WIDTH; i++) s[i] = sbox(s[i]);
        u64 out[WIDTH];
        if (digest_only && r + 1 == ROUNDS) {
            mds_rows<0, DIGEST>(s, out, RC_SPLIT[ROUNDS]);
#pragma unroll
            for (int i = 0; i < DIGEST; i++) s[i] = out[i];
        } else {
            mds_row_group<0>(s, out, RC_SPLIT[r + 1]);
#pragma unroll
            for (int i = 0; i < WIDTH; i++) s[i] = out[i];
        }
    }
}

}  // namespace goldi
