// Goldilocks field arithmetic on gfx950, on 32-bit limbs.
//
// p = 2^64 - 2^32 + 1 (Sec. 2.4, Eq. 1).  An element travels as a uint64_t,
// i.e. a pair of 32-bit VGPRs (lo, hi).  Inside the permutation values are
// kept *weakly reduced*: any 64-bit word w stands for w mod p (a word is
// either x or x + p, because p > 2^63).  Only values leaving the kernel are
// made canonical (0 <= x < p), which is what the paper requires of its
// outputs (Sec. 3.2).
//
// Products use four 32x32->64 multiply-adds (v_mad_u64_u32), the limb split
// of the paper's 32-bit-half multiplication (Sec. 3.2, the SVE branch of the
// mul_128 listing); gfx950 issues them at the full VALU rate, so there is no
// reason to avoid them.  Reduction of a 128-bit value r = r_hh 2^96 +
// r_hl 2^64 + r_l uses 2^64 = 2^32 - 1 (mod p) (Sec. 3.1, Eqs. 2-3):
//     r = r_l + r_hl (2^32 - 1) - r_hh   (mod p),
// which is the paper's Reduce128 (Alg. 2, with the masks read as the equations
// state them: r_l = low 64 bits, r_hl = bits 64..95, r_hh = bits 96..127).
// The multiplication by 2^32 - 1 is one multiply-add with the inline constant
// -1 instead of a shift and a subtract.
#pragma once
#include <stdint.h>

namespace goldi {

typedef uint64_t u64;
typedef uint32_t u32;

static constexpr u64 P = 0xFFFFFFFF00000001ull;
static constexpr u64 EPS = 0xFFFFFFFFull;  // 2^64 mod p = 2^32 - 1

__device__ __forceinline__ u32 lo32(u64 x) { return (u32)x; }
__device__ __forceinline__ u32 hi32(u64 x) { return (u32)(x >> 32); }
__device__ __forceinline__ u64 mk64(u32 lo, u32 hi) { return ((u64)hi << 32) | lo; }

// a * b + c with 32-bit a, b and 64-bit c: one v_mad_u64_u32.  Never overflows
// when c < 2^64 - (2^32-1)^2, in particular when c < 2^33.
__device__ __forceinline__ u64 mad32(u32 a, u32 b, u64 c) { return (u64)a * b + c; }

// Full 128-bit product of two 64-bit words.
#ifndef GOLDI_MUL_ASM
#define GOLDI_MUL_ASM 1
#endif
__device__ __forceinline__ void mul_wide(u64 a, u64 b, u64 &lo, u64 &hi) {
    const u32 a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
#if GOLDI_MUL_ASM
    // p00 = a0 b0; t = a1 b0 + hi(p00) (no overflow); u = a0 b1 + t with
    // carry c (u + c 2^64 = the middle sum); hi = a1 b1 + (hi(u) + c 2^32).
    const u64 p00 = mad32(a0, b0, 0);
    const u64 t = mad32(a1, b0, hi32(p00));
    u64 u, c;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(u), "=s"(c) : "v"(a0), "v"(b1), "v"(t));
    u32 cw;
    asm("s_nop 1\n\tv_addc_co_u32 %0, vcc, 0, 0, %1" : "=v"(cw) : "s"(c) : "vcc");
    lo = mk64(lo32(p00), lo32(u));
    hi = mad32(a1, b1, mk64(hi32(u), cw));
#else
    const u64 p00 = mad32(a0, b0, 0);
    const u64 t = mad32(a0, b1, hi32(p00));   // <= (2^32-1)^2 + 2^32 - 1
    const u64 u = mad32(a1, b0, lo32(t));     // same bound
    const u64 v = mad32(a1, b1, hi32(t));     // same bound
    lo = mk64(lo32(p00), lo32(u));
    hi = v + hi32(u);                          // the true high word: no overflow
#endif
}

// x + y mod p, weak result, valid when at least one operand is < p
// (then a wrapped sum is < p and adding 2^32 - 1 cannot wrap again).
__device__ __forceinline__ u64 add_weak(u64 x, u64 y) {
    u64 s;
    const bool c = __builtin_add_overflow(x, y, &s);
    return s + (c ? EPS : 0);
}

// Inline assembly below: gfx950 needs two wait states between a VALU
// instruction that writes a carry into an SGPR pair and a VALU instruction
// that reads it; the compiler inserts them for its own code but not inside
// inline assembly, hence the explicit "s_nop 1".  VCC is used as a scratch
// carry destination and declared clobbered.

// x + h (2^32 - 1)  (mod p) for any 64-bit x and 32-bit h, as a weak word.
// One multiply-add with carry-out; a carry stands for 2^64 = 2^32 - 1, added
// back with a second multiply-add that cannot overflow (the wrapped sum is
// below h (2^32 - 1) <= 2^64 - 2^33 + 1).
__device__ __forceinline__ u64 mad_eps_fold(u32 h, u64 x) {
    u64 r, c;
    u32 t;
    asm("v_mad_u64_u32 %0, %1, %3, -1, %4\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32 %2, vcc, 0, 0, %1\n\t"
        "v_mad_u64_u32 %0, vcc, %2, -1, %0"
        : "=&v"(r), "=&s"(c), "=&v"(t)
        : "v"(h), "v"(x)
        : "vcc");
    return r;
}

// (x1 2^32 + x0) - h  (mod p) as a weak word.  On a borrow the wrapped word
// exceeds the true difference by 2^64, so p is added back (mod 2^64), which
// cannot borrow again (the wrapped word is >= 2^64 - 2^32 + 1).
__device__ __forceinline__ u64 sub_fold(u32 x0, u32 x1, u32 h) {
    u32 y0, y1, m;
    u64 b;
    asm("v_sub_co_u32 %0, %2, %4, %6\n\t"
        "s_nop 1\n\t"
        "v_subb_co_u32 %1, %2, %5, 0, %2\n\t"
        "s_nop 1\n\t"
        "v_subb_co_u32 %3, vcc, 0, 0, %2\n\t"
        "v_addc_co_u32 %0, %2, %0, 0, %2\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32 %1, vcc, %1, %3, %2"
        : "=&v"(y0), "=&v"(y1), "=&s"(b), "=&v"(m)
        : "v"(x0), "v"(x1), "v"(h)
        : "vcc");
    return mk64(y0, y1);
}

// 128-bit r = hh 2^96 + hl 2^64 + (l1 2^32 + l0) -> weak word congruent to
// r_l - r_hh + r_hl (2^32 - 1), Alg. 2 / Eq. 3.
__device__ __forceinline__ u64 reduce128_parts(u32 l0, u32 l1, u32 hl, u32 hh) {
    return mad_eps_fold(hl, sub_fold(l0, l1, hh));
}

__device__ __forceinline__ u64 reduce128(u64 lo, u64 hi) {
    return reduce128_parts(lo32(lo), hi32(lo), lo32(hi), hi32(hi));
}

#ifndef GOLDI_MUL_FOLD
#define GOLDI_MUL_FOLD 1
#endif
// Products are also available as whole inline-assembly blocks of one, two or
// three independent products (field_asm.inc, generated from the sequence
// below, with exactly the wait states each carry read needs: none for
// three).  The layout with three words per lane uses the three-product
// blocks for its full rounds, the one-word-per-lane layout the one- and
// two-product blocks for its S-boxes.
}  // namespace goldi
#include "field_asm.inc"
namespace goldi {

#if GOLDI_MUL_FOLD && GOLDI_MUL_ASM
// a b mod p as a weak word.  With p00 = a0 b0, t = a1 b0 + hi(p00),
// u + c 2^64 = a0 b1 + t and h = a1 b1 + hi(u), the 128-bit product is
//     r_l + 2^64 (h + c 2^32),   r_l = lo(p00) + lo(u) 2^32,
// and h + c 2^32 < 2^64 (the product is below 2^128), so Eq. 3 gives
//     a b = r_l - hi(h) - c + lo(h) (2^32 - 1)   (mod p).
// * The middle carry c enters the subtraction as its borrow-in.  The
//   subtraction y = r_l - hi(h) - c may borrow (b = 1): the wrapped word is
//   then 2^64 too large, and y >= 2^64 - 2^32 + 1.
// * r1 + k 2^64 = lo(h) (2^32 - 1) + y is one multiply-add with carry-out,
//   and 2^64 = 2^32 - 1 gives  a b = r1 + (k - b)(2^32 - 1)  (mod p).
// * When b = 1, y + lo(h)(2^32 - 1) reaches 2^64 unless lo(h) = 0, so the
//   correction d = k - b is 0 or 1, or -1 only when lo(h) = 0; in every case
//   r1 + d (2^32 - 1) = r1 - d + d 2^32 lies inside 64 bits.  One signed
//   multiply-add (d times -1, plus r1) and one 32-bit add into the high word
//   apply it.  (Measured against fixing the borrow first with three carry
//   instructions: -5% on the 2^22 tree, -8% on small trees.)
__device__ __forceinline__ u64 mul(u64 a, u64 b) {
    const u32 a0 = lo32(a), a1 = hi32(a), b0 = lo32(b), b1 = hi32(b);
    const u64 p00 = mad32(a0, b0, 0);
    const u64 t = mad32(a1, b0, hi32(p00));
    u64 u, c;
    asm("v_mad_u64_u32 %0, %1, %2, %3, %4" : "=v"(u), "=s"(c) : "v"(a0), "v"(b1), "v"(t));
    const u64 h = mad32(a1, b1, hi32(u));
    u32 y0, y1;
    u64 brw;
    asm("s_nop 1\n\t"
        "v_subb_co_u32 %0, %2, %3, %4, %5\n\t"
        "s_nop 1\n\t"
        "v_subb_co_u32 %1, %2, %6, 0, %2"
        : "=&v"(y0), "=&v"(y1), "=&s"(brw)
        : "v"(lo32(p00)), "v"(hi32(h)), "s"(c), "v"(lo32(u)));
    u64 r1, k;
    u32 kv, d;
    asm("v_mad_u64_u32 %0, %1, %4, -1, %5\n\t"
        "s_nop 1\n\t"
        "v_addc_co_u32 %2, vcc, 0, 0, %1\n\t"
        "v_subb_co_u32 %3, vcc, %2, 0, %6"
        : "=&v"(r1), "=&s"(k), "=&v"(kv), "=&v"(d)
        : "v"(lo32(h)), "v"(mk64(y0, y1)), "s"(brw)
        : "vcc");
    u64 r2;
    asm("v_mad_i64_i32 %0, vcc, %1, -1, %2" : "=v"(r2) : "v"(d), "v"(r1) : "vcc");
    return mk64(lo32(r2), hi32(r2) + d);
}
#else
__device__ __forceinline__ u64 mul(u64 a, u64 b) {
    u64 lo, hi;
    mul_wide(a, b, lo, hi);
    return reduce128(lo, hi);
}
#endif

__device__ __forceinline__ u64 sqr(u64 a) { return mul(a, a); }

// Weak word -> canonical representative in [0, p): subtract p when x >= p,
// i.e. when x + (2^32 - 1) carries out of 64 bits.
__device__ __forceinline__ u64 canon(u64 x) {
    u64 y;
    const bool ge = __builtin_add_overflow(x, EPS, &y);
    return ge ? y : x;
}

}  // namespace goldi
