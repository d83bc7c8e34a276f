/*
 * goldi_fieldbench.h -- the basic functions of the paper's Table 1 (the
 * Goldilocks field operations and small mat-vecs behind Poseidon, Sec. 3.1-3.2)
 * as gfx950 device functions, in a separate library libgoldi_fieldbench.so.
 * Same device code as the Merkle builder (field.hpp / poseidon.hpp).
 *
 * All pointers are DEVICE memory owned by the caller.  Inputs must be
 * canonical (< p) except the 128-bit reduction, which takes any words.
 */
#ifndef GOLDI_FIELDBENCH_H
#define GOLDI_FIELDBENCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GOLDI_FB_ADD = 0,          /* add (Alg. 4)                                  */
    GOLDI_FB_SUB = 1,          /* sub (Alg. 6)                                  */
    GOLDI_FB_REDUCE = 2,       /* reduce_128_64: (a 2^64 + b) mod p (Alg. 2)    */
    GOLDI_FB_SQUARE = 3,       /* square_128                                     */
    GOLDI_FB_MULT = 4,         /* mult_128                                       */
    GOLDI_FB_MULT_SMALL = 5,   /* mult_72: a * (b mod 256)                       */
    GOLDI_FB_SBOX = 6,         /* x^7 (Sec. 2.4)                                  */
    GOLDI_FB_MMULT_SMALL = 7,  /* 12x12 mat-vec, the instance's small matrix      */
    GOLDI_FB_MMULT_FULL = 8,   /* 12x12 mat-vec, full 64-bit entries              */
    GOLDI_FB_COUNT = 9
};

/* out[i] = op(a[i], b[i]) for i < n (word ops), or out = op(a) on n states of
 * 12 words (the two mat-vecs; b unused).  Outputs canonical.  Synchronous.
 * Returns 0, -1 for bad arguments, -3 for a HIP error. */
int goldi_fb_eval(int op, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t n);

/* Runs `threads` lanes (a multiple of 256), each applying the function `iters`
 * times in dependent chains (8 independent words per lane for word ops, one
 * 12-word state for the mat-vecs), after one warm-up launch; *ms (host) is
 * the kernel time.  seed: 2 device words; out: `threads` device words. */
int goldi_fb_throughput(int op, const uint64_t *seed, uint64_t *out, size_t threads, int iters, float *ms);

/* Per-opcode issue rates of the vector ALU (the isolated add/sub/multiply
 * IPC measurements of Sec. 4.3, asked of gfx950): the integer instructions the
 * field layer is built from, each written as inline assembly so that exactly
 * that instruction runs, three 1:1 mixes, and forms that show what the wait
 * states the compiler inserts after inline assembly cost.  The "block" forms
 * always run 8 chains (chains = 1 is treated as 8 for them). */
enum {
    GOLDI_RATE_MAD_U64_U32 = 0,  /* 32x32 + 64 -> 64, carry-out to SGPRs      */
    GOLDI_RATE_MUL_LO_U32,
    GOLDI_RATE_MUL_HI_U32,
    GOLDI_RATE_ADD_CO_U32,       /* add with carry-out to SGPRs               */
    GOLDI_RATE_ADDC_CO_U32,      /* add with carry-in and carry-out            */
    GOLDI_RATE_ADD_U32,          /* add without carry                          */
    GOLDI_RATE_SUB_U32,
    GOLDI_RATE_XOR_B32,
    GOLDI_RATE_MOV_B32,
    GOLDI_RATE_LSHRREV_B32,
    GOLDI_RATE_LSHLREV_B64,
    GOLDI_RATE_LSHL_ADD_U64,
    GOLDI_RATE_ADD3_U32,
    GOLDI_RATE_MAD_U32_U24,
    GOLDI_RATE_CNDMASK_VCC,      /* v_cndmask_b32, VOP2 form reading VCC       */
    GOLDI_RATE_CNDMASK_SGPR,     /* v_cndmask_b32_e64 with an SGPR-pair mask   */
    GOLDI_RATE_ALIGNBIT_B32,
    GOLDI_RATE_BFE_U32,
    GOLDI_RATE_DOT4_U32_U8,
    GOLDI_RATE_MIX_MAD_ADD,      /* v_mad_u64_u32 and v_add_u32, alternating   */
    GOLDI_RATE_MIX_ADDCO_ADD,    /* v_add_co_u32 and v_add_u32, alternating    */
    GOLDI_RATE_MIX_MAD_MOV,      /* v_mad_u64_u32 and v_mov_b32, alternating   */
    GOLDI_RATE_MAD_C,            /* v_mad_u64_u32 as the compiler emits it     */
    GOLDI_RATE_MAD_BLOCK,        /* 8 v_mad_u64_u32 in one asm statement       */
    GOLDI_RATE_ADDCO_BLOCK,      /* 8 v_add_co_u32 in one asm statement        */
    GOLDI_RATE_MAD_NOP_BLOCK,    /* v_mad_u64_u32 and s_nop 0, alternating,
                                    in one asm statement                       */
    GOLDI_RATE_COUNT
};

/* Runs `waves` single-wave workgroups (64 lanes each); every lane issues
 * iters * 16 * chains instructions of `op` in `chains` (1 or 8) independent
 * dependent chains, after one warm-up launch, on the null stream.  *ms (host)
 * receives the kernel time.  out: device buffer of waves * 64 words (written
 * with meaningless values).  waves in 1..2^20.  Returns 0, -1 for bad
 * arguments, -3 for a HIP error. */
int goldi_rate_probe(int op, int chains, size_t waves, int iters, uint32_t *out, float *ms);

#ifdef __cplusplus
}
#endif

#endif /* GOLDI_FIELDBENCH_H */
