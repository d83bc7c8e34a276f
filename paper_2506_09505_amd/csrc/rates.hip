// Per-opcode issue rates of gfx950's vector ALU, for the integer instructions
// the field layer is built from (the paper's isolated add/sub/multiply IPC
// measurements, Sec. 4.3, asked of MI355X).
//
// Each lane runs CH chains of one instruction (inline assembly, so the
// instruction is exactly the one named), unrolled 16 times per loop
// iteration.  With CH = 8 and many waves per SIMD the launch measures
// throughput; with CH = 1 and one wave per SIMD it measures the latency of a
// dependent chain; with CH = 8 and one wave per SIMD, how fast a single wave
// can issue independent work.  The values computed are meaningless; they are
// stored so the compiler keeps the work.  Only ALU instructions appear in the
// assembly: no memory access, no branch.
#include <hip/hip_runtime.h>

#include "goldi_fieldbench.h"

namespace {

typedef uint32_t u32;
typedef uint64_t u64;

constexpr int UNROLL = 16;

struct Regs {
    u32 x[8];
    u64 y[8];
};

// One instruction of op OP on chain c.  A carry-out goes to an SGPR pair the
// compiler picks (never read), so independent chains share no register.
template <int OP>
__device__ __forceinline__ void step(Regs &r, int c, u32 a, u32 b, u64 m) {
    if constexpr (OP == GOLDI_RATE_MAD_U64_U32) {
        u64 cc;
        asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(r.y[c]), "=s"(cc) : "v"(a), "v"(b));
    } else if constexpr (OP == GOLDI_RATE_MUL_LO_U32) {
        asm volatile("v_mul_lo_u32 %0, %0, %1" : "+v"(r.x[c]) : "v"(a));
    } else if constexpr (OP == GOLDI_RATE_MUL_HI_U32) {
        asm volatile("v_mul_hi_u32 %0, %0, %1" : "+v"(r.x[c]) : "v"(a));
    } else if constexpr (OP == GOLDI_RATE_ADD_CO_U32) {
        u64 cc;
        asm volatile("v_add_co_u32 %0, %1, %0, %2" : "+v"(r.x[c]), "=s"(cc) : "v"(a));
    } else if constexpr (OP == GOLDI_RATE_ADDC_CO_U32) {
        u64 cc;
        asm volatile("v_addc_co_u32 %0, %1, %0, %2, %3" : "+v"(r.x[c]), "=s"(cc) : "v"(a), "s"(m));
    } else if constexpr (OP == GOLDI_RATE_ADD_U32) {
        asm volatile("v_add_u32 %0, %0, %1" : "+v"(r.x[c]) : "v"(a));
    } else if constexpr (OP == GOLDI_RATE_SUB_U32) {
        asm volatile("v_sub_u32 %0, %0, %1" : "+v"(r.x[c]) : "v"(a));
    } else if constexpr (OP == GOLDI_RATE_XOR_B32) {
        asm volatile("v_xor_b32 %0, %0, %1" : "+v"(r.x[c]) : "v"(a));
    } else if constexpr (OP == GOLDI_RATE_MOV_B32) {
        asm volatile("v_mov_b32 %0, %1" : "=v"(r.x[c]) : "v"(r.x[(c + 1) & 7]));
    } else if constexpr (OP == GOLDI_RATE_LSHRREV_B32) {
        asm volatile("v_lshrrev_b32 %0, 1, %0" : "+v"(r.x[c]));
    } else if constexpr (OP == GOLDI_RATE_LSHLREV_B64) {
        asm volatile("v_lshlrev_b64 %0, 1, %0" : "+v"(r.y[c]));
    } else if constexpr (OP == GOLDI_RATE_LSHL_ADD_U64) {
        asm volatile("v_lshl_add_u64 %0, %0, 1, %1" : "+v"(r.y[c]) : "v"(m));
    } else if constexpr (OP == GOLDI_RATE_ADD3_U32) {
        asm volatile("v_add3_u32 %0, %0, %1, %2" : "+v"(r.x[c]) : "v"(a), "v"(b));
    } else if constexpr (OP == GOLDI_RATE_MAD_U32_U24) {
        asm volatile("v_mad_u32_u24 %0, %0, %1, %2" : "+v"(r.x[c]) : "v"(a), "v"(b));
    } else if constexpr (OP == GOLDI_RATE_CNDMASK_VCC) {
        asm volatile("v_cndmask_b32_e32 %0, %0, %1, vcc" : "+v"(r.x[c]) : "v"(a));
    } else if constexpr (OP == GOLDI_RATE_CNDMASK_SGPR) {
        asm volatile("v_cndmask_b32_e64 %0, %0, %1, %2" : "+v"(r.x[c]) : "v"(a), "s"(m));
    } else if constexpr (OP == GOLDI_RATE_ALIGNBIT_B32) {
        asm volatile("v_alignbit_b32 %0, %0, %1, 7" : "+v"(r.x[c]) : "v"(a));
    } else if constexpr (OP == GOLDI_RATE_BFE_U32) {
        asm volatile("v_bfe_u32 %0, %0, 3, 17" : "+v"(r.x[c]));
    } else if constexpr (OP == GOLDI_RATE_DOT4_U32_U8) {
        asm volatile("v_dot4_u32_u8 %0, %1, %2, %0" : "+v"(r.x[c]) : "v"(a), "v"(b));
    } else if constexpr (OP == GOLDI_RATE_MIX_MAD_ADD) {
        // even chains: a multiply-add; odd chains: a plain 32-bit add
        if (c & 1) {
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(r.x[c]) : "v"(a));
        } else {
            u64 cc;
            asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(r.y[c]), "=s"(cc) : "v"(a), "v"(b));
        }
    } else if constexpr (OP == GOLDI_RATE_MIX_ADDCO_ADD) {
        if (c & 1) {
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(r.x[c]) : "v"(a));
        } else {
            u64 cc;
            asm volatile("v_add_co_u32 %0, %1, %0, %2" : "+v"(r.x[c]), "=s"(cc) : "v"(a));
        }
    } else if constexpr (OP == GOLDI_RATE_MAD_C) {
        r.y[c] = (u64)(u32)r.y[c] * b + r.y[c];  // the compiler's own v_mad_u64_u32
    } else if constexpr (OP == GOLDI_RATE_MIX_MAD_MOV) {
        if (c & 1) {
            asm volatile("v_mov_b32 %0, %1" : "=v"(r.x[c]) : "v"(r.x[c ^ 1]));
        } else {
            u64 cc;
            asm volatile("v_mad_u64_u32 %0, %1, %2, %3, %0" : "+v"(r.y[c]), "=s"(cc) : "v"(a), "v"(b));
        }
    }
}

// The block forms: the eight chains' instructions in one asm statement, so
// the compiler inserts no wait states between them (it does after inline
// assembly it cannot see into).
template <int OP>
__device__ __forceinline__ void step_block(Regs &r, u32 a, u32 b) {
    if constexpr (OP == GOLDI_RATE_MAD_BLOCK) {
        asm volatile(
            "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\tv_mad_u64_u32 %1, vcc, %8, %9, %1\n\t"
            "v_mad_u64_u32 %2, vcc, %8, %9, %2\n\tv_mad_u64_u32 %3, vcc, %8, %9, %3\n\t"
            "v_mad_u64_u32 %4, vcc, %8, %9, %4\n\tv_mad_u64_u32 %5, vcc, %8, %9, %5\n\t"
            "v_mad_u64_u32 %6, vcc, %8, %9, %6\n\tv_mad_u64_u32 %7, vcc, %8, %9, %7"
            : "+v"(r.y[0]), "+v"(r.y[1]), "+v"(r.y[2]), "+v"(r.y[3]), "+v"(r.y[4]), "+v"(r.y[5]), "+v"(r.y[6]),
              "+v"(r.y[7])
            : "v"(a), "v"(b)
            : "vcc");
    } else if constexpr (OP == GOLDI_RATE_ADDCO_BLOCK) {
        asm volatile(
            "v_add_co_u32 %0, vcc, %0, %8\n\tv_add_co_u32 %1, vcc, %1, %8\n\t"
            "v_add_co_u32 %2, vcc, %2, %8\n\tv_add_co_u32 %3, vcc, %3, %8\n\t"
            "v_add_co_u32 %4, vcc, %4, %8\n\tv_add_co_u32 %5, vcc, %5, %8\n\t"
            "v_add_co_u32 %6, vcc, %6, %8\n\tv_add_co_u32 %7, vcc, %7, %8"
            : "+v"(r.x[0]), "+v"(r.x[1]), "+v"(r.x[2]), "+v"(r.x[3]), "+v"(r.x[4]), "+v"(r.x[5]), "+v"(r.x[6]),
              "+v"(r.x[7])
            : "v"(a)
            : "vcc");
    } else if constexpr (OP == GOLDI_RATE_MAD_NOP_BLOCK) {
        asm volatile(
            "v_mad_u64_u32 %0, vcc, %8, %9, %0\n\ts_nop 0\n\tv_mad_u64_u32 %1, vcc, %8, %9, %1\n\ts_nop 0\n\t"
            "v_mad_u64_u32 %2, vcc, %8, %9, %2\n\ts_nop 0\n\tv_mad_u64_u32 %3, vcc, %8, %9, %3\n\ts_nop 0\n\t"
            "v_mad_u64_u32 %4, vcc, %8, %9, %4\n\ts_nop 0\n\tv_mad_u64_u32 %5, vcc, %8, %9, %5\n\ts_nop 0\n\t"
            "v_mad_u64_u32 %6, vcc, %8, %9, %6\n\ts_nop 0\n\tv_mad_u64_u32 %7, vcc, %8, %9, %7\n\ts_nop 0"
            : "+v"(r.y[0]), "+v"(r.y[1]), "+v"(r.y[2]), "+v"(r.y[3]), "+v"(r.y[4]), "+v"(r.y[5]), "+v"(r.y[6]),
              "+v"(r.y[7])
            : "v"(a), "v"(b)
            : "vcc");
    }
}

constexpr bool is_block(int op) {
    return op == GOLDI_RATE_MAD_BLOCK || op == GOLDI_RATE_ADDCO_BLOCK || op == GOLDI_RATE_MAD_NOP_BLOCK;
}

template <int OP, int CH>
__global__ void __launch_bounds__(64) k_rate(u32 *out, int iters, u32 a, u32 b) {
    Regs r;
    const u32 t = blockIdx.x * 64u + threadIdx.x;
#pragma unroll
    for (int c = 0; c < 8; c++) {
        r.x[c] = t + 77u * c;
        r.y[c] = ((u64)t << 20) + c;
    }
    const u64 m = 0x5555555555555555ull;
    for (int it = 0; it < iters; it++) {
#pragma unroll
        for (int u = 0; u < UNROLL; u++) {
            if constexpr (is_block(OP)) {
                step_block<OP>(r, a, b);  // always the eight chains
            } else {
#pragma unroll
                for (int c = 0; c < CH; c++) step<OP>(r, c, a, b, m);
            }
        }
    }
    u32 acc = 0;
#pragma unroll
    for (int c = 0; c < 8; c++) acc ^= r.x[c] ^ (u32)r.y[c] ^ (u32)(r.y[c] >> 32);
    out[t] = acc;
}

template <int OP>
hipError_t launch_op(int chains, unsigned waves, int iters, u32 *out) {
    if (chains == 1 && !is_block(OP)) {
        hipLaunchKernelGGL((k_rate<OP, 1>), dim3(waves), dim3(64), 0, 0, out, iters, 3u, 5u);
    } else {
        hipLaunchKernelGGL((k_rate<OP, 8>), dim3(waves), dim3(64), 0, 0, out, iters, 3u, 5u);
    }
    return hipGetLastError();
}

hipError_t launch(int op, int chains, unsigned waves, int iters, u32 *out) {
    switch (op) {
#define GOLDI_RATE_CASE(X) \
    case X: return launch_op<X>(chains, waves, iters, out);
        GOLDI_RATE_CASE(GOLDI_RATE_MAD_U64_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_MUL_LO_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_MUL_HI_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_ADD_CO_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_ADDC_CO_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_ADD_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_SUB_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_XOR_B32)
        GOLDI_RATE_CASE(GOLDI_RATE_MOV_B32)
        GOLDI_RATE_CASE(GOLDI_RATE_LSHRREV_B32)
        GOLDI_RATE_CASE(GOLDI_RATE_LSHLREV_B64)
        GOLDI_RATE_CASE(GOLDI_RATE_LSHL_ADD_U64)
        GOLDI_RATE_CASE(GOLDI_RATE_ADD3_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_MAD_U32_U24)
        GOLDI_RATE_CASE(GOLDI_RATE_CNDMASK_VCC)
        GOLDI_RATE_CASE(GOLDI_RATE_CNDMASK_SGPR)
        GOLDI_RATE_CASE(GOLDI_RATE_ALIGNBIT_B32)
        GOLDI_RATE_CASE(GOLDI_RATE_BFE_U32)
        GOLDI_RATE_CASE(GOLDI_RATE_DOT4_U32_U8)
        GOLDI_RATE_CASE(GOLDI_RATE_MIX_MAD_ADD)
        GOLDI_RATE_CASE(GOLDI_RATE_MIX_ADDCO_ADD)
        GOLDI_RATE_CASE(GOLDI_RATE_MIX_MAD_MOV)
        GOLDI_RATE_CASE(GOLDI_RATE_MAD_C)
        GOLDI_RATE_CASE(GOLDI_RATE_MAD_BLOCK)
        GOLDI_RATE_CASE(GOLDI_RATE_ADDCO_BLOCK)
        GOLDI_RATE_CASE(GOLDI_RATE_MAD_NOP_BLOCK)
#undef GOLDI_RATE_CASE
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

extern "C" int goldi_rate_probe(int op, int chains, size_t waves, int iters, uint32_t *out, float *ms) {
    if (op < 0 || op >= GOLDI_RATE_COUNT || (chains != 1 && chains != 8) || waves == 0 || waves > (1u << 20) ||
        iters <= 0 || out == nullptr || ms == nullptr)
        return -1;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int rc = -3;
    if (hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess &&
        launch(op, chains, (unsigned)waves, 1, out) == hipSuccess &&  // warm-up (code load, clocks)
        hipEventRecord(e0, 0) == hipSuccess && launch(op, chains, (unsigned)waves, iters, out) == hipSuccess &&
        hipEventRecord(e1, 0) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
        hipEventElapsedTime(ms, e0, e1) == hipSuccess)
        rc = 0;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return rc;
}
