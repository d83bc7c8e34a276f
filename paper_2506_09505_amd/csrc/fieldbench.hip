// The basic functions of the paper's Table 1, as gfx950 device functions on
// 32-bit limbs, exposed for two purposes:
//   * goldi_fb_eval: element-wise evaluation on device arrays, so every field
//     operation of the HIP path can be compared with the CPU oracle;
//   * goldi_fb_throughput: each lane runs a dependent chain of one function,
//     for the per-function rate on MI355X (the paper's Figs. 6-7 questions,
//     asked of gfx950).
// Outputs of goldi_fb_eval are canonical.  Functions (Table 1 name -> here):
//   add            0  canonical add (Alg. 4, with >=)
//   sub            1  canonical sub (Alg. 6)
//   reduce_128_64  2  out = (a 2^64 + b) mod p (Alg. 2 / Eq. 3)
//   square_128     3  a^2 mod p
//   mult_128       4  a b mod p
//   mult_72        5  a (b mod 256) mod p (one factor of at most 8 bits)
//   S-box          6  a^7 mod p (Sec. 2.4)
//   mmult_4x12_8   7  12x12 product with the instance's small matrix, on
//                     12-word states (a: [n][12]); the 8-bit-entry mat-vec
//   mmult_4x12     8  12x12 product with full 64-bit entries (the instance's
//                     round constants C[0..11] used as matrix rows), [n][12]
#include <hip/hip_runtime.h>

#include "goldi_fieldbench.h"
#include "poseidon.hpp"

using namespace goldi;

namespace {

// Canonical add of canonical inputs (Alg. 4): c = a + b; if b >= p - a, c -= p.
__device__ __forceinline__ u64 add_canon(u64 a, u64 b) {
    const u64 d = P - a;
    const u64 c = a + b;
    return b >= d ? c - P : c;
}

// Canonical sub of canonical inputs (Alg. 6): c = a - b; if a < b, c += p.
__device__ __forceinline__ u64 sub_canon(u64 a, u64 b) {
    const u64 c = a - b;
    return a < b ? c + P : c;
}

// a * b8 with a one-byte factor (mult_72): two multiply-adds and the split
// reduction used by the matrix layer.
__device__ __forceinline__ u64 mul_small(u64 a, u32 b8) {
    return reduce_split(mad32(lo32(a), b8, 0), mad32(hi32(a), b8, 0));
}

// Dense 12x12 with full 64-bit entries, row i = C[0][(i + j) mod 12]
// (a stand-in full-width matrix); lazy per-row: 12 products, reduced each.
__device__ __forceinline__ void mmult_full(u64 s[WIDTH]) {
    u64 out[WIDTH];
#pragma unroll
    for (int i = 0; i < WIDTH; i++) {
        u64 acc = 0;
#pragma unroll
        for (int j = 0; j < WIDTH; j++) {
            const u64 c = mk64(lo32(RC_SPLIT[0][(i + j) % WIDTH][0]), lo32(RC_SPLIT[0][(i + j) % WIDTH][1]));
            acc = add_weak(mul(c, s[j]), canon(acc));
        }
        out[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < WIDTH; i++) s[i] = out[i];
}

__device__ __forceinline__ void mmult_small(u64 s[WIDTH]) { mds_add_rc(s, ROUNDS); }

__global__ void k_fb_eval(int op, const u64 *a, const u64 *b, u64 *out, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (op == GOLDI_FB_MMULT_SMALL || op == GOLDI_FB_MMULT_FULL) {
        u64 s[WIDTH];
#pragma unroll
        for (int k = 0; k < WIDTH; k++) s[k] = a[i * WIDTH + k];
        if (op == GOLDI_FB_MMULT_SMALL) mmult_small(s); else mmult_full(s);
#pragma unroll
        for (int k = 0; k < WIDTH; k++) out[i * WIDTH + k] = canon(s[k]);
        return;
    }
    const u64 x = a[i], y = b[i];
    u64 r = 0;
    switch (op) {
        case GOLDI_FB_ADD: r = add_canon(x, y); break;
        case GOLDI_FB_SUB: r = sub_canon(x, y); break;
        case GOLDI_FB_REDUCE: r = canon(reduce128(y, x)); break;
        case GOLDI_FB_SQUARE: r = canon(sqr(x)); break;
        case GOLDI_FB_MULT: r = canon(mul(x, y)); break;
        case GOLDI_FB_MULT_SMALL: r = canon(mul_small(x, (u32)(y & 0xFF))); break;
        case GOLDI_FB_SBOX: r = canon(sbox(x)); break;
        default: r = 0;
    }
    out[i] = r;
}

// Dependent chains: x <- f(x, y) `iters` times per lane; the result is stored
// so nothing is dead.  Chains of the 1-word functions are 8 wide per lane
// (independent accumulators), so the rate is the issue rate, not the latency.
template <int OP>
__global__ void __launch_bounds__(256) k_fb_chain(const u64 *seed, u64 *out, int iters) {
    const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if constexpr (OP == GOLDI_FB_MMULT_SMALL || OP == GOLDI_FB_MMULT_FULL) {
        u64 s[WIDTH];
#pragma unroll
        for (int k = 0; k < WIDTH; k++) s[k] = seed[k] + t;
        for (int it = 0; it < iters; it++) {
            if constexpr (OP == GOLDI_FB_MMULT_SMALL) mmult_small(s); else mmult_full(s);
        }
        u64 acc = 0;
#pragma unroll
        for (int k = 0; k < WIDTH; k++) acc ^= s[k];
        out[t] = acc;
    } else {
        u64 x[8];
        const u64 y = seed[1] + t;
#pragma unroll
        for (int k = 0; k < 8; k++) x[k] = (seed[0] + t * 8 + k) % P;
        for (int it = 0; it < iters; it++) {
#pragma unroll
            for (int k = 0; k < 8; k++) {
                if constexpr (OP == GOLDI_FB_ADD) x[k] = add_canon(x[k], y % P);
                else if constexpr (OP == GOLDI_FB_SUB) x[k] = sub_canon(x[k], y % P);
                else if constexpr (OP == GOLDI_FB_REDUCE) x[k] = reduce128(y, x[k]);
                else if constexpr (OP == GOLDI_FB_SQUARE) x[k] = sqr(x[k]);
                else if constexpr (OP == GOLDI_FB_MULT) x[k] = mul(x[k], y);
                else if constexpr (OP == GOLDI_FB_MULT_SMALL) x[k] = mul_small(x[k], 45u);
                else if constexpr (OP == GOLDI_FB_SBOX) x[k] = sbox(x[k]);
            }
        }
        u64 acc = 0;
#pragma unroll
        for (int k = 0; k < 8; k++) acc ^= x[k];
        out[t] = acc;
    }
}

template <int OP>
hipError_t launch_chain(const u64 *seed, u64 *out, size_t threads, int iters, hipStream_t st) {
    hipLaunchKernelGGL(k_fb_chain<OP>, dim3((unsigned)(threads / 256)), dim3(256), 0, st, seed, out, iters);
    return hipGetLastError();
}

}  // namespace

extern "C" {

int goldi_fb_eval(int op, const uint64_t *a, const uint64_t *b, uint64_t *out, size_t n) {
    if (op < 0 || op >= GOLDI_FB_COUNT || a == nullptr || out == nullptr || n == 0) return -1;
    const bool state_op = op == GOLDI_FB_MMULT_SMALL || op == GOLDI_FB_MMULT_FULL;
    if (!state_op && b == nullptr) return -1;
    hipLaunchKernelGGL(k_fb_eval, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, 0, op, a, b, out, n);
    if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) return -3;
    return 0;
}

int goldi_fb_throughput(int op, const uint64_t *seed, uint64_t *out, size_t threads, int iters, float *ms) {
    if (op < 0 || op >= GOLDI_FB_COUNT || seed == nullptr || out == nullptr || ms == nullptr || threads == 0 ||
        threads % 256 != 0 || iters <= 0)
        return -1;
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return -3;
    hipError_t e = hipSuccess;
    for (int rep = 0; rep < 2 && e == hipSuccess; rep++) {  // rep 0 warms up
        if (rep == 1) (void)hipEventRecord(e0, 0);
        switch (op) {
            case GOLDI_FB_ADD: e = launch_chain<GOLDI_FB_ADD>(seed, out, threads, iters, 0); break;
            case GOLDI_FB_SUB: e = launch_chain<GOLDI_FB_SUB>(seed, out, threads, iters, 0); break;
            case GOLDI_FB_REDUCE: e = launch_chain<GOLDI_FB_REDUCE>(seed, out, threads, iters, 0); break;
            case GOLDI_FB_SQUARE: e = launch_chain<GOLDI_FB_SQUARE>(seed, out, threads, iters, 0); break;
            case GOLDI_FB_MULT: e = launch_chain<GOLDI_FB_MULT>(seed, out, threads, iters, 0); break;
            case GOLDI_FB_MULT_SMALL: e = launch_chain<GOLDI_FB_MULT_SMALL>(seed, out, threads, iters, 0); break;
            case GOLDI_FB_SBOX: e = launch_chain<GOLDI_FB_SBOX>(seed, out, threads, iters, 0); break;
            case GOLDI_FB_MMULT_SMALL: e = launch_chain<GOLDI_FB_MMULT_SMALL>(seed, out, threads, iters, 0); break;
            case GOLDI_FB_MMULT_FULL: e = launch_chain<GOLDI_FB_MMULT_FULL>(seed, out, threads, iters, 0); break;
        }
    }
    if (e == hipSuccess) e = hipEventRecord(e1, 0);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e == hipSuccess ? 0 : -3;
}

}  // extern "C"
