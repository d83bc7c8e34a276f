"""Binding of libgoldi_fieldbench.so (include/goldi_fieldbench.h): the
paper's Table-1 functions as gfx950 device functions -- element-wise
evaluation and per-function throughput -- and the per-opcode issue-rate
probe of the vector ALU."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgoldi_fieldbench.so")

OPS = {"add": 0, "sub": 1, "reduce_128_64": 2, "square_128": 3, "mult_128": 4, "mult_72": 5, "sbox": 6,
       "mmult_12x12_small": 7, "mmult_12x12_full": 8}
STATE_OPS = ("mmult_12x12_small", "mmult_12x12_full")

# Opcodes of goldi_rate_probe, in the order of the header's enum.
RATE_OPS = ("v_mad_u64_u32", "v_mul_lo_u32", "v_mul_hi_u32", "v_add_co_u32", "v_addc_co_u32", "v_add_u32",
            "v_sub_u32", "v_xor_b32", "v_mov_b32", "v_lshrrev_b32", "v_lshlrev_b64", "v_lshl_add_u64",
            "v_add3_u32", "v_mad_u32_u24", "v_cndmask_b32 (vcc)", "v_cndmask_b32_e64 (sgpr)", "v_alignbit_b32",
            "v_bfe_u32", "v_dot4_u32_u8", "mix v_mad_u64_u32 + v_add_u32", "mix v_add_co_u32 + v_add_u32",
            "mix v_mad_u64_u32 + v_mov_b32", "v_mad_u64_u32 (compiler)", "v_mad_u64_u32 x8 (one asm)",
            "v_add_co_u32 x8 (one asm)", "v_mad_u64_u32 + s_nop 0 x8 (one asm)")
BLOCK_OPS = RATE_OPS[-3:]
# One wave64 instruction per SIMD every 4 cycles: 256 CUs x 4 SIMDs x 16
# lanes x 2.4 GHz lane-instructions per second.
FULL_RATE_LANE_OPS = 256 * 4 * 16 * 2.4e9

_lib = None


def lib():
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (bind to torch's HIP runtime)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("%s is missing: run python -m paper_2506_09505_amd.build" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, sz = ctypes.c_void_p, ctypes.c_size_t
        L.goldi_fb_eval.argtypes = [ctypes.c_int, vp, vp, vp, sz]
        L.goldi_fb_eval.restype = ctypes.c_int
        L.goldi_fb_throughput.argtypes = [ctypes.c_int, vp, vp, sz, ctypes.c_int, ctypes.POINTER(ctypes.c_float)]
        L.goldi_fb_throughput.restype = ctypes.c_int
        L.goldi_rate_probe.argtypes = [ctypes.c_int, ctypes.c_int, sz, ctypes.c_int, vp,
                                       ctypes.POINTER(ctypes.c_float)]
        L.goldi_rate_probe.restype = ctypes.c_int
        _lib = L
    return _lib


def evaluate(name: str, a, b=None):
    """Element-wise op on uint64 device tensors; returns a new tensor."""
    import torch
    out = torch.empty_like(a)
    n = a.numel() // 12 if name in STATE_OPS else a.numel()
    rc = lib().goldi_fb_eval(OPS[name], a.data_ptr(), b.data_ptr() if b is not None else None, out.data_ptr(), n)
    if rc != 0:
        raise RuntimeError("goldi_fb_eval(%s) failed (%d)" % (name, rc))
    return out


def throughput(name: str, threads: int = 256 * 1024 * 4, iters: int = 64):
    """(operations per second, kernel ms) for one function."""
    import torch
    seed = torch.tensor([0x123456789, 0xABCDEF01234], dtype=torch.int64, device="cuda:0").view(torch.uint64)
    out = torch.empty(threads, dtype=torch.uint64, device="cuda:0")
    ms = ctypes.c_float()
    rc = lib().goldi_fb_throughput(OPS[name], seed.data_ptr(), out.data_ptr(), threads, iters, ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError("goldi_fb_throughput(%s) failed (%d)" % (name, rc))
    ops = threads * iters * (1 if name in STATE_OPS else 8)
    return ops / (ms.value * 1e-3), ms.value


def rate_probe(op: str, chains: int, waves: int, iters: int):
    """Kernel ms of goldi_rate_probe for one opcode (a name of RATE_OPS)."""
    import torch
    out = torch.empty(waves * 64, dtype=torch.int32, device="cuda:0")
    ms = ctypes.c_float()
    rc = lib().goldi_rate_probe(RATE_OPS.index(op), chains, waves, iters, out.data_ptr(), ctypes.byref(ms))
    if rc != 0:
        raise RuntimeError("goldi_rate_probe(%s) failed (%d)" % (op, rc))
    return ms.value


def rates(iters: int = 2048):
    """Per opcode: throughput as a fraction of one wave64 instruction per SIMD
    per 4 cycles at 2.4 GHz (8 waves per SIMD, 8 chains per lane), and the
    cycles (at 2.4 GHz) between instructions of one wave alone on its SIMD,
    for a dependent chain and for 8 independent chains."""
    simds = 256 * 4
    out = {}
    for op in RATE_OPS:
        waves = 8 * simds
        ms = rate_probe(op, 8, waves, iters)
        lane_ops = waves * 64 * iters * 16 * 8
        row = {"throughput_frac_of_full_rate": round(lane_ops / (ms * 1e-3) / FULL_RATE_LANE_OPS, 3)}
        for chains, key in ((1, "cycles_per_instr_one_wave_dependent"), (8, "cycles_per_instr_one_wave_8_chains")):
            if chains == 1 and op in BLOCK_OPS:
                continue
            it = max(1, iters // (4 if chains == 8 else 1))
            ms1 = rate_probe(op, chains, simds, it)
            row[key] = round(ms1 * 1e-3 * 2.4e9 / (it * 16 * chains), 2)
        out[op] = row
    return out
