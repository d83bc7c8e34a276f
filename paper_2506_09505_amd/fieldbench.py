"""Binding of libgoldi_fieldbench.so (include/goldi_fieldbench.h): the
paper's Table-1 functions as gfx950 device functions -- element-wise
evaluation and per-function throughput."""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgoldi_fieldbench.so")

OPS = {"add": 0, "sub": 1, "reduce_128_64": 2, "square_128": 3, "mult_128": 4, "mult_72": 5, "sbox": 6,
       "mmult_12x12_small": 7, "mmult_12x12_full": 8}
STATE_OPS = ("mmult_12x12_small", "mmult_12x12_full")

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
