"""Device-side twin of ``synth.inputs.goldilocks_words`` (``fill.hip``)."""

from __future__ import annotations

import ctypes
import os
import subprocess

from .inputs import stream_key

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fill.hip")
LIB = os.path.join(HERE, "libsynthfill.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

_lib = None


def build() -> str:
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call([HIPCC, "-O3", "--offload-arch=gfx950", "-fPIC", "-shared",
                           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", tmp])
    os.replace(tmp, LIB)
    return LIB


def lib():
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (bind to torch's HIP runtime, see paper_2506_09505_amd.lib)
        if not os.path.exists(LIB):
            raise RuntimeError("%s missing: run __graft_entry__.build()" % LIB)
        L = ctypes.CDLL(LIB)
        L.synth_fill_goldilocks.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint64,
                                            ctypes.c_uint64, ctypes.c_void_p]
        L.synth_fill_goldilocks.restype = ctypes.c_int
        _lib = L
    return _lib


def fill_words(t, seed: int, stream: int = 0, start: int = 0, torch_stream=None):
    """Fill the uint64 device tensor ``t`` with words start.. of (seed, stream)."""
    import torch
    s = torch_stream if torch_stream is not None else torch.cuda.current_stream()
    key = int(stream_key(seed, stream))
    rc = lib().synth_fill_goldilocks(t.data_ptr(), t.numel(), key, start, ctypes.c_void_p(s.cuda_stream))
    if rc != 0:
        raise RuntimeError("synth_fill_goldilocks failed (%d)" % rc)
    return t


def leaves_colmajor_dev(n_rows: int, n_cols: int, seed: int, stream: int = 0, device="cuda:0"):
    """Same words as ``synth.inputs.leaves_colmajor``, generated on the device."""
    import torch
    t = torch.empty(n_rows * n_cols, dtype=torch.uint64, device=device)
    return fill_words(t, seed, stream)
