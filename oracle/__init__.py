"""CPU oracle for Poseidon-12 Merkle building over Goldilocks.

TEST INFRASTRUCTURE ONLY: only the tests, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP path (``paper_2506_09505_amd``) and the product never calls it.

* ``oracle.c`` (compiled with gcc to ``liboracle.so``) is the plain textbook
  definition: dense matrix in every round, exact 128-bit products reduced with
  ``%``; POSIX threads only across independent hashes.
* ``oracle.mini`` is a second, pure-Python big-integer implementation used on
  tiny inputs.

Parity unpinned: the permutation's values against the paper (it prints no
constants and no test vectors).  The field, round structure, constant
placement, matrix orientation, sponge and tree are pinned in the CPU tests.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

P = 0xFFFFFFFF00000001
WIDTH, ROUNDS, DIGEST = 12, 30, 4


def build(force: bool = False) -> str:
    """Compile oracle.c with gcc into liboracle.so (host code only)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
                               "-pthread", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("rc", (ctypes.c_uint64 * WIDTH) * ROUNDS),
                ("mds", (ctypes.c_uint64 * WIDTH) * WIDTH)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        u64, sz, ptr, i32 = ctypes.c_uint64, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_int
        for name in ("oracle_fadd", "oracle_fsub", "oracle_fmul", "oracle_fpow"):
            getattr(L, name).restype = u64
            getattr(L, name).argtypes = [u64, u64]
        L.oracle_reduce128.restype = u64
        L.oracle_reduce128.argtypes = [u64, u64]
        L.oracle_permute.argtypes = [ptr, ptr, sz, i32]
        L.oracle_field_array.argtypes = [i32, ptr, ptr, ptr, sz]
        L.oracle_leaf_hash.argtypes = [ptr, ptr, sz, sz, ptr, i32]
        L.oracle_merkle_level.argtypes = [ptr, ptr, sz, ptr, i32]
        L.oracle_merkle_build.argtypes = [ptr, ptr, sz, sz, ptr, i32]
        L.oracle_merkle_num_nodes.restype = sz
        L.oracle_merkle_num_nodes.argtypes = [sz]
        _lib = L
    return _lib


def default_threads() -> int:
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


class Params:
    """Round constants rc[30][12] and matrix mds[12][12] (Python ints)."""

    def __init__(self, rc, mds):
        assert len(rc) == ROUNDS and all(len(r) == WIDTH for r in rc)
        assert len(mds) == WIDTH and all(len(r) == WIDTH for r in mds)
        self.rc = [[int(v) for v in r] for r in rc]
        self.mds = [[int(v) for v in r] for r in mds]
        self._c = _Params()
        for r in range(ROUNDS):
            for i in range(WIDTH):
                self._c.rc[r][i] = self.rc[r][i]
        for i in range(WIDTH):
            for j in range(WIDTH):
                self._c.mds[i][j] = self.mds[i][j]

    @property
    def ptr(self):
        return ctypes.addressof(self._c)


def spec_params() -> Params:
    """The seeded instance from synth/poseidon12.json."""
    from synth.constants import load_constants
    rc, mds = load_constants()
    return Params(rc, mds)


def _u64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.uint64))


def fadd(a, b): return lib().oracle_fadd(a, b)
def fsub(a, b): return lib().oracle_fsub(a, b)
def fmul(a, b): return lib().oracle_fmul(a, b)
def fpow(a, e): return lib().oracle_fpow(a, e)
def reduce128(hi, lo): return lib().oracle_reduce128(hi, lo)


FIELD_OPS = {"add": 0, "sub": 1, "reduce_128_64": 2, "square_128": 3, "mult_128": 4, "mult_72": 5, "sbox": 6}


def field_array(name: str, a, b=None) -> np.ndarray:
    """Element-wise field operation (plain definitions), see oracle_field_array."""
    a = _u64(a).reshape(-1)
    b = a if b is None else _u64(b).reshape(-1)
    out = np.zeros_like(a)
    lib().oracle_field_array(FIELD_OPS[name], a.ctypes.data, b.ctypes.data, out.ctypes.data, a.size)
    return out


def permute(params: Params, states, threads: int | None = None) -> np.ndarray:
    s = _u64(states).reshape(-1, WIDTH).copy()
    lib().oracle_permute(params.ptr, s.ctypes.data, s.shape[0], threads or default_threads())
    return s


def leaf_hash(params: Params, leaves_colmajor, n_rows: int, n_cols: int,
              threads: int | None = None) -> np.ndarray:
    lv = _u64(leaves_colmajor).reshape(-1)
    assert lv.size == n_rows * n_cols
    out = np.zeros((n_rows, DIGEST), dtype=np.uint64)
    lib().oracle_leaf_hash(params.ptr, lv.ctypes.data, n_rows, n_cols, out.ctypes.data,
                           threads or default_threads())
    return out


def merkle_level(params: Params, children, threads: int | None = None) -> np.ndarray:
    ch = _u64(children).reshape(-1, DIGEST)
    out = np.zeros(((ch.shape[0] + 1) // 2, DIGEST), dtype=np.uint64)
    lib().oracle_merkle_level(params.ptr, ch.ctypes.data, ch.shape[0], out.ctypes.data,
                              threads or default_threads())
    return out


def num_nodes(n_rows: int) -> int:
    return lib().oracle_merkle_num_nodes(n_rows)


def level_sizes(n_rows: int):
    sizes = [n_rows]
    while sizes[-1] > 1:
        sizes.append((sizes[-1] + 1) // 2)
    return sizes


def merkle_build(params: Params, leaves_colmajor, n_rows: int, n_cols: int,
                 threads: int | None = None) -> np.ndarray:
    lv = _u64(leaves_colmajor).reshape(-1)
    assert lv.size == n_rows * n_cols
    out = np.zeros((num_nodes(n_rows), DIGEST), dtype=np.uint64)
    lib().oracle_merkle_build(params.ptr, lv.ctypes.data, n_rows, n_cols, out.ctypes.data,
                              threads or default_threads())
    return out
