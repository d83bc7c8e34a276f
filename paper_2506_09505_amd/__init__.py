"""MI355X (gfx950) Poseidon-12 / Goldilocks Merkle builder -- Python binding.

A thin ctypes layer over ``libgoldi.so`` (C ABI in ``include/goldi.h``) with
the same function names.  It only marshals arguments: every step of the
permutation, leaf hashing and tree reduction runs in the HIP kernels.
PyTorch supplies device memory and streams; tensors are ``torch.uint64`` on a
ROCm device.  If the library is not built, every call raises -- there is no
CPU fallback.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgoldi.so")

GOLDI_OK, GOLDI_EINVAL, GOLDI_ENONCANON, GOLDI_EDEVICE, GOLDI_ENOMEM = 0, -1, -2, -3, -4
GOLDI_ECANCELED, GOLDI_ETIMEDOUT = -5, -6
P = 0xFFFFFFFF00000001
WIDTH, RATE, DIGEST = 12, 8, 4

# Symbols declared in include/goldi.h.
EXPORTS = ("goldi_poseidon_permute", "goldi_poseidon_permute_async", "goldi_merkle_num_nodes",
           "goldi_leaf_hash", "goldi_leaf_hash_async", "goldi_merkle_build", "goldi_merkle_build_async",
           "goldi_merkle_build_many", "goldi_merkle_build_many_async", "goldi_strerror",
           "goldi_last_error", "goldi_profile_enable", "goldi_profile_read",
           "goldi_tune_set", "goldi_tune_get", "goldi_server_create", "goldi_server_submit",
           "goldi_server_wait", "goldi_server_release", "goldi_server_stats", "goldi_server_destroy",
           "goldi_admission_plan", "goldi_server_read_nodes", "goldi_profile_select",
           "goldi_merkle_build_many_status_async", "goldi_server_set", "goldi_merkle_build_many_noalloc")


class GoldiError(RuntimeError):
    def __init__(self, code: int, where: str, detail: str):
        self.code = code
        super().__init__("%s failed: %s (%d): %s" % (where, _strerror(code), code, detail))


class _ReqInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("n_rows", ctypes.c_size_t), ("n_cols", ctypes.c_size_t),
                ("nodes", ctypes.c_void_p), ("t_submit_ns", ctypes.c_int64), ("t_admit_ns", ctypes.c_int64),
                ("t_done_ns", ctypes.c_int64), ("group_size", ctypes.c_int), ("root", ctypes.c_uint64 * 4)]


class _Tree(ctypes.Structure):
    _fields_ = [("leaves", ctypes.c_void_p), ("n_rows", ctypes.c_size_t),
                ("n_cols", ctypes.c_size_t), ("nodes_out", ctypes.c_void_p)]


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch bundles its own HIP runtime (same soname as the system one).
        # Importing it first makes libgoldi.so bind to that runtime, so both
        # share one device context and torch's pointers are valid here.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("%s is missing: build it with `python -m paper_2506_09505_amd.build` "
                               "(or __graft_entry__.build())" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        vp, sz, ci = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
        L.goldi_poseidon_permute.argtypes = [vp, sz]
        L.goldi_poseidon_permute_async.argtypes = [vp, sz, vp, vp]
        L.goldi_merkle_num_nodes.argtypes = [sz]
        L.goldi_merkle_num_nodes.restype = sz
        L.goldi_leaf_hash.argtypes = [vp, sz, sz, vp]
        L.goldi_leaf_hash_async.argtypes = [vp, sz, sz, vp, vp, vp]
        L.goldi_merkle_build.argtypes = [vp, sz, sz, vp]
        L.goldi_merkle_build_async.argtypes = [vp, sz, sz, vp, vp, vp]
        L.goldi_merkle_build_many.argtypes = [ctypes.POINTER(_Tree), sz]
        L.goldi_merkle_build_many_async.argtypes = [ctypes.POINTER(_Tree), sz, vp, vp]
        L.goldi_merkle_build_many_status_async.argtypes = [ctypes.POINTER(_Tree), sz, vp, vp]
        L.goldi_merkle_build_many_noalloc.argtypes = [ctypes.POINTER(_Tree), sz, ctypes.POINTER(ctypes.c_int), vp]
        L.goldi_strerror.argtypes = [ci]
        L.goldi_strerror.restype = ctypes.c_char_p
        L.goldi_last_error.restype = ctypes.c_char_p
        L.goldi_profile_enable.argtypes = [ci]
        L.goldi_profile_select.argtypes = [ctypes.c_char_p]
        L.goldi_tune_set.argtypes = [ctypes.c_char_p, sz]
        L.goldi_tune_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_size_t)]
        psz = ctypes.POINTER(ctypes.c_size_t)
        L.goldi_server_create.argtypes = [sz, ctypes.c_uint, ctypes.c_uint, ctypes.POINTER(vp)]
        L.goldi_server_submit.argtypes = [vp, vp, vp, sz, sz, ctypes.POINTER(ctypes.c_uint64)]
        L.goldi_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(_ReqInfo)]
        L.goldi_server_release.argtypes = [vp, ctypes.c_uint64]
        L.goldi_server_stats.argtypes = [vp, psz, psz, psz]
        L.goldi_server_destroy.argtypes = [vp]
        L.goldi_server_set.argtypes = [vp, ctypes.c_char_p, ctypes.c_uint64]
        L.goldi_server_read_nodes.argtypes = [vp, ctypes.c_uint64, vp, sz]
        L.goldi_admission_plan.argtypes = [psz, sz, sz, sz, sz, psz]
        L.goldi_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_size_t)]
        for name in EXPORTS:
            if name not in ("goldi_merkle_num_nodes", "goldi_strerror", "goldi_last_error"):
                getattr(L, name).restype = ci
        _lib = L
    return _lib


def _strerror(code: int) -> str:
    try:
        return lib().goldi_strerror(code).decode()
    except Exception:  # pragma: no cover
        return "status"


def _check(code: int, where: str):
    if code != GOLDI_OK:
        raise GoldiError(code, where, lib().goldi_last_error().decode())


def _torch():
    import torch
    return torch


def _dev_u64(t, what: str, min_words: int = 0, device=None):
    """Checks that ``t`` is a contiguous uint64 device tensor holding at least
    ``min_words`` words (on ``device`` if given); the C side can only check the
    allocation a pointer lies in, and torch's caching allocator hands out
    pieces of larger blocks."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint64 or not t.is_cuda:
        raise TypeError("%s must be a torch.uint64 tensor on a ROCm device" % what)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)
    if t.numel() < min_words:
        raise ValueError("%s holds %d words, %d needed" % (what, t.numel(), min_words))
    if device is not None and t.device != device:
        raise ValueError("%s is on %s, expected %s" % (what, t.device, device))
    return t


def _dev_status(t, words: int, device):
    """A contiguous int32/uint32 device tensor of at least ``words`` status words."""
    torch = _torch()
    if not isinstance(t, torch.Tensor) or t.dtype not in (torch.int32, torch.uint32) or not t.is_cuda:
        raise TypeError("dev_status must be an int32 tensor on a ROCm device")
    if not t.is_contiguous() or t.numel() < words:
        raise ValueError("dev_status must be contiguous with at least %d words" % words)
    if t.device != device:
        raise ValueError("dev_status is on %s, expected %s" % (t.device, device))
    return t


def _positive(n: int, what: str) -> int:
    n = int(n)
    if n < 1:
        raise ValueError("%s must be >= 1" % what)
    return n


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def goldi_merkle_num_nodes(n_rows: int) -> int:
    return lib().goldi_merkle_num_nodes(n_rows)


def goldi_poseidon_permute(states):
    """Permutes ``states`` ([n, 12] uint64, on device) in place."""
    _dev_u64(states, "states")
    n = states.numel() // WIDTH
    if states.numel() != n * WIDTH:
        raise ValueError("states must hold a multiple of 12 words")
    with _torch().cuda.device(states.device):
        _check(lib().goldi_poseidon_permute(states.data_ptr(), n), "goldi_poseidon_permute")
    return states


def goldi_poseidon_permute_async(states, dev_status, stream=None):
    _dev_u64(states, "states")
    if states.numel() % WIDTH:
        raise ValueError("states must hold a multiple of 12 words")
    _dev_status(dev_status, 1, states.device)
    with _torch().cuda.device(states.device):
        _check(lib().goldi_poseidon_permute_async(states.data_ptr(), states.numel() // WIDTH,
                                                  dev_status.data_ptr(), _stream_ptr(stream)),
               "goldi_poseidon_permute_async")
    return states


def _alloc(n_words: int, like):
    torch = _torch()
    return torch.empty(n_words, dtype=torch.uint64, device=like.device)


def goldi_leaf_hash(leaves, n_rows: int, n_cols: int, digests=None):
    """Digests ``[n_rows, 4]`` of the rows of the column-major ``leaves``."""
    n_rows, n_cols = _positive(n_rows, "n_rows"), _positive(n_cols, "n_cols")
    _dev_u64(leaves, "leaves", n_rows * n_cols)
    if digests is None:
        digests = _alloc(n_rows * DIGEST, leaves).view(n_rows, DIGEST)
    _dev_u64(digests, "digests", n_rows * DIGEST, leaves.device)
    with _torch().cuda.device(leaves.device):
        _check(lib().goldi_leaf_hash(leaves.data_ptr(), n_rows, n_cols, digests.data_ptr()), "goldi_leaf_hash")
    return digests


def goldi_leaf_hash_async(leaves, n_rows, n_cols, digests, dev_status, stream=None):
    n_rows, n_cols = _positive(n_rows, "n_rows"), _positive(n_cols, "n_cols")
    _dev_u64(leaves, "leaves", n_rows * n_cols)
    _dev_u64(digests, "digests", n_rows * DIGEST, leaves.device)
    _dev_status(dev_status, 1, leaves.device)
    with _torch().cuda.device(leaves.device):
        _check(lib().goldi_leaf_hash_async(leaves.data_ptr(), n_rows, n_cols, digests.data_ptr(),
                                           dev_status.data_ptr(), _stream_ptr(stream)), "goldi_leaf_hash_async")
    return digests


def goldi_merkle_build(leaves, n_rows: int, n_cols: int, nodes_out=None):
    """Every node (level-major, ``[num_nodes, 4]``) of the tree over the rows
    of the column-major ``leaves`` (``leaves[c*n_rows + r]``)."""
    n_rows, n_cols = _positive(n_rows, "n_rows"), _positive(n_cols, "n_cols")
    _dev_u64(leaves, "leaves", n_rows * n_cols)
    if nodes_out is None:
        nodes_out = _alloc(goldi_merkle_num_nodes(n_rows) * DIGEST, leaves).view(-1, DIGEST)
    _dev_u64(nodes_out, "nodes_out", goldi_merkle_num_nodes(n_rows) * DIGEST, leaves.device)
    with _torch().cuda.device(leaves.device):
        _check(lib().goldi_merkle_build(leaves.data_ptr(), n_rows, n_cols, nodes_out.data_ptr()),
               "goldi_merkle_build")
    return nodes_out


def goldi_merkle_build_async(leaves, n_rows, n_cols, nodes_out, dev_status, stream=None):
    n_rows, n_cols = _positive(n_rows, "n_rows"), _positive(n_cols, "n_cols")
    _dev_u64(leaves, "leaves", n_rows * n_cols)
    _dev_u64(nodes_out, "nodes_out", goldi_merkle_num_nodes(n_rows) * DIGEST, leaves.device)
    _dev_status(dev_status, 1, leaves.device)
    with _torch().cuda.device(leaves.device):
        _check(lib().goldi_merkle_build_async(leaves.data_ptr(), n_rows, n_cols, nodes_out.data_ptr(),
                                              dev_status.data_ptr(), _stream_ptr(stream)),
               "goldi_merkle_build_async")
    return nodes_out


def _tree_array(trees):
    if len(trees) == 0:
        raise ValueError("need at least one tree")
    dev = trees[0][0].device if hasattr(trees[0][0], "device") else None
    arr = (_Tree * len(trees))()
    for k, (leaves, n_rows, n_cols, out) in enumerate(trees):
        n_rows, n_cols = _positive(n_rows, "n_rows"), _positive(n_cols, "n_cols")
        _dev_u64(leaves, "leaves of tree %d" % k, n_rows * n_cols, dev)
        _dev_u64(out, "nodes_out of tree %d" % k, goldi_merkle_num_nodes(n_rows) * DIGEST, dev)
        arr[k] = _Tree(leaves.data_ptr(), n_rows, n_cols, out.data_ptr())
    return arr


def goldi_merkle_build_many(trees, outputs=None):
    """``trees``: list of ``(leaves, n_rows, n_cols)``; returns the list of node tensors."""
    if outputs is None:
        outputs = [_alloc(goldi_merkle_num_nodes(n) * DIGEST, lv).view(-1, DIGEST) for lv, n, _ in trees]
    if len(outputs) != len(trees):
        raise ValueError("one output per tree")
    arr = _tree_array([(lv, n, w, o) for (lv, n, w), o in zip(trees, outputs)])
    with _torch().cuda.device(trees[0][0].device):
        _check(lib().goldi_merkle_build_many(arr, len(trees)), "goldi_merkle_build_many")
    return outputs


def goldi_merkle_build_many_async(trees, outputs, dev_status, stream=None):
    if len(outputs) != len(trees):
        raise ValueError("one output per tree")
    arr = _tree_array([(lv, n, w, o) for (lv, n, w), o in zip(trees, outputs)])
    _dev_status(dev_status, 1, trees[0][0].device)
    with _torch().cuda.device(trees[0][0].device):
        _check(lib().goldi_merkle_build_many_async(arr, len(trees), dev_status.data_ptr(), _stream_ptr(stream)),
               "goldi_merkle_build_many_async")
    return outputs


def goldi_merkle_build_many_status_async(trees, outputs, dev_status, stream=None):
    """Like goldi_merkle_build_many_async, with one status word per tree:
    ``dev_status`` is a zeroed int32 device tensor of at least len(trees) words."""
    if len(outputs) != len(trees):
        raise ValueError("one output per tree")
    arr = _tree_array([(lv, n, w, o) for (lv, n, w), o in zip(trees, outputs)])
    _dev_status(dev_status, len(trees), trees[0][0].device)
    with _torch().cuda.device(trees[0][0].device):
        _check(lib().goldi_merkle_build_many_status_async(arr, len(trees), dev_status.data_ptr(),
                                                          _stream_ptr(stream)),
               "goldi_merkle_build_many_status_async")
    return outputs


def goldi_profile_enable(on: bool = True) -> None:
    """Bracket every kernel launch with HIP events on its own stream."""
    _check(lib().goldi_profile_enable(1 if on else 0), "goldi_profile_enable")


def goldi_profile_select(kernel=None) -> None:
    """Time only one kernel kind (None: all kinds)."""
    _check(lib().goldi_profile_select(kernel.encode() if kernel else None), "goldi_profile_select")


def goldi_profile_read(kernel: str):
    """(total_ms, launches) of the recorded launches of one kernel kind; clears them."""
    ms, cnt = ctypes.c_double(), ctypes.c_size_t()
    _check(lib().goldi_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "goldi_profile_read")
    return ms.value, cnt.value


TUNE_KEYS = ("quad_max_rows", "quad_max_parents", "lane12_max_rows", "lane12_max_parents", "top_max_parents",
             "split_parts", "split_min_rows", "split_join_parents", "batch_mode", "graph")


def goldi_tune_set(key: str, value: int) -> None:
    """Set a schedule knob (one of TUNE_KEYS, documented in include/goldi.h);
    every setting computes the same bytes, only speed changes."""
    _check(lib().goldi_tune_set(key.encode(), value), "goldi_tune_set")


def goldi_tune_get(key: str) -> int:
    """Current value of a schedule knob, or of the read-only "partial_form"
    (how the loaded library evaluates the partial rounds: 2 blocks, 1 sparse, 0 dense)."""
    v = ctypes.c_size_t()
    _check(lib().goldi_tune_get(key.encode(), ctypes.byref(v)), "goldi_tune_get")
    return v.value


def goldi_admission_plan(pending_bytes, budget: int, inflight_bytes: int, max_group: int) -> int:
    """How many requests from the head of the queue the server admits together."""
    arr = (ctypes.c_size_t * max(1, len(pending_bytes)))(*pending_bytes)
    take = ctypes.c_size_t()
    _check(lib().goldi_admission_plan(arr, len(pending_bytes), budget, inflight_bytes, max_group,
                                      ctypes.byref(take)), "goldi_admission_plan")
    return take.value


class GoldiServer:
    """Serving loop with continuous batching (goldi_server_* in include/goldi.h)."""

    def __init__(self, hbm_budget_bytes: int, n_slots: int = 8, max_group: int = 8):
        import torch
        self._device = torch.cuda.current_device()
        h = ctypes.c_void_p()
        _check(lib().goldi_server_create(hbm_budget_bytes, n_slots, max_group, ctypes.byref(h)),
               "goldi_server_create")
        self._h = h
        self._keep = {}   # inputs referenced until their request completes

    def submit(self, leaves, n_rows: int, n_cols: int) -> int:
        """Queue a build; `leaves` is a uint64 torch tensor (device, or host --
        pinned for asynchronous copies) or a uint64 numpy array (host)."""
        import numpy as np
        rid = ctypes.c_uint64()
        host = dev = None
        if isinstance(leaves, np.ndarray):
            if leaves.dtype != np.uint64 or not leaves.flags.c_contiguous:
                raise TypeError("host leaves must be a contiguous uint64 array")
            host = leaves.ctypes.data
        else:
            torch = _torch()
            if leaves.dtype != torch.uint64 or not leaves.is_contiguous():
                raise TypeError("leaves must be a contiguous torch.uint64 tensor")
            if leaves.is_cuda:
                if leaves.device.index != self._device:
                    raise ValueError("leaves are on %s, the server on cuda:%d" % (leaves.device, self._device))
                dev = leaves.data_ptr()
            else:
                host = leaves.data_ptr()
        count = leaves.size if isinstance(leaves, np.ndarray) else leaves.numel()
        if count < n_rows * n_cols:
            raise ValueError("leaves hold fewer than n_rows * n_cols words")
        with _torch().cuda.device(self._device):
            _check(lib().goldi_server_submit(self._h, host, dev, n_rows, n_cols, ctypes.byref(rid)),
                   "goldi_server_submit")
        self._keep[rid.value] = leaves
        return rid.value

    def wait(self, rid: int) -> dict:
        info = _ReqInfo()
        _check(lib().goldi_server_wait(self._h, rid, ctypes.byref(info)), "goldi_server_wait")
        self._keep.pop(rid, None)
        return {"status": info.status, "n_rows": info.n_rows, "n_cols": info.n_cols, "nodes_ptr": info.nodes,
                "t_submit_ns": info.t_submit_ns, "t_admit_ns": info.t_admit_ns, "t_done_ns": info.t_done_ns,
                "group_size": info.group_size, "root": [int(v) for v in info.root]}

    def nodes(self, rid: int):
        """Copy of a completed, unreleased request's nodes as a [num_nodes, 4]
        uint64 device tensor."""
        torch = _torch()
        info = _ReqInfo()
        _check(lib().goldi_server_wait(self._h, rid, ctypes.byref(info)), "goldi_server_wait")
        n = goldi_merkle_num_nodes(info.n_rows) * DIGEST
        out = torch.empty(n, dtype=torch.uint64, device="cuda:%d" % self._device)
        _check(lib().goldi_server_read_nodes(self._h, rid, out.data_ptr(), n), "goldi_server_read_nodes")
        return out.view(-1, DIGEST)

    def release(self, rid: int) -> None:
        _check(lib().goldi_server_release(self._h, rid), "goldi_server_release")

    def set(self, key: str, value: int) -> None:
        """Server setting: "watchdog_us" or the test hook "fail_next_batches"
        (see goldi_server_set in include/goldi.h)."""
        _check(lib().goldi_server_set(self._h, key.encode(), value), "goldi_server_set")

    def stats(self) -> dict:
        a, g, p = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib().goldi_server_stats(self._h, ctypes.byref(a), ctypes.byref(g), ctypes.byref(p)),
               "goldi_server_stats")
        return {"admitted": a.value, "groups": g.value, "peak_bytes": p.value}

    def close(self) -> None:
        if self._h is not None:
            _check(lib().goldi_server_destroy(self._h), "goldi_server_destroy")
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
