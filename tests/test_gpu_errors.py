"""GPU error paths: non-canonical input words are caught on the device and
reported as GOLDI_ENONCANON; bad pointers and sizes are rejected on the host
before anything is launched (GOLDI_EINVAL).  No case launches a kernel on
memory it does not own."""

import ctypes

import numpy as np
import pytest

import paper_2506_09505_amd as goldi
from synth.inputs import GOLDILOCKS_P, leaves_colmajor, uniform_states

from .gpu_util import to_dev

pytestmark = pytest.mark.gpu
P = GOLDILOCKS_P


def test_noncanonical_state_word():
    x = uniform_states(100, seed=3)
    x[57, 4] = np.uint64(P)
    with pytest.raises(goldi.GoldiError) as e:
        goldi.goldi_poseidon_permute(to_dev(x))
    assert e.value.code == goldi.GOLDI_ENONCANON


def test_noncanonical_leaf_word():
    n, w = 300, 9
    lv = leaves_colmajor(n, w, seed=4)
    lv[8 * n + 299] = np.uint64(2**64 - 1)
    with pytest.raises(goldi.GoldiError) as e:
        goldi.goldi_merkle_build(to_dev(lv), n, w)
    assert e.value.code == goldi.GOLDI_ENONCANON


def test_status_clears_between_calls():
    # A failed call must not poison the next one.
    x = uniform_states(10, seed=5)
    y = x.copy()
    y[0, 0] = np.uint64(P + 5)
    with pytest.raises(goldi.GoldiError):
        goldi.goldi_poseidon_permute(to_dev(y))
    goldi.goldi_poseidon_permute(to_dev(x))


def test_zero_and_null_arguments():
    L = goldi.lib()
    d = to_dev(uniform_states(4, seed=6))
    assert L.goldi_poseidon_permute(d.data_ptr(), 0) == goldi.GOLDI_EINVAL
    assert L.goldi_poseidon_permute(None, 4) == goldi.GOLDI_EINVAL
    assert L.goldi_merkle_build(d.data_ptr(), 0, 8, d.data_ptr()) == goldi.GOLDI_EINVAL
    assert L.goldi_merkle_build(d.data_ptr(), 4, 0, d.data_ptr()) == goldi.GOLDI_EINVAL
    assert L.goldi_merkle_build_many(None, 3) == goldi.GOLDI_EINVAL


def test_host_pointer_rejected():
    L = goldi.lib()
    host = np.zeros(12 * 4, dtype=np.uint64)
    assert L.goldi_poseidon_permute(host.ctypes.data, 4) == goldi.GOLDI_EINVAL
    assert b"device" in L.goldi_last_error()


def test_buffer_too_small_rejected():
    import torch
    L = goldi.lib()
    n, w = 1024, 8
    lv = to_dev(leaves_colmajor(n, w, seed=7))
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    # A node buffer one node short, a leaf matrix one word short, a status
    # tensor of the wrong type: the binding refuses each before any launch
    # (torch may carve the tensor out of a larger block, which the C side,
    # checking allocations, cannot see).
    short = torch.empty((goldi.goldi_merkle_num_nodes(n) - 1) * 4, dtype=torch.uint64, device="cuda:0")
    with pytest.raises(ValueError):
        goldi.goldi_merkle_build(lv, n, w, short)
    with pytest.raises(ValueError):
        goldi.goldi_merkle_build_async(lv, n, w, short, status)
    with pytest.raises(ValueError):
        goldi.goldi_merkle_build(lv[:-1], n, w)
    with pytest.raises(ValueError):
        goldi.goldi_leaf_hash(lv, n, w, torch.empty(n * 4 - 1, dtype=torch.uint64, device="cuda:0"))
    with pytest.raises(ValueError):
        goldi.goldi_merkle_build_many([(lv, n, w)], [short])
    with pytest.raises(TypeError):
        goldi.goldi_merkle_build_async(lv, n, w, torch.empty(goldi.goldi_merkle_num_nodes(n) * 4,
                                                             dtype=torch.uint64, device="cuda:0"),
                                       torch.zeros(1, dtype=torch.int64, device="cuda:0"))
    with pytest.raises(TypeError):
        goldi.goldi_merkle_build(leaves_colmajor(n, w, seed=7), n, w)
    # Claiming more rows than the leaf buffer holds is caught by the C side
    # too when the allocation is exactly sized.
    exact = torch.empty(n * w, dtype=torch.uint64, device="cuda:0")
    big_out = torch.empty(goldi.goldi_merkle_num_nodes(1 << 24) * 4, dtype=torch.uint64, device="cuda:0")
    assert L.goldi_merkle_build(exact.data_ptr(), 1 << 24, w, big_out.data_ptr()) == goldi.GOLDI_EINVAL


def test_overlap_rejected():
    L = goldi.lib()
    n, w = 64, 8
    buf = to_dev(np.zeros(n * w + goldi.goldi_merkle_num_nodes(n) * 4, dtype=np.uint64))
    assert L.goldi_merkle_build(buf.data_ptr(), n, w, buf.data_ptr() + 8 * 8) == goldi.GOLDI_EINVAL


def test_error_text():
    L = goldi.lib()
    assert L.goldi_strerror(goldi.GOLDI_ENONCANON) == b"input word not canonical (>= p)"
    assert isinstance(L.goldi_last_error(), bytes)
    assert ctypes.sizeof(goldi._Tree) == 32


def test_dispatch_limit():
    # One dispatch covers at most 2^32 - 1 work-items.  Too many states is
    # refused before any buffer is inspected; a tree whose row count times the
    # lanes per row (forced to 16 by the one-word-per-lane knob) crosses the
    # limit is refused at its first launch, so nothing runs.  (Unsplit: split
    # in two, each half's launch would stay below the limit.)
    import torch
    L = goldi.lib()
    d = to_dev(uniform_states(4, seed=8))
    assert L.goldi_poseidon_permute(d.data_ptr(), 1 << 32) == goldi.GOLDI_EINVAL
    n = (1 << 28) + 16
    lv = torch.empty(n, dtype=torch.uint64, device="cuda:0")
    out = torch.empty(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device="cuda:0")
    old = goldi.goldi_tune_get("lane12_max_rows")
    old_split = goldi.goldi_tune_get("split_parts")
    try:
        goldi.goldi_tune_set("lane12_max_rows", 1 << 40)
        goldi.goldi_tune_set("split_parts", 0)
        assert L.goldi_merkle_build(lv.data_ptr(), n, 1, out.data_ptr()) == goldi.GOLDI_EINVAL
        assert b"dispatch" in L.goldi_last_error()
    finally:
        goldi.goldi_tune_set("lane12_max_rows", old)
        goldi.goldi_tune_set("split_parts", old_split)
    del lv, out
    torch.cuda.empty_cache()
