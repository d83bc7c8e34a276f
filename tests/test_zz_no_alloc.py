"""GPU: goldi_merkle_build_many_noalloc, the entry point that allocates
nothing (its per-tree status words live in a fixed device array inside the
library), called through the C ABI.  Its outputs must equal
goldi_merkle_build_many's word for word, on two calls in a row with the
second one smaller; it must report a bad tree alone; it must refuse more
trees than its array holds; and device memory must not change across calls."""

import ctypes

import numpy as np
import pytest

import paper_2506_09505_amd as goldi
from synth.inputs import GOLDILOCKS_P, leaves_colmajor, tree_shapes

from .gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu


def trees_for(seed, count, lo, hi, widths):
    rows, ws = tree_shapes(seed, count, lo, hi, widths)
    return [(int(n), int(w), leaves_colmajor(int(n), int(w), seed=seed, stream=k)) for k, (n, w) in enumerate(zip(rows, ws))]


def noalloc(batch_dev, outs):
    import torch
    L = goldi.lib()
    arr = (goldi._Tree * len(batch_dev))()
    for k, ((lv, n, w), o) in enumerate(zip(batch_dev, outs)):
        arr[k] = goldi._Tree(lv.data_ptr(), n, w, o.data_ptr())
    st = (ctypes.c_int * len(batch_dev))()
    rc = L.goldi_merkle_build_many_noalloc(arr, len(batch_dev), st, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return rc, list(st)


def empty_outs(batch_dev):
    import torch
    return [torch.full((goldi.goldi_merkle_num_nodes(n) * 4,), 7, dtype=torch.int64, device="cuda:0").view(torch.uint64)
            for _, n, _ in batch_dev]


def test_noalloc_equals_build_many_twice():
    import torch
    banner("noalloc: two calls, the second smaller")
    big = [(to_dev(lv), n, w) for n, w, lv in trees_for(31, 9, 8, 16, (1, 8, 9, 32, 64))]
    small = [(to_dev(lv), n, w) for n, w, lv in trees_for(32, 3, 2, 10, (8, 16))]
    for batch in (big, small):
        want = goldi.goldi_merkle_build_many(batch)
        outs = empty_outs(batch)
        rc, st = noalloc(batch, outs)
        assert rc == goldi.GOLDI_OK and st == [0] * len(batch)
        for o, w_ in zip(outs, want):
            assert torch.equal(o.view(torch.int64), w_.reshape(-1).view(torch.int64))


def test_noalloc_reports_a_bad_tree_alone():
    import torch
    banner("noalloc: one non-canonical tree among four")
    host = trees_for(33, 4, 4, 11, (8, 24))
    n, w, lv = host[1]
    lv = lv.copy()
    lv[n * (w - 1)] = np.uint64(GOLDILOCKS_P)
    host[1] = (n, w, lv)
    batch = [(to_dev(lv), n, w) for n, w, lv in host]
    outs = empty_outs(batch)
    rc, st = noalloc(batch, outs)
    assert rc == goldi.GOLDI_ENONCANON
    assert st == [0, goldi.GOLDI_ENONCANON, 0, 0]
    for k in (0, 2, 3):
        want = goldi.goldi_merkle_build(batch[k][0], batch[k][1], batch[k][2])
        assert torch.equal(outs[k].view(torch.int64), want.reshape(-1).view(torch.int64))
    # the next call starts from cleared words
    good = [batch[0], batch[2]]
    rc, st = noalloc(good, [outs[0], outs[2]])
    assert rc == goldi.GOLDI_OK and st == [0, 0]


def test_noalloc_refuses_too_many_trees():
    banner("noalloc: more trees than its array")
    L = goldi.lib()
    arr = (goldi._Tree * 4097)()
    assert L.goldi_merkle_build_many_noalloc(arr, 4097, None, None) == goldi.GOLDI_EINVAL
    assert b"4096" in L.goldi_last_error()
    assert L.goldi_merkle_build_many_noalloc(arr, 0, None, None) == goldi.GOLDI_EINVAL


def test_noalloc_allocates_nothing():
    import torch
    banner("noalloc: device memory unchanged across calls")
    batch = [(to_dev(lv), n, w) for n, w, lv in trees_for(34, 5, 6, 12, (8, 16))]
    outs = empty_outs(batch)
    for _ in range(2):                      # warm: code objects loaded, symbol resolved
        assert noalloc(batch, outs)[0] == goldi.GOLDI_OK
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(3):
        assert noalloc(batch, outs)[0] == goldi.GOLDI_OK
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    want = goldi.goldi_merkle_build_many(batch)
    for o, w_ in zip(outs, want):
        assert (to_host(o) == to_host(w_).reshape(-1)).all()


def test_noalloc_plain_schedule_keeps_one_stream():
    # With batch_mode 0 the trees go through the single-tree schedule, which
    # splits trees of 2^20 rows and more over two streams; the allocation-free
    # entry point keeps every tree on the caller's stream, with the same bytes.
    import torch
    from synth import fill
    banner("noalloc: plain schedule, a tree large enough to split elsewhere")
    old = goldi.goldi_tune_get("batch_mode")
    try:
        goldi.goldi_tune_set("batch_mode", 0)
        n, w = (1 << 20) + 5, 8
        lv = fill.leaves_colmajor_dev(n, w, seed=35, device=torch.device("cuda:0"))
        small = [(to_dev(lv_), n_, w_) for n_, w_, lv_ in trees_for(36, 2, 4, 9, (8,))]
        batch = [(lv, n, w)] + small
        outs = empty_outs(batch)
        rc, st = noalloc(batch, outs)
        assert rc == goldi.GOLDI_OK and st == [0, 0, 0]
        for (d, n_, w_), o in zip(batch, outs):
            want = goldi.goldi_merkle_build(d, n_, w_)
            assert torch.equal(o.view(torch.int64), want.reshape(-1).view(torch.int64))
    finally:
        goldi.goldi_tune_set("batch_mode", old)
