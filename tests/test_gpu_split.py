"""GPU: single-tree builds split into row ranges on several streams
("split_parts"): the leaf hash and the wide levels of each range run on their
own stream and join on the caller's stream.  A split build must write the
same bytes as an unsplit one and as the oracle, for every part count and join
width, ragged sizes included, on the null stream, on a side stream and inside
a captured graph (where the library does not split)."""

import numpy as np
import pytest

import oracle
import paper_2506_09505_amd as goldi
from synth.inputs import GOLDILOCKS_P, leaves_colmajor

from .gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu
KEYS = ("split_parts", "split_min_rows", "split_join_parents")


@pytest.fixture(scope="module")
def prm():
    return oracle.spec_params()


@pytest.fixture
def split():
    old = {k: goldi.goldi_tune_get(k) for k in KEYS}

    def set_(parts, min_rows=None, join=None):
        goldi.goldi_tune_set("split_parts", parts)
        if min_rows is not None:
            goldi.goldi_tune_set("split_min_rows", min_rows)
        if join is not None:
            goldi.goldi_tune_set("split_join_parents", join)
    yield set_
    for k, v in old.items():
        goldi.goldi_tune_set(k, v)


@pytest.mark.parametrize("parts", [2, 3, 4])
@pytest.mark.parametrize("join", [16, 64, 700])
def test_split_small_trees_vs_oracle(prm, split, parts, join):
    # The split forced onto trees the oracle builds in moments: ragged row
    # counts, single- and multi-chunk rows, boundaries that are multiples of
    # 2^depth, and a last part with an odd number of nodes at several levels.
    split(parts, min_rows=64, join=join)
    for n, w in [(4096, 8), (5000, 9), (3001, 1), (777, 16)]:
        banner("split %d parts join %d, tree %dx%d" % (parts, join, n, w))
        lv = leaves_colmajor(n, w, seed=n + 3 * w + parts)
        got = to_host(goldi.goldi_merkle_build(to_dev(lv), n, w)).reshape(-1, 4)
        assert (got == oracle.merkle_build(prm, lv, n, w)).all(), (parts, join, n, w)


@pytest.mark.parametrize("n,w", [((1 << 21) + 12345, 9), ((1 << 20) + 1, 3), ((1 << 23) - 7, 8)])
def test_split_equals_unsplit_full_size(split, n, w):
    # Paper-scale shapes with ragged tails: every node of the 2-, 3- and
    # 4-part builds equals the unsplit build's (which the oracle pins
    # elsewhere), at the default join width.
    import torch
    from synth import fill
    x = fill.leaves_colmajor_dev(n, w, seed=7, device=torch.device("cuda:0"))
    outs = []
    for parts in (0, 2, 3, 4):
        banner("split %d parts, tree %dx%d" % (parts, n, w))
        split(parts, min_rows=1 << 20)
        outs.append(goldi.goldi_merkle_build(x, n, w))
    ref = outs[0].view(torch.int64)
    for parts, o in zip((2, 3, 4), outs[1:]):
        assert torch.equal(ref, o.view(torch.int64)), parts


def test_split_reports_a_bad_word_in_the_last_part(split):
    # A non-canonical word in the last row (hashed on a side stream) fails
    # the call like an unsplit build.
    split(2, min_rows=64, join=16)
    n, w = 5000, 8
    lv = leaves_colmajor(n, w, seed=31)
    lv[(w - 1) * n + n - 1] = np.uint64(GOLDILOCKS_P)
    banner("split build with p in the last row")
    with pytest.raises(goldi.GoldiError) as ei:
        goldi.goldi_merkle_build(to_dev(lv), n, w)
    assert ei.value.code == goldi.GOLDI_ENONCANON


def test_split_async_on_a_side_stream(prm, split):
    import torch
    split(2, min_rows=64, join=16)
    n, w = 6000, 8
    lv = leaves_colmajor(n, w, seed=32)
    d = to_dev(lv)
    out = torch.empty(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device="cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    banner("split async build on a side stream")
    with torch.cuda.stream(s):
        goldi.goldi_merkle_build_async(d, n, w, out, status, stream=s)
    s.synchronize()
    assert int(status.item()) == 0
    assert (to_host(out).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all()


def test_build_captured_in_a_graph_is_not_split(prm, split):
    # Inside a stream capture the library keeps every launch on the captured
    # stream.  Each replay (with eager work in between) must equal the eager
    # build.
    import torch
    split(2, min_rows=64, join=16)
    n, w = 6000, 8
    lv = leaves_colmajor(n, w, seed=33)
    d = to_dev(lv)
    want = oracle.merkle_build(prm, lv, n, w)
    out = torch.zeros(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device="cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    banner("split build captured into a graph")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside the capture
        goldi.goldi_merkle_build_async(d, n, w, out, status, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        goldi.goldi_merkle_build_async(d, n, w, out, status, stream=torch.cuda.current_stream())
    for rep in range(3):
        out.zero_()
        scratch = torch.arange(1 << 20, device="cuda:0").sum()  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        assert int(scratch.item()) == (1 << 20) * ((1 << 20) - 1) // 2
        assert int(status.item()) == 0
        assert (to_host(out).reshape(-1, 4) == want).all(), rep


def test_split_builds_from_two_host_threads(prm, split):
    # Two host threads build different trees at the same time, each on its own
    # stream; both splits share the library's second stream and its event
    # pool.  Each result must equal the oracle's.
    import threading
    import torch
    split(2, min_rows=64, join=16)
    shapes = [(5000, 8, 41), (4097, 9, 42)]
    host = [(n, w, leaves_colmajor(n, w, seed=s_)) for n, w, s_ in shapes]
    want = [oracle.merkle_build(prm, lv, n, w) for n, w, lv in host]
    dev = [to_dev(lv) for _, _, lv in host]
    outs = [torch.zeros(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device="cuda:0") for n, _, _ in host]
    stats = [torch.zeros(1, dtype=torch.int32, device="cuda:0") for _ in host]
    streams = [torch.cuda.Stream() for _ in host]
    for s_ in streams:
        s_.wait_stream(torch.cuda.current_stream())
    errors = []

    def worker(k):
        try:
            n, w, _ = host[k]
            for _ in range(20):
                goldi.goldi_merkle_build_async(dev[k], n, w, outs[k], stats[k], stream=streams[k])
            streams[k].synchronize()
        except Exception as e:  # reported below
            errors.append(e)

    banner("split builds from two host threads")
    threads = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for k in range(2):
        assert int(stats[k].item()) == 0
        assert (to_host(outs[k]).reshape(-1, 4) == want[k]).all(), k
