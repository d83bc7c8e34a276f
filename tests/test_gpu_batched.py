"""GPU: batched many-tree builds (goldi_merkle_build_many) against the plain
single-tree build and the oracle, under every schedule (per-tree launches,
batched level launches, captured and replayed hipGraphs)."""

import numpy as np
import pytest

import oracle
import paper_2506_09505_amd as goldi
from synth.inputs import leaves_colmajor, tree_shapes

from .gpu_util import level_offsets, rows_from_colmajor, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prm():
    return oracle.spec_params()


@pytest.fixture
def knobs():
    keys = ("batch_mode", "graph", "quad_max_rows", "quad_max_parents", "lane12_max_rows", "lane12_max_parents")
    old = {k: goldi.goldi_tune_get(k) for k in keys}
    yield goldi.goldi_tune_set
    for k, v in old.items():
        goldi.goldi_tune_set(k, v)


def banner(msg):
    print("[case] " + msg, flush=True)


def small_batch(seed, count, lo=0, hi=12, widths=(1, 7, 8, 9, 16, 33)):
    rows, ws = tree_shapes(seed, count, lo, hi, widths)
    return [(int(n), int(w), leaves_colmajor(int(n), int(w), seed=seed * 1000 + k))
            for k, (n, w) in enumerate(zip(rows, ws))]


@pytest.mark.parametrize("batch_mode,graph", [(0, 0), (1, 0), (1, 1)])
def test_many_vs_oracle(prm, knobs, batch_mode, graph):
    knobs("batch_mode", batch_mode)
    knobs("graph", graph)
    banner("build_many batch_mode=%d graph=%d" % (batch_mode, graph))
    batch = small_batch(11, 23)
    trees = [(to_dev(lv), n, w) for n, w, lv in batch]
    outs = goldi.goldi_merkle_build_many(trees)
    for (n, w, lv), o in zip(batch, outs):
        assert (to_host(o).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all(), (n, w)


def test_more_than_64_trees(prm, knobs):
    knobs("batch_mode", 1)
    banner("build_many 70 trees")
    batch = small_batch(12, 70, 0, 9)
    trees = [(to_dev(lv), n, w) for n, w, lv in batch]
    outs = goldi.goldi_merkle_build_many(trees)
    for (n, w, lv), o in zip(batch, outs):
        assert (to_host(o).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all(), (n, w)


def test_quad_cutovers_in_batches(prm, knobs):
    banner("build_many quad cut-overs")
    batch = small_batch(13, 9)
    trees = [(to_dev(lv), n, w) for n, w, lv in batch]
    want = [oracle.merkle_build(prm, lv, n, w) for n, w, lv in batch]
    for rows, parents, l12r, l12p in [(0, 0, 0, 0), (1 << 40, 1 << 40, 0, 0), (50, 3000, 0, 0),
                                      (0, 0, 1 << 40, 1 << 40), (1 << 40, 1 << 40, 20, 700)]:
        knobs("quad_max_rows", rows)
        knobs("quad_max_parents", parents)
        knobs("lane12_max_rows", l12r)
        knobs("lane12_max_parents", l12p)
        outs = goldi.goldi_merkle_build_many(trees)
        for o, w_ in zip(outs, want):
            assert (to_host(o).reshape(-1, 4) == w_).all()


@pytest.mark.parametrize("forced", [True, False])
def test_single_chunk_batches(prm, knobs, forced):
    # Every tree of the batch has rows of at most 8 words, so the batched leaf
    # kernel takes its single-absorption form; forced onto one lane per state
    # for small trees, and by size with the default cut-overs.
    banner("build_many single-chunk rows, forced=%s" % forced)
    if forced:
        for k in ("quad_max_rows", "quad_max_parents", "lane12_max_rows", "lane12_max_parents"):
            knobs(k, 0)
        batch = small_batch(14, 12, 0, 11, widths=(1, 5, 8))
    else:
        batch = small_batch(15, 6, 13, 16, widths=(2, 8))
    trees = [(to_dev(lv), n, w) for n, w, lv in batch]
    outs = goldi.goldi_merkle_build_many(trees)
    for (n, w, lv), o in zip(batch, outs):
        assert (to_host(o).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all(), (n, w)


def test_graph_replays_with_eager_work_between(prm, knobs):
    # A captured graph is replayed several times, with other (eager) work and
    # synchronisations in between; every replay must equal the eager result.
    import torch
    knobs("batch_mode", 1)
    banner("graph replays")
    batch = small_batch(14, 12)
    trees = [(to_dev(lv), n, w) for n, w, lv in batch]
    knobs("graph", 0)
    eager = [to_host(o).reshape(-1) for o in goldi.goldi_merkle_build_many(trees)]
    knobs("graph", 1)
    outs = [torch.zeros_like(torch.empty(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device="cuda:0"))
            for _, n, _ in trees]
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    for rep in range(4):
        for o in outs:
            o.view(torch.int64).fill_(-1)      # eager work between replays
        torch.cuda.synchronize()
        goldi.goldi_merkle_build_many_async(trees, outs, status)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        for o, e in zip(outs, eager):
            assert (to_host(o).reshape(-1) == e).all(), "replay %d" % rep
        goldi.goldi_merkle_build(trees[0][0], trees[0][1], trees[0][2])   # more eager work


def test_batched_workload_full_size(prm, knobs):
    # Batched workload: 64 trees, rows log-uniform in [2^10, 2^20], widths in
    # {8, 16, 32, 64, 128}, seed 3 (device-generated inputs).  Batched output
    # must equal 64 plain builds word for word; sampled nodes are checked
    # against the oracle.
    import torch
    from synth import fill
    from synth.inputs import words_at
    rows, ws = tree_shapes(3, 64, 10, 20, (8, 16, 32, 64, 128))
    banner("batched 64 trees, %d rows total" % int(rows.sum()))
    trees = [(fill.leaves_colmajor_dev(int(n), int(w), seed=3, stream=k), int(n), int(w))
             for k, (n, w) in enumerate(zip(rows, ws))]
    knobs("batch_mode", 1)
    outs = goldi.goldi_merkle_build_many(trees)
    rng = np.random.default_rng(4)
    for k, ((lv, n, w), o) in enumerate(zip(trees, outs)):
        plain = goldi.goldi_merkle_build(lv, n, w)
        assert torch.equal(o.view(torch.int64), plain.view(torch.int64)), "tree %d" % k
        if k % 8 == 0:
            nodes = to_host(o).reshape(-1, 4)
            r = np.unique(rng.integers(0, n, 16))
            cols = np.arange(w, dtype=np.int64)
            sub = words_at(3, k, (cols[:, None] * n + r[None, :]).reshape(-1))
            assert (nodes[r] == oracle.leaf_hash(prm, sub, r.size, w)).all()
            offs, sizes = level_offsets(n)
            for lvl in range(1, len(sizes)):
                idx = np.unique(rng.integers(0, sizes[lvl], 8))
                ch = offs[lvl - 1] + 2 * idx
                ok = ch + 1 < offs[lvl - 1] + sizes[lvl - 1]
                idx, ch = idx[ok], ch[ok]
                if idx.size:
                    pairs = np.stack([nodes[ch], nodes[ch + 1]], axis=1).reshape(-1, 4)
                    assert (nodes[offs[lvl] + idx] == oracle.merkle_level(prm, pairs)).all()


@pytest.mark.parametrize("batch_mode", [1, 0])
def test_per_tree_status(prm, knobs, batch_mode):
    # One status word per tree: a non-canonical word marks its own tree only,
    # and every other tree of the call equals the oracle.
    import torch
    from synth.inputs import GOLDILOCKS_P
    knobs("batch_mode", batch_mode)
    banner("per-tree status, batch_mode %d" % batch_mode)
    batch = small_batch(16, 6, 4, 11, widths=(8, 9, 16))
    n_bad, w_bad, lv_bad = batch[2]
    lv_bad = lv_bad.copy()
    lv_bad[(w_bad - 1) * n_bad + n_bad // 2] = np.uint64(GOLDILOCKS_P + 3)
    batch[2] = (n_bad, w_bad, lv_bad)
    trees = [(to_dev(lv), n, w) for n, w, lv in batch]
    outs = [torch.empty(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device="cuda:0")
            for _, n, _ in trees]
    status = torch.zeros(len(trees), dtype=torch.int32, device="cuda:0")
    goldi.goldi_merkle_build_many_status_async(trees, outs, status)
    torch.cuda.synchronize()
    assert status.cpu().tolist() == [0, 0, 1, 0, 0, 0]
    for k, ((n, w, lv), o) in enumerate(zip(batch, outs)):
        if k != 2:
            assert (to_host(o).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all(), k
    with pytest.raises(ValueError):
        goldi.goldi_merkle_build_many_status_async(trees, outs, status[:5])
