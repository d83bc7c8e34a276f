"""GPU parity: the HIP path (through the C ABI) against the CPU oracle,
word for word.  Every comparison is exact (tolerance 0): the method is exact
integer arithmetic and each input has exactly one correct output."""

import numpy as np
import pytest

import oracle
import paper_2506_09505_amd as goldi
from synth.inputs import GOLDILOCKS_P, edge_states, leaves_colmajor, uniform_states

from .gpu_util import banner, level_offsets, rows_from_colmajor, to_dev, to_host

pytestmark = pytest.mark.gpu
P = GOLDILOCKS_P


@pytest.fixture(scope="module")
def prm():
    return oracle.spec_params()


def test_library_is_native():
    assert goldi.lib() is not None
    import torch
    assert torch.cuda.is_available()


@pytest.mark.parametrize("n", [1, 63, 64, 65, 1000, 4096 + 17])
def test_permute_small(prm, n):
    banner("permute n=%d" % n)
    x = uniform_states(n, seed=1000 + n)
    d = to_dev(x)
    goldi.goldi_poseidon_permute(d)
    assert (to_host(d).reshape(n, 12) == oracle.permute(prm, x)).all()


def test_permute_edge_states(prm):
    banner("permute edge states")
    x = edge_states()
    d = to_dev(x)
    goldi.goldi_poseidon_permute(d)
    assert (to_host(d).reshape(-1, 12) == oracle.permute(prm, x)).all()


def test_permute_large(prm):
    n = 1 << 18
    banner("permute n=%d" % n)
    x = uniform_states(n, seed=7)
    d = to_dev(x)
    goldi.goldi_poseidon_permute(d)
    assert (to_host(d).reshape(n, 12) == oracle.permute(prm, x)).all()


def test_permute_bench_size_sampled(prm):
    # The size the benchmark times (2^24 states, 1.5 GiB); sampled outputs.
    n = 1 << 24
    banner("permute n=%d sampled" % n)
    x = uniform_states(n, seed=8)
    d = to_dev(x)
    goldi.goldi_poseidon_permute(d)
    y = to_host(d).reshape(n, 12)
    idx = np.unique(np.concatenate([np.arange(64), n - 1 - np.arange(64),
                                    np.random.default_rng(0).integers(0, n, 4096)]))
    assert (y[idx] == oracle.permute(prm, x[idx])).all()
    assert (y < np.uint64(P)).all()


def check_tree_full(prm, n, w, seed):
    lv = leaves_colmajor(n, w, seed=seed)
    got = to_host(goldi.goldi_merkle_build(to_dev(lv), n, w)).reshape(-1, 4)
    want = oracle.merkle_build(prm, lv, n, w)
    assert got.shape == want.shape
    bad = np.nonzero((got != want).any(axis=1))[0]
    assert bad.size == 0, "first mismatching nodes %s" % bad[:8]


def test_tree_plain_small(prm):
    # Plain single tree, 2^10 leaves x 8 words, seed 0: every node.
    banner("tree 1024x8 seed 0")
    check_tree_full(prm, 1 << 10, 8, 0)


@pytest.mark.parametrize("n", [1, 2, 3, 5, 7, 64, 255, 256, 257, 1000, 4097])
@pytest.mark.parametrize("w", [1, 7, 8, 9, 16, 33])
def test_tree_shapes(prm, n, w):
    banner("tree %dx%d" % (n, w))
    check_tree_full(prm, n, w, seed=n * 131 + w)


def test_tree_wide_ragged(prm):
    banner("tree 3001x256")
    check_tree_full(prm, 3001, 256, seed=2)


def test_tree_65536(prm):
    banner("tree 65536x8")
    check_tree_full(prm, 1 << 16, 8, seed=5)


def test_leaf_hash_entry(prm):
    n, w = 1000, 24
    banner("leaf hash %dx%d" % (n, w))
    lv = leaves_colmajor(n, w, seed=9)
    got = to_host(goldi.goldi_leaf_hash(to_dev(lv), n, w)).reshape(n, 4)
    assert (got == oracle.leaf_hash(prm, lv, n, w)).all()


def test_tree_paper_scale_sampled(prm):
    # Plain single tree at the paper's scale: 2^22 leaves x 8 words, seed 1.
    n, w = 1 << 22, 8
    banner("tree %dx%d sampled" % (n, w))
    lv = leaves_colmajor(n, w, seed=1)
    nodes = to_host(goldi.goldi_merkle_build(to_dev(lv), n, w)).reshape(-1, 4)
    offs, sizes = level_offsets(n)
    assert nodes.shape[0] == sum(sizes) == 2 * n - 1
    assert (nodes < np.uint64(P)).all()
    rng = np.random.default_rng(1)
    # leaves: sampled rows hashed by the oracle
    rows = np.unique(np.concatenate([[0, 1, n - 1], rng.integers(0, n, 2048)]))
    sub = rows_from_colmajor(lv, n, w, rows)
    assert (nodes[rows] == oracle.leaf_hash(prm, sub, rows.size, w)).all()
    # every level: sampled parents recomputed from the GPU's children
    for lvl in range(1, len(sizes)):
        m = sizes[lvl]
        idx = np.unique(np.concatenate([[0, m - 1], rng.integers(0, m, min(m, 512))]))
        ch = offs[lvl - 1] + 2 * idx
        pairs = np.stack([nodes[ch], nodes[ch + 1]], axis=1).reshape(-1, 4)
        assert (nodes[offs[lvl] + idx] == oracle.merkle_level(prm, pairs)).all(), "level %d" % lvl


def test_many_equals_plain(prm):
    banner("build_many")
    shapes = [(1, 8), (100, 16), (1 << 12, 8), (777, 9), (5000, 1)]
    trees = [(to_dev(leaves_colmajor(n, w, seed=40 + k)), n, w) for k, (n, w) in enumerate(shapes)]
    outs = goldi.goldi_merkle_build_many(trees)
    for (lv, n, w), o in zip(trees, outs):
        assert (to_host(o) == to_host(goldi.goldi_merkle_build(lv, n, w))).all()
        assert (to_host(o).reshape(-1, 4) == oracle.merkle_build(prm, to_host(lv), n, w)).all()


def test_async_on_torch_stream(prm):
    import torch
    banner("async build on a side stream")
    n, w = 3000, 8
    lv = leaves_colmajor(n, w, seed=50)
    d = to_dev(lv)
    out = torch.empty(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device="cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        goldi.goldi_merkle_build_async(d, n, w, out, status, stream=s)
    s.synchronize()
    assert int(status.item()) == 0
    assert (to_host(out).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all()


def test_device_generator_matches_host():
    from synth import fill
    from synth.inputs import words_at
    banner("device input generator")
    n = (1 << 20) + 3
    t = fill.leaves_colmajor_dev(n, 1, seed=77, stream=5)
    got = to_host(t)
    assert (got == leaves_colmajor(n, 1, seed=77, stream=5)).all()
    idx = np.array([0, 1, n - 1])
    assert (got[idx] == words_at(77, 5, idx)).all()


BIG = 1 << 40


@pytest.mark.parametrize("rows,parents,l12_rows,l12_parents", [
    (0, 0, 0, 0), (BIG, BIG, 0, 0), (0, BIG, 0, 0), (BIG, 0, 0, 0), (100, 7, 0, 0),
    (0, 0, BIG, BIG), (BIG, BIG, 3, 300), (0, 0, 0, BIG), (0, 0, BIG, 0), (5000, 5000, 64, 17)])
def test_schedule_independence(prm, rows, parents, l12_rows, l12_parents):
    # Every schedule (one, four or twelve lanes per state, at any cut-over)
    # must write the same bytes.
    banner("schedule quad %d/%d lane12 %d/%d" % (rows, parents, l12_rows, l12_parents))
    keys = ("quad_max_rows", "quad_max_parents", "lane12_max_rows", "lane12_max_parents")
    old = [goldi.goldi_tune_get(k) for k in keys]
    try:
        for k, v in zip(keys, (rows, parents, l12_rows, l12_parents)):
            goldi.goldi_tune_set(k, v)
        for n, w in [(1, 8), (3, 9), (200, 8), (1000, 33), (5000, 8)]:
            check_tree_full(prm, n, w, seed=7 * n + w)
    finally:
        for k, v in zip(keys, old):
            goldi.goldi_tune_set(k, v)


@pytest.mark.parametrize("top", [0, 1, 2, 7, 64])
def test_top_of_tree_in_one_launch(prm, top):
    # The levels from the first one of at most `top` parents up to the root run
    # in one single-workgroup launch (0: every level its own launch); ragged
    # levels and trees that start below the cut-over included.
    banner("top of tree, top_max_parents %d" % top)
    old = goldi.goldi_tune_get("top_max_parents")
    try:
        goldi.goldi_tune_set("top_max_parents", top)
        for n, w in [(1, 8), (2, 3), (3, 8), (5, 8), (13, 9), (127, 8), (128, 8), (129, 8), (300, 1), (4097, 8)]:
            check_tree_full(prm, n, w, seed=11 * n + w + top)
    finally:
        goldi.goldi_tune_set("top_max_parents", old)


def test_tree_wide_rows_full_size_sampled(prm):
    # Wide-row commitment tree: 2^21 rows x 256 columns, column-major (4 GiB),
    # seed 2; generated on the device; sampled rows and parents checked.
    import torch
    from synth import fill
    from synth.inputs import words_at
    n, w, seed = 1 << 21, 256, 2
    banner("tree %dx%d sampled" % (n, w))
    lv = fill.leaves_colmajor_dev(n, w, seed=seed)
    nodes_t = goldi.goldi_merkle_build(lv, n, w)
    del lv
    torch.cuda.empty_cache()
    nodes = to_host(nodes_t).reshape(-1, 4)
    offs, sizes = level_offsets(n)
    assert nodes.shape[0] == 2 * n - 1 and (nodes < np.uint64(P)).all()
    rng = np.random.default_rng(3)
    rows = np.unique(np.concatenate([[0, n - 1], rng.integers(0, n, 254)]))
    cols = np.arange(w, dtype=np.int64)
    sub = words_at(seed, 0, (cols[:, None] * n + rows[None, :]).reshape(-1))
    assert (nodes[rows] == oracle.leaf_hash(prm, sub, rows.size, w)).all()
    for lvl in range(1, len(sizes)):
        m = sizes[lvl]
        idx = np.unique(np.concatenate([[0, m - 1], rng.integers(0, m, min(m, 256))]))
        ch = offs[lvl - 1] + 2 * idx
        pairs = np.stack([nodes[ch], nodes[ch + 1]], axis=1).reshape(-1, 4)
        assert (nodes[offs[lvl] + idx] == oracle.merkle_level(prm, pairs)).all(), "level %d" % lvl


def test_golden_vectors_on_gpu():
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_vectors.json")))
    ins = np.array([[int(v) for v in s] for s in g["permute"]["inputs"]], dtype=np.uint64)
    d = to_dev(ins)
    goldi.goldi_poseidon_permute(d)
    assert [[int(v) for v in s] for s in to_host(d).reshape(-1, 12)] == \
        [[int(v) for v in s] for s in g["permute"]["outputs"]]
    n, w = 1 << 10, 8
    nodes = to_host(goldi.goldi_merkle_build(to_dev(leaves_colmajor(n, w, seed=0)), n, w)).reshape(-1, 4)
    assert [int(v) for v in nodes[-1]] == [int(v) for v in g["tree_1024x8_seed0"]["root"]]
