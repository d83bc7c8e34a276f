"""Pins of the oracle's sponge (Sec. 2.4 "Poseidon Hash") and Merkle tree
(Sec. 2.4 "Merkle Tree", Sec. 4.2): closed forms in terms of the permutation,
a recursive big-integer definition of the tree, and the one-path invariant."""

import numpy as np
import pytest

import oracle
from oracle import mini
from synth.constants import CONSTANTS_PATH, build_spec, spec_bytes
from synth.inputs import leaves_colmajor

P = oracle.P


@pytest.fixture(scope="module")
def prm():
    return oracle.spec_params()


def rows_of(lv, n, w):
    return lv.reshape(w, n).T   # column-major flat -> [n][w]


def test_constants_file_reproducible():
    with open(CONSTANTS_PATH, "rb") as f:
        assert f.read() == spec_bytes(build_spec())


def test_matrix_and_submatrix_invertible(prm):
    # Needed for the inverse pin and by any sparse partial-round form.
    mini._mat_inv(prm.mds)
    mini._mat_inv([row[1:] for row in prm.mds[1:]])


@pytest.mark.parametrize("w", [1, 3, 8])
def test_sponge_single_chunk(prm, w):
    n = 5
    lv = leaves_colmajor(n, w, seed=21)
    d = oracle.leaf_hash(prm, lv, n, w)
    st = np.zeros((n, 12), dtype=np.uint64)
    st[:, :w] = rows_of(lv, n, w)
    want = oracle.permute(prm, st)[:, :4]
    assert (d == want).all()


@pytest.mark.parametrize("w", [9, 12, 16, 24])
def test_sponge_multi_chunk(prm, w):
    n = 4
    lv = leaves_colmajor(n, w, seed=22)
    rows = rows_of(lv, n, w)
    d = oracle.leaf_hash(prm, lv, n, w)
    for r in range(n):
        s = [0] * 12
        for k in range(0, w, 8):
            chunk = [int(v) for v in rows[r, k:k + 8]]
            for i, v in enumerate(chunk):
                s[i] = (s[i] + v) % P
            s = [int(v) for v in oracle.permute(prm, np.array([s], dtype=np.uint64))[0]]
        assert [int(v) for v in d[r]] == s[:4]


def test_node_counts():
    for n in range(1, 70):
        sizes = oracle.level_sizes(n)
        assert oracle.num_nodes(n) == sum(sizes)
        if n & (n - 1) == 0:
            assert oracle.num_nodes(n) == 2 * n - 1


@pytest.mark.parametrize("n,w", [(1, 8), (2, 8), (3, 1), (5, 9), (7, 8), (8, 16), (13, 7),
                                 (16, 8), (17, 3), (33, 8)])
def test_tree_vs_bigint_recursion(prm, n, w):
    lv = leaves_colmajor(n, w, seed=100 + n)
    nodes = oracle.merkle_build(prm, lv, n, w)
    rows = rows_of(lv, n, w)
    digests = [mini.sponge([int(v) for v in rows[r]], prm.rc, prm.mds) for r in range(n)]
    levels = mini.merkle_levels(digests, prm.rc, prm.mds)
    flat = [d for lev in levels for d in lev]
    assert [[int(v) for v in row] for row in nodes] == flat
    assert [int(v) for v in nodes[-1]] == mini.merkle_root_recursive(digests, prm.rc, prm.mds)


def test_single_leaf_tree(prm):
    lv = leaves_colmajor(1, 8, seed=5)
    nodes = oracle.merkle_build(prm, lv, 1, 8)
    assert nodes.shape == (1, 4)
    assert (nodes[0] == oracle.leaf_hash(prm, lv, 1, 8)[0]).all()


@pytest.mark.parametrize("n", [16, 21, 64])
def test_one_leaf_flip_changes_one_path(prm, n):
    w = 8
    lv = leaves_colmajor(n, w, seed=31)
    a = oracle.merkle_build(prm, lv, n, w)
    for r in (0, n // 2, n - 1):
        lv2 = lv.copy()
        lv2[3 * n + r] = (lv2[3 * n + r] + np.uint64(1)) % np.uint64(P)
        b = oracle.merkle_build(prm, lv2, n, w)
        changed = np.nonzero((a != b).any(axis=1))[0]
        sizes = oracle.level_sizes(n)
        want, off, idx = [], 0, r
        for s in sizes:
            want.append(off + idx)
            off += s
            idx //= 2
        assert list(changed) == want


def test_level_function_matches_build(prm):
    n, w = 11, 8
    lv = leaves_colmajor(n, w, seed=41)
    nodes = oracle.merkle_build(prm, lv, n, w)
    lvl0 = oracle.leaf_hash(prm, lv, n, w)
    lvl1 = oracle.merkle_level(prm, lvl0)
    assert (nodes[:n] == lvl0).all() and (nodes[n:n + 6] == lvl1).all()
    # last odd node moves up unchanged
    assert (lvl1[5] == lvl0[10]).all()


def test_golden_regression(prm):
    import json
    import os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_vectors.json")))
    ins = np.array([[int(v) for v in s] for s in g["permute"]["inputs"]], dtype=np.uint64)
    outs = [[int(v) for v in s] for s in g["permute"]["outputs"]]
    assert [[int(v) for v in s] for s in oracle.permute(prm, ins)] == outs
    n, w = 1 << 10, 8
    nodes = oracle.merkle_build(prm, leaves_colmajor(n, w, seed=0), n, w)
    assert [int(v) for v in nodes[-1]] == [int(v) for v in g["tree_1024x8_seed0"]["root"]]
