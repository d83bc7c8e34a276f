"""GPU path against closed forms, independently of the oracle.

The library is also compiled against three special instances whose
permutation has a closed form (paper_2506_09505_amd/gen_constants.py,
special_specs):
  identity  M = I, C = 0            word 0 -> x0^(7^30), words 1..11 -> x^(7^8)
  shift     M = one-place shift, C = 0  words travel one position per round;
            each S-box a word passes through multiplies its exponent by 7
  const     M = I, C[5][0] = 3, C[27][4] = 5
This pins the round counts, the S-box position, the matrix orientation and
the constant placement of every kernel layout (one, four and twelve lanes
per state) without the oracle."""

import ctypes
import os

import numpy as np
import pytest

from synth.inputs import GOLDILOCKS_P, goldilocks_words

from .gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu
P = GOLDILOCKS_P
FULL = [r < 4 or r >= 26 for r in range(30)]
BIG = 1 << 40


def closed_form(name, x):
    x = [int(v) for v in x]
    if name == "identity":
        return [pow(x[0], 7 ** 30, P)] + [pow(v, 7 ** 8, P) for v in x[1:]]
    if name == "const":
        out = [pow(v, 7 ** 8, P) for v in x]
        out[0] = pow((pow(x[0], 7 ** 5, P) + 3) % P, 7 ** 25, P)
        out[4] = pow((pow(x[4], 7 ** 5, P) + 5) % P, 7 ** 3, P)
        return out
    if name == "shift":
        # new_i = x_{i+1}: the word at position q moves to q - 1 each round.
        pos, exp = list(range(12)), [1] * 12
        for r in range(30):
            for k in range(12):
                if FULL[r] or pos[k] == 0:
                    exp[k] *= 7
            pos = [(q - 1) % 12 for q in pos]
        out = [0] * 12
        for k in range(12):
            out[pos[k]] = pow(x[k], exp[k], P)
        return out
    raise ValueError(name)


def load(name):
    import torch  # noqa: F401  (bind to torch's HIP runtime first)
    from paper_2506_09505_amd import build
    path = build.special_lib(name)
    assert os.path.exists(path), "build the special libraries first"
    L = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    L.goldi_poseidon_permute.argtypes = [vp, sz]
    L.goldi_leaf_hash.argtypes = [vp, sz, sz, vp]
    L.goldi_tune_set.argtypes = [ctypes.c_char_p, sz]
    return L


@pytest.mark.parametrize("name", ["identity", "shift", "const"])
def test_permute_closed_form(name):
    L = load(name)
    n = 256
    x = goldilocks_words(40, 0, 0, n * 12).reshape(n, 12)
    x[0] = np.arange(12, dtype=np.uint64)
    d = to_dev(x)
    assert L.goldi_poseidon_permute(d.data_ptr(), n) == 0
    got = to_host(d).reshape(n, 12)
    for row, g in zip(x, got):
        assert [int(v) for v in g] == closed_form(name, row)


@pytest.mark.parametrize("name", ["identity", "shift", "const"])
@pytest.mark.parametrize("layout", ["one", "quad", "lane12"])
def test_leaf_layouts_closed_form(name, layout):
    # Leaf hashing of n rows of 12 words: two permutations per row (a full
    # chunk of 8, then 4 words + zeros); compare with the closed form chained.
    L = load(name)
    knobs = {"one": (0, 0), "quad": (BIG, 0), "lane12": (BIG, BIG)}[layout]
    assert L.goldi_tune_set(b"quad_max_rows", knobs[0]) == 0
    assert L.goldi_tune_set(b"lane12_max_rows", knobs[1]) == 0
    n, w = 100, 12
    lv = goldilocks_words(41, 0, 0, n * w)
    out = to_dev(np.zeros(n * 4, dtype=np.uint64))
    assert L.goldi_leaf_hash(to_dev(lv).data_ptr(), n, w, out.data_ptr()) == 0
    got = to_host(out).reshape(n, 4)
    rows = lv.reshape(w, n).T
    for r in range(n):
        s = [int(v) for v in rows[r, :8]] + [0] * 4
        s = closed_form(name, s)
        s = [(a + int(b)) % P for a, b in zip(s[:4], rows[r, 8:])] + s[4:]
        s = closed_form(name, s)
        assert [int(v) for v in got[r]] == s[:4], (layout, r)


@pytest.mark.parametrize("name", ["identity", "shift", "const"])
def test_single_chunk_rows_and_nodes_closed_form(name):
    # Rows of at most 8 words (one absorption of a zero-capacity state, only
    # the digest kept) and the tree nodes above them, one lane per state:
    # the permutations with the shortened first round and the digest-only
    # last matrix, against the closed form.
    L = load(name)
    for k in (b"quad_max_rows", b"quad_max_parents", b"lane12_max_rows", b"lane12_max_parents",
              b"top_max_parents"):
        assert L.goldi_tune_set(k, 0) == 0
    L.goldi_merkle_build.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_size_t, ctypes.c_void_p]
    L.goldi_merkle_num_nodes.restype = ctypes.c_size_t
    L.goldi_merkle_num_nodes.argtypes = [ctypes.c_size_t]
    n, w = 37, 8
    lv = goldilocks_words(42, 0, 0, n * w)
    out = to_dev(np.zeros(L.goldi_merkle_num_nodes(n) * 4, dtype=np.uint64))
    assert L.goldi_merkle_build(to_dev(lv).data_ptr(), n, w, out.data_ptr()) == 0
    got = to_host(out).reshape(-1, 4)
    rows = lv.reshape(w, n).T
    level = [closed_form(name, [int(v) for v in rows[r]] + [0] * 4)[:4] for r in range(n)]
    want = list(level)
    while len(level) > 1:
        nxt = []
        for i in range(0, len(level), 2):
            if i + 1 < len(level):
                nxt.append(closed_form(name, level[i] + level[i + 1] + [0] * 4)[:4])
            else:
                nxt.append(level[i])
        want += nxt
        level = nxt
    assert [[int(v) for v in g] for g in got] == want
