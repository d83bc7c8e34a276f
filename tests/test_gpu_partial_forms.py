"""The default library evaluates the partial rounds of the one-state-per-lane
kernels in blocks of three; the sparse form (Sec. 2.4, Alg. 1) and the dense
form (the textbook matrix in every round) stay built as test libraries on the
seeded instance, and so does the full-round matrix on 24-bit multipliers
(22-bit limbs).  Each must give the oracle's results bit for bit:
permutations (random and edge states) and a ragged tree built with one lane
per state at every level."""

import ctypes
import os

import numpy as np
import pytest

import oracle
from synth.inputs import edge_states, leaves_colmajor, uniform_states

from .gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu


FORMS = ["sparse", "dense", "limb24"]


def load_form(form):
    import torch  # noqa: F401  (bind to torch's HIP runtime first)
    from paper_2506_09505_amd import build
    path = build.special_lib(form)
    assert os.path.exists(path), "build the libraries first"
    L = ctypes.CDLL(path)
    vp, sz = ctypes.c_void_p, ctypes.c_size_t
    L.goldi_poseidon_permute.argtypes = [vp, sz]
    L.goldi_merkle_build.argtypes = [vp, sz, sz, vp]
    L.goldi_merkle_num_nodes.restype = sz
    L.goldi_merkle_num_nodes.argtypes = [sz]
    L.goldi_tune_set.argtypes = [ctypes.c_char_p, sz]
    L.goldi_tune_get.argtypes = [ctypes.c_char_p, ctypes.POINTER(sz)]
    v = sz(99)
    assert L.goldi_tune_get(b"partial_form", ctypes.byref(v)) == 0
    assert v.value == {"sparse": 1, "dense": 0, "limb24": 2}[form]
    assert L.goldi_tune_get(b"mds_limb_bits", ctypes.byref(v)) == 0
    assert v.value == (22 if form == "limb24" else 32)
    return L


@pytest.fixture(scope="module")
def prm():
    return oracle.spec_params()


@pytest.mark.parametrize("form", FORMS)
def test_form_permute(prm, form):
    banner("%s form: permute 4096 random + edge states" % form)
    L = load_form(form)
    x = np.concatenate([uniform_states(4096, seed=50), edge_states()])
    d = to_dev(x)
    assert L.goldi_poseidon_permute(d.data_ptr(), x.shape[0]) == 0
    got = to_host(d).reshape(-1, 12)
    assert (got == oracle.permute(prm, x)).all()


@pytest.mark.parametrize("form", FORMS)
def test_form_tree(prm, form):
    banner("%s form: tree 3001 x 9, one lane per state" % form)
    L = load_form(form)
    for k in (b"quad_max_rows", b"quad_max_parents", b"lane12_max_rows", b"lane12_max_parents"):
        assert L.goldi_tune_set(k, 0) == 0
    n, w = 3001, 9
    lv = leaves_colmajor(n, w, seed=51)
    out = to_dev(np.zeros(L.goldi_merkle_num_nodes(n) * 4, dtype=np.uint64))
    assert L.goldi_merkle_build(to_dev(lv).data_ptr(), n, w, out.data_ptr()) == 0
    got = to_host(out).reshape(-1, 4)
    assert (got == oracle.merkle_build(prm, lv, n, w)).all()
