"""GPU: every device field operation of the HIP path (the paper's Table-1
functions on 32-bit limbs) against the oracle, on edge-class pairs and
random pairs; the two 12x12 mat-vecs against the plain definition."""

import itertools

import numpy as np
import pytest

import oracle
from synth.inputs import EDGE_WORDS, GOLDILOCKS_P, goldilocks_words

from .gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu
P = GOLDILOCKS_P
EDGE = sorted(set([e for e in EDGE_WORDS if e < P] + [P - 3, 5, 7, 1 << 63, (1 << 32) - 2, 1 << 32]))


def pairs():
    e = np.array(list(itertools.product(EDGE, EDGE)), dtype=np.uint64)
    n = 1 << 20
    a = np.concatenate([e[:, 0], goldilocks_words(31, 0, 0, n)])
    b = np.concatenate([e[:, 1], goldilocks_words(31, 1, 0, n)])
    return a, b


@pytest.mark.parametrize("name", ["add", "sub", "reduce_128_64", "square_128", "mult_128", "mult_72", "sbox"])
def test_word_ops(name):
    from paper_2506_09505_amd import fieldbench
    a, b = pairs()
    if name == "reduce_128_64":
        # any 128-bit value: also words >= p in both halves
        a = np.concatenate([a, np.array([2**64 - 1, 2**64 - 1, P, 0], dtype=np.uint64)])
        b = np.concatenate([b, np.array([2**64 - 1, 0, 2**64 - 1, P], dtype=np.uint64)])
    got = to_host(fieldbench.evaluate(name, to_dev(a), to_dev(b)))
    want = oracle.field_array(name, a, b)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, "%s: first mismatch at %s: a=%d b=%d got=%d want=%d" % (
        name, bad[:3], int(a[bad[0]]), int(b[bad[0]]), int(got[bad[0]]), int(want[bad[0]]))


@pytest.mark.parametrize("name", ["mmult_12x12_small", "mmult_12x12_full"])
def test_matvecs(name):
    from paper_2506_09505_amd import fieldbench
    prm = oracle.spec_params()
    n = 64
    s = goldilocks_words(32, 0, 0, n * 12).reshape(n, 12)
    s[:4] = np.array([[0] * 12, [P - 1] * 12, list(range(12)), [(1 << 32) - 1] * 12], dtype=np.uint64)
    got = to_host(fieldbench.evaluate(name, to_dev(s))).reshape(n, 12)
    if name == "mmult_12x12_small":
        mat = prm.mds
    else:
        c0 = prm.rc[0]
        mat = [[c0[(i + j) % 12] for j in range(12)] for i in range(12)]
    for row_s, row_g in zip(s, got):
        x = [int(v) for v in row_s]
        assert [int(v) for v in row_g] == [sum(mat[i][j] * x[j] for j in range(12)) % P for i in range(12)]
