"""Pins of the oracle's Poseidon-12 permutation (Sec. 2.4, Alg. 1).

The paper prints no constants or test vectors, so the permutation's values
cannot be pinned to it ("parity unpinned").  Its *structure* is pinned by
special instances whose output has a closed form computed with Python's
``pow``:

* M = I, C = 0: word 0 goes through all 30 S-boxes, words 1..11 through the
  8 full rounds only -> round counts 4 + 22 + 4 and the partial S-box on word 0;
* M = a 7-cycle permutation matrix, C = 0: words travel through positions;
  pins M * state (not state * M), S-box before M, and which rounds are full;
* M = all-ones: every word of every row counts; pins the dense sum;
* M = I, one nonzero constant C[r0][k]: pins that C[r] enters round r before
  its S-box;
* the inverse permutation (mini-oracle) undoes the oracle's forward one;
* a second, big-integer implementation agrees on random states.
"""

import random

import numpy as np
import pytest

import oracle
from oracle import mini
from synth.inputs import edge_states, uniform_states

P = oracle.P
FULL = [r < 4 or r >= 26 for r in range(30)]


def ident():
    return [[int(i == j) for j in range(12)] for i in range(12)]


def zero_rc():
    return [[0] * 12 for _ in range(30)]


def rand_states(n, seed):
    return uniform_states(n, seed)


def test_identity_matrix_round_counts():
    prm = oracle.Params(zero_rc(), ident())
    x = rand_states(64, 11)
    out = oracle.permute(prm, x)
    e0, ei = pow(7, 30, P - 1), pow(7, 8, P - 1)
    for s, o in zip(x, out):
        assert int(o[0]) == pow(int(s[0]), e0, P)
        for i in range(1, 12):
            assert int(o[i]) == pow(int(s[i]), ei, P)


def test_permutation_matrix_orientation():
    # pi is a 7-cycle on positions 0..6; M[i][j] = 1 iff j = pi(i), i.e. new_i = s_{pi(i)}.
    pi = {i: (i + 1) % 7 for i in range(7)}
    pi.update({i: i for i in range(7, 12)})
    m = [[int(j == pi[i]) for j in range(12)] for i in range(12)]
    prm = oracle.Params(zero_rc(), m)
    x = rand_states(32, 12)
    out = oracle.permute(prm, x)
    # Track each input word: its position and its exponent.
    pos = list(range(12))          # pos[k] = current position of input word k
    exp = [1] * 12
    for r in range(30):
        for k in range(12):
            if FULL[r] or pos[k] == 0:
                exp[k] *= 7
        inv = {pi[i]: i for i in range(12)}   # word at position j moves to position inv[j]
        pos = [inv[p_] for p_ in pos]
    for s, o in zip(x, out):
        for k in range(12):
            assert int(o[pos[k]]) == pow(int(s[k]), exp[k], P)
    # The transposed reading (new_i = s_{pi^-1(i)}) would put words elsewhere.
    assert pos != list(range(12))


def test_all_ones_matrix_dense_sum():
    ones = [[1] * 12 for _ in range(12)]
    prm = oracle.Params(zero_rc(), ones)
    x = rand_states(16, 13)
    out = oracle.permute(prm, x)
    for s, o in zip(x, out):
        v = sum(pow(int(t), 7, P) for t in s) % P       # after round 0 all words equal v
        for r in range(1, 30):
            v = (12 * pow(v, 7, P)) % P if FULL[r] else (pow(v, 7, P) + 11 * v) % P
        assert all(int(t) == v for t in o)


@pytest.mark.parametrize("r0,k", [(0, 0), (0, 5), (3, 11), (4, 0), (4, 3), (15, 0), (25, 7),
                                  (26, 0), (26, 9), (29, 0), (29, 11)])
def test_single_round_constant_placement(r0, k):
    rc = zero_rc()
    c = 0x123456789ABCDEF % P
    rc[r0][k] = c
    prm = oracle.Params(rc, ident())
    out = oracle.permute(prm, np.zeros((1, 12), dtype=np.uint64))[0]
    # From round r0 on, word k is S-boxed in every full round, and word 0 also
    # in every partial round.
    n_sbox = sum(1 for r in range(r0, 30) if FULL[r] or k == 0)
    want = [0] * 12
    want[k] = pow(c, 7 ** n_sbox, P)
    assert [int(v) for v in out] == want


def test_inverse_round_trip_spec_constants():
    prm = oracle.spec_params()
    x = np.concatenate([rand_states(6, 14), edge_states()[:4]])
    out = oracle.permute(prm, x)
    for s, o in zip(x, out):
        back = mini.inverse_permute([int(v) for v in o], prm.rc, prm.mds)
        assert back == [int(v) for v in s]


def test_bigint_implementation_agrees():
    prm = oracle.spec_params()
    x = np.concatenate([rand_states(24, 15), edge_states()])
    out = oracle.permute(prm, x)
    for s, o in zip(x, out):
        assert mini.permute([int(v) for v in s], prm.rc, prm.mds) == [int(v) for v in o]


def test_threads_do_not_change_results():
    prm = oracle.spec_params()
    x = rand_states(257, 16)
    assert (oracle.permute(prm, x, threads=1) == oracle.permute(prm, x, threads=7)).all()


def test_outputs_canonical_and_nonlinear():
    prm = oracle.spec_params()
    x = rand_states(64, 17)
    out = oracle.permute(prm, x)
    assert (out < np.uint64(P)).all()
    # a single flipped input bit changes every output word
    y = x.copy()
    y[:, 3] ^= np.uint64(1)
    y[:, 3] %= np.uint64(P)
    out2 = oracle.permute(prm, y)
    assert (out2 != out).all()
