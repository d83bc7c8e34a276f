"""The partial rounds taken three at a time must be the textbook permutation.

A partial round maps a state b that holds its round constant to
M P b + c0 S(b_0) + C[r+1] (P zeroes word 0, c0 is column 0 of M), so m
rounds map b to (M P)^m b + sum_j f_m[j] S_j + K_m; the first partial round
rides on the last opening round's matrix as (M P M) y + c0 S(u) + ...
(Sec. 2.4 for the round structure).  ``gen_constants.block_form`` derives
those integers and constants; here they are evaluated in that shape, in
Python integers, and compared with the oracle's dense textbook permutation,
for the seeded instance and the special test instances.  A wrong power, a
coefficient of the wrong S-box output, a misplaced block constant or a lost
lead term changes the permutation and fails.  The 64-bit accumulator bound
the kernels rely on is checked on the worst-case inputs."""

import copy

import numpy as np
import pytest

import oracle
from paper_2506_09505_amd import gen_constants as gc
from synth.constants import load_constants
from synth.inputs import EDGE_WORDS, uniform_states

P = gc.P
W = 12
HALF_FULL = 4


def sbox(x):
    return pow(x, 7, P)


def block_permute(x, rc, mds, bf):
    """Opening rounds 0..2 dense; round 3's matrix with partial round 4 on it;
    partial rounds 5..25 in blocks; closing rounds 26..29 dense."""
    x = [(x[i] + rc[0][i]) % P for i in range(W)]
    for r in range(HALF_FULL - 1):
        y = [sbox(t) for t in x]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + rc[r + 1][i]) % P for i in range(W)]
    y = [sbox(t) for t in x]
    u = (sum(mds[0][j] * y[j] for j in range(W)) + rc[HALF_FULL][0]) % P
    s0 = sbox(u)
    x = [(sum(bf["lead_b"][i][j] * y[j] for j in range(W)) + mds[i][0] * s0 + bf["lead_k"][i]) % P
         for i in range(W)]
    k = bf["k"]
    for b, _ in enumerate(bf["starts"]):
        kc = bf["kc"][b]
        s = [sbox(x[0])]
        for m in range(1, k):
            u = (sum(bf["a"][m][0][j] * x[j] for j in range(1, W))
                 + sum(bf["f"][m][0][j] * s[j] for j in range(m)) + kc[m - 1]) % P
            s.append(sbox(u))
        x = [(sum(bf["a"][k][i][j] * x[j] for j in range(1, W))
              + sum(bf["f"][k][i][j] * s[j] for j in range(k)) + kc[k - 1 + i]) % P for i in range(W)]
    for r in bf["tail"]:
        y = [sbox(x[0])] + x[1:]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + rc[r + 1][i]) % P for i in range(W)]
    for r in range(26, 30):
        y = [sbox(t) for t in x]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + (rc[r + 1][i] if r < 29 else 0)) % P for i in range(W)]
    return x


def _states(n, seed):
    s = uniform_states(n, seed=seed).astype(object).tolist()
    edge = [int(e) for e in EDGE_WORDS]
    s.append([edge[i % len(edge)] for i in range(W)])
    s.append([edge[(5 * i + 2) % len(edge)] for i in range(W)])
    return s


def _check(rc, mds, bf, states):
    want = oracle.permute(oracle.Params(rc, mds), np.array(states, dtype=np.uint64))
    return all(block_permute([int(v) for v in st], rc, mds, bf) == [int(v) for v in w]
               for st, w in zip(states, want))


def test_block_form_equals_textbook_seeded():
    rc, mds = load_constants()
    bf = gc.block_form(rc, mds)
    assert bf is not None and bf["k"] == 3
    assert bf["starts"] == [5, 8, 11, 14, 17, 20, 23] and bf["tail"] == []
    assert _check(rc, mds, bf, _states(12, seed=60))


@pytest.mark.parametrize("name", ["identity", "shift", "const"])
def test_block_form_equals_textbook_special(name):
    spec = gc.special_specs()[name]
    rc = [[int(v) for v in row] for row in spec["rc"]]
    mds = spec["mds"]
    bf = gc.block_form(rc, mds)
    assert bf is not None
    assert _check(rc, mds, bf, _states(4, seed=61))


@pytest.mark.parametrize("k", [1, 2])
def test_other_block_sizes_equal_textbook(k):
    # Blocks of one and two rounds (with a tail for 21 = 10 * 2 + 1) reach
    # the same permutation: the derivation does not depend on k.
    rc, mds = load_constants()
    bf = gc.block_form(rc, mds, k=k)
    assert bf is not None
    assert _check(rc, mds, bf, _states(3, seed=62))


MISTAKES = [
    ("a", lambda bf: bf["a"][3][4].__setitem__(7, bf["a"][3][4][7] + 1)),
    ("a_row0", lambda bf: bf["a"][2][0].__setitem__(1, bf["a"][2][0][1] + 1)),
    ("f_old", lambda bf: bf["f"][3][2].__setitem__(0, bf["f"][3][2][0] + 1)),
    ("f_mid", lambda bf: bf["f"][2][0].__setitem__(0, bf["f"][2][0][0] + 1)),
    ("f_swap", lambda bf: bf["f"][3].__setitem__(5, bf["f"][3][5][::-1])),
    ("kc_word0", lambda bf: bf["kc"][3].__setitem__(0, (bf["kc"][3][0] + 1) % P)),
    ("kc_row", lambda bf: bf["kc"][6].__setitem__(13, (bf["kc"][6][13] + 1) % P)),
    ("lead_b", lambda bf: bf["lead_b"][9].__setitem__(0, bf["lead_b"][9][0] + 1)),
    ("lead_k", lambda bf: bf["lead_k"].__setitem__(2, (bf["lead_k"][2] + 1) % P)),
    ("a_power", lambda bf: bf["a"].__setitem__(3, bf["a"][2])),
]


@pytest.mark.parametrize("name,plant", MISTAKES, ids=[m[0] for m in MISTAKES])
def test_planted_mistakes_are_caught(name, plant):
    rc, mds = load_constants()
    bf = copy.deepcopy(gc.block_form(rc, mds))
    plant(bf)
    assert not _check(rc, mds, bf, _states(1, seed=63)[:1])


def test_accumulators_fit_64_bits():
    # Each row of a block (and of the lead round) adds products of 32-bit
    # limbs (< 2^32) by its coefficients, plus a 32-bit half of its constant,
    # in one 64-bit accumulator; the kernels' split reduction needs the sum
    # below 2^63.
    rc, mds = load_constants()
    bf = gc.block_form(rc, mds)
    lim = (1 << 32) - 1
    rows = [bf["a"][m][i][1:] + bf["f"][m][i] for m in range(1, 4) for i in range(W)]
    rows += [bf["lead_b"][i] + [mds[i][0]] for i in range(W)]
    for r in rows:
        assert max(r) < 1 << 32
        assert sum(r) * lim + lim < 1 << 63
    # Four rounds per block would not fit: the generator refuses them.
    assert gc.block_form(rc, mds, k=4) is None


def test_block_matrices_are_powers():
    # A_m = (M P)^m with the column of word 0 zero; f_m[j] = A_(m-1-j) c0.
    rc, mds = load_constants()
    bf = gc.block_form(rc, mds)
    mp = np.array([[0 if j == 0 else mds[i][j] for j in range(W)] for i in range(W)], dtype=object)
    c0 = np.array([mds[i][0] for i in range(W)], dtype=object)
    power = np.identity(W, dtype=object)
    for m in range(1, 4):
        power = mp.dot(power)
        assert (np.array(bf["a"][m], dtype=object) == power).all()
        assert all(v == 0 for v in power[:, 0])
    a1 = np.array(bf["a"][1], dtype=object)
    assert [row[2] for row in bf["f"][3]] == list(c0)
    assert [row[1] for row in bf["f"][3]] == list(a1.dot(c0))
    assert (np.array(bf["lead_b"], dtype=object) == mp.dot(np.array(mds, dtype=object))).all()
