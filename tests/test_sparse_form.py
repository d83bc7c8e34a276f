"""The partial rounds in sparse form (Sec. 2.4, Alg. 1: a pre-matrix once,
then per round a matrix whose first row and column are full and whose rest is
the identity, with scalar round constants) must be the textbook permutation.

``gen_constants.sparse_form`` derives those constants from C and M; here they
are evaluated in the sparse shape, in Python integers, and compared with the
oracle's dense textbook permutation on random and edge states, for the seeded
instance and for the special test instances.  A wrong power of the 11 x 11
block, a transposed row or column, a misplaced scalar constant or a lost
carry changes the permutation and fails."""

import numpy as np
import pytest

import oracle
from paper_2506_09505_amd import gen_constants as gc
from synth.constants import load_constants
from synth.inputs import EDGE_WORDS, uniform_states

P = gc.P
W = 12


def sbox(x):
    return pow(x, 7, P)


def sparse_permute(x, rc, mds, sp):
    """Sparse-form evaluation: rounds 0..2 dense; round 3 with the pre-matrix
    folded into its matrix; 22 sparse partial rounds; rounds 26..29 dense."""
    x = [(x[i] + rc[0][i]) % P for i in range(W)]
    for r in range(3):
        y = [sbox(t) for t in x]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + rc[r + 1][i]) % P for i in range(W)]
    y = [sbox(t) for t in x]
    x = [(sum(mds[0][j] * y[j] for j in range(W)) + sp["k"][0]) % P]
    x += [sum(sp["pre_m"][i][j] * y[j] for j in range(W)) % P for i in range(W - 1)]
    for j in range(22):
        s = sbox(x[0])
        nxt = sp["k"][j + 1] if j < 21 else sp["c_end"][0]
        x0 = (mds[0][0] * s + sum(sp["row"][j][i] * x[i + 1] for i in range(W - 1)) + nxt) % P
        rest = [(x[i + 1] + sp["col"][j][i] * s) % P for i in range(W - 1)]
        x = [x0] + rest
    x = [x[0]] + [(x[i] + sp["c_end"][i]) % P for i in range(1, W)]
    for r in range(26, 30):
        y = [sbox(t) for t in x]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + (rc[r + 1][i] if r < 29 else 0)) % P for i in range(W)]
    return x


def grouped_permute(x, rc, mds, sp, groups):
    """The same with the partial rounds in groups (sizes `groups`, summing to
    22), as the kernels take them: round g of a group reads the words from the
    start of the group plus lag terms times the group's earlier S-box
    outputs; each word then takes all of the group's column terms at once."""
    x = [(x[i] + rc[0][i]) % P for i in range(W)]
    for r in range(3):
        y = [sbox(t) for t in x]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + rc[r + 1][i]) % P for i in range(W)]
    y = [sbox(t) for t in x]
    x = [(sum(mds[0][j] * y[j] for j in range(W)) + sp["k"][0]) % P]
    x += [sum(sp["pre_m"][i][j] * y[j] for j in range(W)) % P for i in range(W - 1)]
    j = 0
    for gsize in groups:
        outs = [sbox(x[0])]
        for g in range(gsize):
            r = j + g
            nxt = sp["k"][r + 1] if r + 1 < 22 else sp["c_end"][0]
            d0 = (mds[0][0] * outs[g] + sum(sp["row"][r][i] * x[i + 1] for i in range(W - 1))
                  + sum(sp["lag"][r][g - 1 - h] * outs[h] for h in range(g)) + nxt) % P
            if g + 1 < gsize:
                outs.append(sbox(d0))
        x = [d0] + [(x[i + 1] + sum(sp["col"][j + g][i] * outs[g] for g in range(gsize))) % P for i in range(W - 1)]
        j += gsize
    assert j == 22
    x = [x[0]] + [(x[i] + sp["c_end"][i]) % P for i in range(1, W)]
    for r in range(26, 30):
        y = [sbox(t) for t in x]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + (rc[r + 1][i] if r < 29 else 0)) % P for i in range(W)]
    return x


GROUPINGS = [[1] * 22, [2] * 11, [4] * 5 + [2], [3] * 6 + [4]]


def _states(n, seed):
    s = uniform_states(n, seed=seed).astype(object).tolist()
    edge = [int(e) for e in EDGE_WORDS]
    s.append([edge[i % len(edge)] for i in range(W)])
    s.append([edge[(3 * i + 1) % len(edge)] for i in range(W)])
    return s


def test_sparse_form_equals_textbook_seeded():
    rc, mds = load_constants()
    sp = gc.sparse_form(rc, mds)
    assert sp is not None
    states = _states(12, seed=40)
    want = oracle.permute(oracle.Params(rc, mds), np.array(states, dtype=np.uint64))
    for st, w in zip(states, want):
        assert sparse_permute([int(v) for v in st], rc, mds, sp) == [int(v) for v in w]
        for groups in GROUPINGS:
            assert grouped_permute([int(v) for v in st], rc, mds, sp, groups) == [int(v) for v in w]


@pytest.mark.parametrize("name", ["identity", "const"])
def test_sparse_form_equals_textbook_special(name):
    spec = gc.special_specs()[name]
    rc = [[int(v) for v in row] for row in spec["rc"]]
    mds = spec["mds"]
    sp = gc.sparse_form(rc, mds)
    states = _states(4, seed=41)
    want = oracle.permute(oracle.Params(rc, mds), np.array(states, dtype=np.uint64))
    for st, w in zip(states, want):
        assert sparse_permute([int(v) for v in st], rc, mds, sp) == [int(v) for v in w]
        for groups in GROUPINGS:
            assert grouped_permute([int(v) for v in st], rc, mds, sp, groups) == [int(v) for v in w]


@pytest.mark.parametrize("d", [0, 1, 2])
def test_lag_mistake_is_caught(d):
    # A wrong lag scalar changes the grouped permutation.
    rc, mds = load_constants()
    sp = gc.sparse_form(rc, mds)
    st = [int(v) for v in _states(1, seed=42)[0]]
    groups = [4] * 5 + [2]
    good = grouped_permute(st, rc, mds, sp, groups)
    sp["lag"] = [list(r) for r in sp["lag"]]
    sp["lag"][7][d] = (sp["lag"][7][d] + 1) % P  # round 7 is the fourth of its group
    assert grouped_permute(st, rc, mds, sp, groups) != good


def test_sparse_form_absent_when_block_singular():
    spec = gc.special_specs()["shift"]
    assert gc.sparse_form([[int(v) for v in row] for row in spec["rc"]], spec["mds"]) is None


def test_limb_split_roundtrip():
    for x in [0, 1, P - 1, 2**63, 0x123456789ABCDEF0 % P]:
        l = gc._limbs22(x)
        assert all(v < 2**22 for v in l) and l[0] + (l[1] << 22) + (l[2] << 44) == x


def test_zero_capacity_round0_constants():
    # Round 0 of a state whose words 8..11 are zero, as the kernels take it
    # (S-boxes of words 0..7 only, the matrix over those words, CAP0_RC1 as
    # the row constants), equals the textbook round 0 followed by C[1].
    rc, mds = load_constants()
    r1 = gc.cap0_constants(rc, mds)
    for st in _states(6, seed=43):
        x = [int(v) for v in st[:8]] + [0] * 4
        y = [sbox((x[i] + rc[0][i]) % P) for i in range(W)]
        want = [(sum(mds[i][j] * y[j] for j in range(W)) + rc[1][i]) % P for i in range(W)]
        got = [(sum(mds[i][j] * y[j] for j in range(8)) + r1[i]) % P for i in range(W)]
        assert got == want
