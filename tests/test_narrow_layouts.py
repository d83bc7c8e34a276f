"""CPU replays of how the two narrow layouts split one permutation over lanes,
in exact integers mod p, checked against the oracle's textbook permutation
(Sec. 2.4, Alg. 1).  Each replay keeps the layout's data movement:

* one word per lane (poseidon_lane12.hpp): lane i of a 16-lane row holds
  word i; a round's product takes every word of the row by broadcast and
  the lane's own coefficient row; partial rounds go three at a time, with
  the block's chained S-box inputs computed by the helper lanes 12 and 13
  (row 0 of A_1 and of A_2) and each S-box output broadcast from the lane
  that made it; the first partial round rides on the last opening round
  (lanes 0..11 take M P M, lane 12 row 0 of M);
* four lanes per state (poseidon_quad.hpp): lane q holds words 3q..3q+2;
  a block's rows 3q..3q+2 of A_3 read the quad's words as fetched at quad
  distance D, and the chain rows are summed over the quad from each lane's
  share over its own three words.

The coefficient tables are built here from gen_constants.block_form the
way the kernels' tables are laid out; a lane that takes the wrong row,
constant or broadcast source fails the comparison."""

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
ROUNDS = 30


def sbox(x):
    return pow(x, 7, P)


def lane12_tables(mds, rc, bf):
    """Per-lane rows and constants of a 16-lane row (lanes 14, 15 copy a
    helper lane and are never read)."""
    k = bf["k"]
    t = {"m": [], "lead": [], "f_lead": [], "k_lead": [], "blk": [], "f": [], "k_blk": []}
    for lane in range(16):
        i = lane if lane < W else 0
        t["m"].append(list(mds[i]))
        t["lead"].append(list(bf["lead_b"][lane]) if lane < W else list(mds[0]))
        t["f_lead"].append(mds[lane][0] if lane < W else 0)
        t["k_lead"].append(bf["lead_k"][lane] if lane < W else rc[HALF_FULL][0])
        m = k if lane < W else (lane - W + 1 if lane - W + 1 < k else 1)
        row = lane if lane < W else 0
        t["blk"].append(list(bf["a"][m][row]))
        t["f"].append(list(bf["f"][m][row]) + [0] * (k - m))
        kidx = k - 1 + lane if lane < W else m - 1
        t["k_blk"].append([bf["kc"][b][kidx] for b in range(len(bf["starts"]))])
    return t


def lane12_permute(state, rc, mds, bf, t, lead_src=W, chain0=W):
    """One state over a 16-lane row; lead_src / chain0 are the lanes whose
    S-box output is broadcast for the lead and the first chained S-box."""
    k = bf["k"]
    x = [(state[i] + rc[0][i]) % P for i in range(W)] + [0] * 4
    bcast = lambda v, j: v[j]

    def row(c, words, const, lanes=range(16)):
        return [(sum(c[l][j] * words[j] for j in range(W)) + const[l]) % P for l in lanes]

    for r in range(HALF_FULL - 1):
        s = [sbox(v) for v in x]
        x = row(t["m"], s[:W], [rc[r + 1][l if l < W else 0] for l in range(16)])
    s = [sbox(v) for v in x]
    a = row(t["lead"], s[:W], t["k_lead"])
    su = sbox(bcast(a, lead_src))
    x = [(a[l] + t["f_lead"][l] * su) % P for l in range(16)]
    for b in range(len(bf["starts"])):
        a = [(sum(t["blk"][l][j] * x[j] for j in range(1, W)) + t["k_blk"][l][b]) % P for l in range(16)]
        sb = sbox(bcast(x, 0))
        a = [(a[l] + t["f"][l][0] * sb) % P for l in range(16)]
        for m in range(1, k):
            sb = sbox(bcast(a, chain0 + m - 1))
            a = [(a[l] + t["f"][l][m] * sb) % P for l in range(16)]
        x = a
    assert not bf["tail"]
    for r in range(HALF_FULL + 22, ROUNDS):
        s = [sbox(v) for v in x]
        x = row(t["m"], s[:W], [(rc[r + 1][l if l < W else 0] if r + 1 < ROUNDS else 0) for l in range(16)])
    return x[:W]


def quad_tables(bf):
    k = bf["k"]
    t = {"a": [], "c": [], "f": [], "k": []}
    for q in range(4):
        t["a"].append([[bf["a"][k][3 * q + r][3 * ((q + d) % 4) + kk] for d in range(4) for kk in range(3)]
                       for r in range(3)])
        t["c"].append([[bf["a"][m][0][3 * q + kk] for kk in range(3)] for m in range(1, k)])
        t["f"].append([list(bf["f"][k][3 * q + r]) for r in range(3)])
        t["k"].append([[bf["kc"][b][k - 1 + 3 * q + r] for r in range(3)]
                       + [bf["kc"][b][m - 1] if q == 0 else 0 for m in range(1, k)]
                       for b in range(len(bf["starts"]))])
    return t


def quad_block(w, bf, t, b):
    """One block over the quad: w[q] = words 3q..3q+2 of lane q."""
    k = bf["k"]
    x = [[w[(q + d) % 4] for d in range(4)] for q in range(4)]       # x[q][D] = lane q+D's words
    s = [sbox(w[0][0])]                                              # lane 0's word 0
    share = [[(sum(t["c"][q][m][kk] * w[q][kk] for kk in range(3)) + t["k"][q][b][3 + m]) % P
              for m in range(k - 1)] for q in range(4)]
    chain = [sum(share[q][m] for q in range(4)) % P for m in range(k - 1)]   # the two DPP steps
    for m in range(1, k):
        u = (chain[m - 1] + sum(bf["f"][m][0][j] * s[j] for j in range(m))) % P
        s.append(sbox(u))
    out = []
    for q in range(4):
        lane = []
        for r in range(3):
            acc = t["k"][q][b][r]
            acc += sum(t["a"][q][r][3 * d + kk] * x[q][d][kk] for d in range(4) for kk in range(3))
            acc += sum(t["f"][q][r][m] * s[m] for m in range(k))
            lane.append(acc % P)
        out.append(lane)
    return out


def quad_permute(state, rc, mds, bf, t):
    x = [(state[i] + rc[0][i]) % P for i in range(W)]
    for r in range(HALF_FULL):
        y = [sbox(v) for v in x]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + rc[r + 1][i]) % P for i in range(W)]
    y = [sbox(x[0])] + x[1:]                                         # the first partial round alone
    x = [(sum(mds[i][j] * y[j] for j in range(W)) + rc[HALF_FULL + 1][i]) % P for i in range(W)]
    w = [x[3 * q:3 * q + 3] for q in range(4)]
    for b in range(len(bf["starts"])):
        w = quad_block(w, bf, t, b)
    x = [v for lane in w for v in lane]
    for r in range(HALF_FULL + 22, ROUNDS):
        y = [sbox(v) for v in x]
        x = [(sum(mds[i][j] * y[j] for j in range(W)) + (rc[r + 1][i] if r + 1 < ROUNDS else 0)) % P
             for i in range(W)]
    return x


def _states(n, seed):
    s = uniform_states(n, seed=seed).astype(object).tolist()
    edge = [int(e) for e in EDGE_WORDS]
    s.append([edge[(3 * i + 1) % len(edge)] for i in range(W)])
    return [[int(v) for v in st] for st in s]


@pytest.fixture(scope="module")
def inst():
    rc, mds = load_constants()
    bf = gc.block_form(rc, mds)
    states = _states(6, seed=70)
    want = oracle.permute(oracle.Params(rc, mds), np.array(states, dtype=np.uint64))
    return rc, mds, bf, states, [[int(v) for v in w] for w in want]


def test_lane12_layout_equals_textbook(inst):
    rc, mds, bf, states, want = inst
    t = lane12_tables(mds, rc, bf)
    for st, w in zip(states, want):
        assert lane12_permute(st, rc, mds, bf, t) == w


def test_quad_layout_equals_textbook(inst):
    rc, mds, bf, states, want = inst
    t = quad_tables(bf)
    for st, w in zip(states, want):
        assert quad_permute(st, rc, mds, bf, t) == w


LANE12_MISTAKES = [
    ("chain_from_lane_13", dict(chain0=W + 1)),
    ("lead_from_lane_0", dict(lead_src=0)),
]


@pytest.mark.parametrize("name,kw", LANE12_MISTAKES, ids=[m[0] for m in LANE12_MISTAKES])
def test_lane12_wrong_broadcast_source_is_caught(inst, name, kw):
    rc, mds, bf, states, want = inst
    t = lane12_tables(mds, rc, bf)
    assert lane12_permute(states[0], rc, mds, bf, t, **kw) != want[0]


def test_lane12_swapped_helper_rows_are_caught(inst):
    rc, mds, bf, states, want = inst
    t = lane12_tables(mds, rc, bf)
    t["blk"][W], t["blk"][W + 1] = t["blk"][W + 1], t["blk"][W]
    assert lane12_permute(states[0], rc, mds, bf, t) != want[0]


def test_quad_unrotated_coefficients_are_caught(inst):
    # Lane q's entries must follow its own quad rotation: lane 0's table in
    # every lane gives a different permutation.
    rc, mds, bf, states, want = inst
    t = quad_tables(bf)
    bad = copy.deepcopy(t)
    for q in range(1, 4):
        bad["a"][q] = t["a"][0]
    assert quad_permute(states[0], rc, mds, bf, bad) != want[0]


def test_quad_chain_constant_only_in_lane_0(inst):
    rc, mds, bf, states, want = inst
    bad = quad_tables(bf)
    for b in range(len(bf["starts"])):
        bad["k"][1][b][3] = bad["k"][0][b][3]                        # added twice over the quad
    assert quad_permute(states[0], rc, mds, bf, bad) != want[0]
