"""Pins of the oracle's field layer (Sec. 2.4 Eq. 1; the reduction identity
of Sec. 3.1 Eqs. 2-4; the canonical-output claims for unsigned Add/Sub of
Sec. 3.2).  The oracle computes with '%'; these tests check it against
Python big integers, closed-form identities and Fermat's little theorem."""

import random

import pytest

import oracle
from synth.inputs import EDGE_WORDS

P = oracle.P
EDGE = sorted(set(EDGE_WORDS + [P - 3, 5, 7, 1 << 63, (1 << 32) - 2]))
EDGE = [e for e in EDGE if e < P]


def test_prime_shape():
    # Eq. 1 and the factorisation that makes x -> x^7 a bijection.
    assert P == 2**64 - 2**32 + 1
    assert P - 1 == 2**32 * 3 * 5 * 17 * 257 * 65537
    import math
    assert math.gcd(7, P - 1) == 1


@pytest.mark.parametrize("a", EDGE)
def test_edge_pairs(a):
    for b in EDGE:
        assert oracle.fmul(a, b) == (a * b) % P
        assert oracle.fadd(a, b) == (a + b) % P
        assert oracle.fsub(a, b) == (a - b) % P


def test_random_pairs():
    rnd = random.Random(1234)
    for _ in range(20000):
        a, b = rnd.randrange(P), rnd.randrange(P)
        assert oracle.fmul(a, b) == (a * b) % P
        assert oracle.fadd(a, b) == (a + b) % P
        assert oracle.fsub(a, b) == (a - b) % P


def test_outputs_canonical():
    # Sec. 3.2: add and sub of canonical inputs give canonical outputs.
    for a in EDGE:
        for b in EDGE:
            assert oracle.fadd(a, b) < P and oracle.fsub(a, b) < P and oracle.fmul(a, b) < P


def test_reduce128_any_input():
    # Eqs. 2-4: r = r_h 2^64 + r_l is congruent to r_hl (2^32 - 1) + r_l - r_hh.
    rnd = random.Random(99)
    vals = [(0, 0), (0, P), (0, 2**64 - 1), (2**64 - 1, 2**64 - 1), (P - 1, P - 1), (2**32, 0)]
    vals += [(rnd.randrange(2**64), rnd.randrange(2**64)) for _ in range(20000)]
    for hi, lo in vals:
        r = (hi << 64) | lo
        got = oracle.reduce128(hi, lo)
        assert got == r % P
        r_hh, r_hl = hi >> 32, hi & 0xFFFFFFFF
        assert got == (r_hl * (2**32 - 1) + lo - r_hh) % P


def test_identities():
    two32 = 1 << 32
    t64 = oracle.fmul(two32, two32)
    assert t64 == two32 - 1                          # 2^64 = 2^32 - 1   (Eq. 3)
    t96 = oracle.fmul(t64, two32)
    assert t96 == P - 1                               # 2^96 = -1
    t128 = oracle.fmul(t96, two32)
    assert t128 == oracle.fsub(0, two32)              # 2^128 = -2^32
    assert oracle.fmul(t96, t96) == 1                 # 2^192 = 1
    assert oracle.fadd(P - 1, 1) == 0
    assert oracle.fmul(P - 1, P - 1) == 1
    # Eq. 4 bound: (2^32-1)^2 + 2^64 - 1 = 2p - 2
    assert (2**32 - 1) ** 2 + 2**64 - 1 == 2 * P - 2


def test_fermat_inverse_and_sbox_bijection():
    rnd = random.Random(7)
    d = pow(7, -1, P - 1)
    for _ in range(300):
        a = rnd.randrange(1, P)
        assert oracle.fmul(a, oracle.fpow(a, P - 2)) == 1
        assert oracle.fpow(oracle.fpow(a, 7), d) == a
    assert oracle.fpow(0, 7) == 0 and oracle.fpow(1, 7) == 1 and oracle.fpow(P - 1, 7) == P - 1


def test_field_array_matches_scalar_definitions():
    import numpy as np
    rnd = random.Random(3)
    a = np.array([rnd.randrange(P) for _ in range(500)] + EDGE, dtype=np.uint64)
    b = np.array([rnd.randrange(P) for _ in range(500)] + EDGE[::-1], dtype=np.uint64)
    ai, bi = [int(v) for v in a], [int(v) for v in b]
    assert [int(v) for v in oracle.field_array("add", a, b)] == [(x + y) % P for x, y in zip(ai, bi)]
    assert [int(v) for v in oracle.field_array("sub", a, b)] == [(x - y) % P for x, y in zip(ai, bi)]
    assert [int(v) for v in oracle.field_array("reduce_128_64", a, b)] == [((x << 64) | y) % P for x, y in zip(ai, bi)]
    assert [int(v) for v in oracle.field_array("square_128", a)] == [x * x % P for x in ai]
    assert [int(v) for v in oracle.field_array("mult_128", a, b)] == [x * y % P for x, y in zip(ai, bi)]
    assert [int(v) for v in oracle.field_array("mult_72", a, b)] == [x * (y & 255) % P for x, y in zip(ai, bi)]
    assert [int(v) for v in oracle.field_array("sbox", a)] == [pow(x, 7, P) for x in ai]
