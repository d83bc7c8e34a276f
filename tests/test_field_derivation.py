"""CPU checks of the device field layer's instruction sequences (field.hpp),
replayed step by step with exact integers: every intermediate must fit the
register it lives in, and the result must be congruent to the product mod p
(Sec. 3.1, Eqs. 2-3: 2^64 = 2^32 - 1 mod p).  The inputs are any 64-bit
words (the permutation keeps values weakly reduced), edge words and random
words."""

import random

P = 2**64 - 2**32 + 1
M32, M64 = 2**32 - 1, 2**64 - 1
EPS = 2**32 - 1


def mad(a, b, c):
    """v_mad_u64_u32: 32 x 32 + 64 -> 64 bits, carry-out."""
    assert 0 <= a <= M32 and 0 <= b <= M32 and 0 <= c <= M64
    r = a * b + c
    return r & M64, r >> 64


def mad_eps_fold(h, x):
    # r, c = h (2^32 - 1) + x; t = c; r = t (2^32 - 1) + r (no carry)
    r, c = mad(h, EPS, x)
    r2, c2 = mad(c, EPS, r)
    assert c2 == 0
    return r2


def mul_fold(a, b):
    """The product with the middle carry folded into the reduction."""
    a0, a1, b0, b1 = a & M32, a >> 32, b & M32, b >> 32
    p00, c0 = mad(a0, b0, 0)
    t, c1 = mad(a1, b0, p00 >> 32)
    u, c = mad(a0, b1, t)
    h, c3 = mad(a1, b1, u >> 32)
    assert c0 == c1 == c3 == 0
    assert (h >> 32) + c <= M32          # r3 = hi(h) + c fits 32 bits
    # 128-bit product is r_l + 2^64 (h + c 2^32)
    r_l = (p00 & M32) | ((u & M32) << 32)
    assert a * b == r_l + ((h + (c << 32)) << 64)
    # subtraction with borrow-in c, then p added back on a borrow
    d = r_l - (h >> 32) - c
    if d < 0:
        y = (d + 2**64 + P) & M64         # wrapped word plus p, mod 2^64
        assert d + 2**64 >= 2**64 - 2**32 + 1 and y == d + 2**64 + P - 2**64
    else:
        y = d
    r = mad_eps_fold(h & M32, y)
    assert 0 <= r <= M64
    return r


def mul_plain(a, b):
    """The earlier sequence: the carry added into the high word first."""
    a0, a1, b0, b1 = a & M32, a >> 32, b & M32, b >> 32
    p00, _ = mad(a0, b0, 0)
    t, _ = mad(a1, b0, p00 >> 32)
    u, c = mad(a0, b1, t)
    hi, c3 = mad(a1, b1, (u >> 32) | (c << 32))
    assert c3 == 0
    lo = (p00 & M32) | ((u & M32) << 32)
    assert a * b == lo + (hi << 64)
    d = lo - (hi >> 32)
    y = d if d >= 0 else (d + 2**64 + P) & M64
    return mad_eps_fold(hi & M32, y)


EDGE = [0, 1, 2, EPS - 1, EPS, EPS + 1, 2**32, 2**63 - 1, 2**63, P - 2, P - 1, P, P + 1, M64 - 1, M64,
        0xFFFFFFFE00000000, 0xFFFFFFFF00000000, 0x00000001FFFFFFFF, 0xFFFFFFFEFFFFFFFF]


def test_fold_product_edges():
    for a in EDGE:
        for b in EDGE:
            r = mul_fold(a, b)
            assert r % P == a * b % P, (a, b)
            assert r == mul_plain(a, b), (a, b)


def test_fold_product_random():
    rnd = random.Random(5)
    for _ in range(20000):
        a, b = rnd.getrandbits(64), rnd.getrandbits(64)
        if rnd.random() < 0.2:
            a = rnd.choice(EDGE) ^ rnd.getrandbits(8)
        r = mul_fold(a, b)
        assert r % P == a * b % P
        assert r == mul_plain(a, b)


def test_fold_catches_a_dropped_carry():
    # The middle carry matters: a product that produces it, with the carry
    # ignored, gives a different residue (so the borrow-in is not dead).
    a = b = M64
    a0, a1, b0, b1 = a & M32, a >> 32, b & M32, b >> 32
    p00, _ = mad(a0, b0, 0)
    t, _ = mad(a1, b0, p00 >> 32)
    u, c = mad(a0, b1, t)
    assert c == 1
    h, _ = mad(a1, b1, u >> 32)
    r_l = (p00 & M32) | ((u & M32) << 32)
    wrong = (r_l - (h >> 32) + (h & M32) * EPS) % P
    assert wrong != a * b % P
