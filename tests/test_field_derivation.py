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
    """The product with the middle carry folded into the reduction and the
    borrow fixed up (p added) before the final fold: the earlier sequence of
    the generated blocks, kept as a second derivation of the same residue."""
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


def reduce_split(a_lo, a_hi):
    """The row reduction of poseidon.hpp, for a_lo, a_hi < 2^63: r = a_lo +
    h1 (2^32 - 1) with one multiply-add, then h0 added into r's high word
    (carry c out of 64 bits), then c (2^32 - 1) added back."""
    assert 0 <= a_lo < 2**63 and 0 <= a_hi < 2**63
    h0, h1 = a_hi & M32, a_hi >> 32
    r, c0 = mad(h1, EPS, a_lo)
    assert c0 == 0                       # the first multiply-add never carries
    s_hi = (r >> 32) + h0
    c = s_hi >> 32
    s = (r & M32) | ((s_hi & M32) << 32)
    out, c1 = mad(c, EPS, s)
    assert c1 == 0                       # nor does the last one
    return out


def test_row_reduction_edges_and_random():
    rnd = random.Random(9)
    edge = [0, 1, M32, M32 + 1, 2**42, 2**58 - 1, 2**62, 2**63 - 1, 2**63 - 2**32, P >> 1]
    cases = [(a, b) for a in edge for b in edge]
    cases += [(rnd.getrandbits(63), rnd.getrandbits(63)) for _ in range(20000)]
    cases += [(rnd.getrandbits(43), rnd.getrandbits(43)) for _ in range(5000)]   # full-round rows
    for a_lo, a_hi in cases:
        r = reduce_split(a_lo, a_hi)
        assert 0 <= r <= M64 and r % P == (a_lo + (a_hi << 32)) % P, (a_lo, a_hi)


def test_row_reduction_needs_its_bound():
    # Above 2^63 the first multiply-add can overflow: the bound is needed, and
    # the generator keeps every block row below it.
    a_lo, a_hi = M64 - 5, M64 - 5
    _, c0 = mad(a_hi >> 32, EPS, a_lo)
    assert c0 == 1


def mul_merged(a, b):
    """field.hpp's product, with the borrow's fix-up merged into the final
    fold: y = r_l - hi(h) - c with borrow b,
    r1 + k 2^64 = lo(h) (2^32 - 1) + y, d = k - b, r = r1 - d + d 2^32.
    Returns (r, d)."""
    a0, a1, b0, b1 = a & M32, a >> 32, b & M32, b >> 32
    p00, _ = mad(a0, b0, 0)
    t, _ = mad(a1, b0, p00 >> 32)
    u, c = mad(a0, b1, t)
    h, _ = mad(a1, b1, u >> 32)
    r_l = (p00 & M32) | ((u & M32) << 32)
    y = r_l - (h >> 32) - c
    brw = 1 if y < 0 else 0
    y &= M64
    r1, k = mad(h & M32, EPS, y)
    d = k - brw
    assert d in (-1, 0, 1)
    if d == -1:
        assert (h & M32) == 0            # only when lo(h) = 0
    # v_mad_i64_i32 d, -1, r1 (signed 64-bit result), then d into the high word
    r2 = (r1 - d) & M64
    r = (r2 & M32) | ((((r2 >> 32) + d) & M32) << 32)
    assert r == r1 + d * EPS             # exact: no wrap in any case
    return r, d


def test_merged_product_edges_and_random():
    rnd = random.Random(17)
    cases = [(a, b) for a in EDGE for b in EDGE]
    cases += [(rnd.getrandbits(64), rnd.getrandbits(64)) for _ in range(30000)]
    seen = set()
    for a, b in cases:
        r, d = mul_merged(a, b)
        seen.add(d)
        assert 0 <= r <= M64 and r % P == a * b % P, (a, b)
    assert {0, 1} <= seen


def test_merged_product_negative_correction():
    # a = s 2^48, b = t 2^48: a b = s t 2^96, so bits 64..95 are zero (lo(h) = 0)
    # and the low word (0) is below the top part: the subtraction borrows and
    # nothing carries, d = -1, the rarely taken case.
    rnd = random.Random(23)
    pairs = [(1, 1), (3, 5), (1 << 14, (1 << 15) + 1)]
    pairs += [(rnd.randrange(1, 1 << 15), rnd.randrange(1, 1 << 15)) for _ in range(2000)]
    for s_, t_ in pairs:
        a, b = s_ << 48, t_ << 48
        r, d = mul_merged(a, b)
        assert d == -1, (s_, t_)
        assert r % P == a * b % P
