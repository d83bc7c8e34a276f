"""Pure-Python big-integer mini-oracle (tiny inputs only).

TEST INFRASTRUCTURE ONLY.  A second, independent transcription of the
textbook definitions that ``oracle.c`` implements, in Python integers:
field p = 2^64 - 2^32 + 1 (Sec. 2.4, Eq. 1); Poseidon with 4 full, 22
partial, 4 full rounds and x^7 (Sec. 2.4, Alg. 1 in its dense textbook
shape); rate-8 sponge with digest = state[0..3] (Sec. 2.4, Sec. 4.2); the
Merkle tree defined recursively (Sec. 2.4 "Merkle Tree", Sec. 4.2).  It also
holds the inverse permutation, used for a round-trip pin.
"""

from __future__ import annotations

P = (1 << 64) - (1 << 32) + 1
WIDTH, HALF_FULL, PARTIAL, ALPHA = 12, 4, 22, 7
ROUNDS = 2 * HALF_FULL + PARTIAL


def is_full(r: int) -> bool:
    return r < HALF_FULL or r >= HALF_FULL + PARTIAL


def permute(state, rc, mds):
    s = [v % P for v in state]
    for r in range(ROUNDS):
        s = [(s[i] + rc[r][i]) % P for i in range(WIDTH)]
        if is_full(r):
            s = [pow(v, ALPHA, P) for v in s]
        else:
            s[0] = pow(s[0], ALPHA, P)
        s = [sum(mds[i][j] * s[j] for j in range(WIDTH)) % P for i in range(WIDTH)]
    return s


def _mat_inv(m):
    """Inverse of a square matrix mod P by Gauss-Jordan elimination."""
    n = len(m)
    a = [[m[i][j] % P for j in range(n)] + [int(i == j) for j in range(n)] for i in range(n)]
    for c in range(n):
        piv = next(r for r in range(c, n) if a[r][c])
        a[c], a[piv] = a[piv], a[c]
        inv = pow(a[c][c], P - 2, P)
        a[c] = [v * inv % P for v in a[c]]
        for r in range(n):
            if r != c and a[r][c]:
                f = a[r][c]
                a[r] = [(x - f * y) % P for x, y in zip(a[r], a[c])]
    return [row[n:] for row in a]


def inverse_permute(state, rc, mds):
    """Undo ``permute``: inverse matrix, then the S-box inverse x^d with
    d = 7^-1 mod (p - 1) (it exists because gcd(7, p - 1) = 1), then minus C."""
    d = pow(ALPHA, -1, P - 1)
    minv = _mat_inv(mds)
    s = [v % P for v in state]
    for r in reversed(range(ROUNDS)):
        s = [sum(minv[i][j] * s[j] for j in range(WIDTH)) % P for i in range(WIDTH)]
        if is_full(r):
            s = [pow(v, d, P) for v in s]
        else:
            s[0] = pow(s[0], d, P)
        s = [(s[i] - rc[r][i]) % P for i in range(WIDTH)]
    return s


def sponge(words, rc, mds):
    s = [0] * WIDTH
    for k in range(0, len(words), 8):
        chunk = list(words[k:k + 8]) + [0] * (8 - len(words[k:k + 8]))
        s = [(s[i] + chunk[i]) % P for i in range(8)] + s[8:]
        s = permute(s, rc, mds)
    return s[:4]


def merkle_root_recursive(digests, rc, mds):
    """Root of the tree over ``digests`` by the recursive definition: the
    root of a list is the hash of the roots of its left part (the largest
    power of two strictly below its length) and its right part.  This is the
    same tree as level-by-level pairing with an unpaired last node moved up."""
    n = len(digests)
    if n == 1:
        return list(digests[0])
    k = 1
    while k * 2 < n:
        k *= 2
    left = merkle_root_recursive(digests[:k], rc, mds)
    right = merkle_root_recursive(digests[k:], rc, mds)
    return sponge(left + right, rc, mds)


def merkle_levels(digests, rc, mds):
    """All levels, bottom-up, by pairing (2i, 2i+1)."""
    levels = [[list(d) for d in digests]]
    while len(levels[-1]) > 1:
        cur = levels[-1]
        nxt = []
        for i in range(0, len(cur), 2):
            nxt.append(sponge(cur[i] + cur[i + 1], rc, mds) if i + 1 < len(cur) else cur[i])
        levels.append(nxt)
    return levels
