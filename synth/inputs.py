"""Counter-based generator of uniform Goldilocks words.

Definition (the same definition is implemented a second time, in HIP, by
``synth/fill.hip`` for device-side generation of large inputs):

    mix(z):   z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
              z = (z ^ (z >> 27)) * 0x94D049BB133111EB
              return z ^ (z >> 31)                      (all mod 2^64)

This is the SplitMix64 output finaliser (Steele, Lea, Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014).

    key(seed, stream)   = mix(seed * 0x9E3779B97F4A7C15 + stream * 0xD1B54A32D192ED03 + 1)
    word(seed, stream, i):
        z = mix(key + (i + 1) * 0x9E3779B97F4A7C15)
        while z >= p:  z = mix(z + 0x9E3779B97F4A7C15)  # rejection: uniform on [0, p)
        return z

``i`` is the element index.  For a column-major leaf matrix of ``n_rows``
rows, element (r, c) has index ``c * n_rows + r``.
"""

from __future__ import annotations

import numpy as np

GOLDILOCKS_P = 0xFFFFFFFF00000001
_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_STREAM_MUL = np.uint64(0xD1B54A32D192ED03)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_P = np.uint64(GOLDILOCKS_P)


def splitmix64_mix(z):
    """SplitMix64 finaliser on a uint64 array (wrapping arithmetic)."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def stream_key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        k = (np.uint64(seed % 2**64) * _GAMMA + np.uint64(stream % 2**64) * _STREAM_MUL
             + np.uint64(1))
    return splitmix64_mix(np.array([k], dtype=np.uint64))[0]


def goldilocks_words(seed: int, stream: int, start: int, count: int,
                     chunk: int = 1 << 24) -> np.ndarray:
    """Words ``start .. start+count-1`` of stream (seed, stream), uniform on [0, p)."""
    key = stream_key(seed, stream)
    out = np.empty(count, dtype=np.uint64)
    for off in range(0, count, chunk):
        m = min(chunk, count - off)
        idx = np.arange(start + off + 1, start + off + 1 + m, dtype=np.uint64)
        with np.errstate(over="ignore"):
            z = splitmix64_mix(key + idx * _GAMMA)
        bad = z >= _P
        while bad.any():
            with np.errstate(over="ignore"):
                z[bad] = splitmix64_mix(z[bad] + _GAMMA)
            bad = z >= _P
        out[off:off + m] = z
    return out


def words_at(seed: int, stream: int, indices) -> np.ndarray:
    """Words at arbitrary element indices (for sampled checks of huge inputs)."""
    key = stream_key(seed, stream)
    idx = np.asarray(indices, dtype=np.uint64) + np.uint64(1)
    with np.errstate(over="ignore"):
        z = splitmix64_mix(key + idx * _GAMMA)
    bad = z >= _P
    while bad.any():
        with np.errstate(over="ignore"):
            z[bad] = splitmix64_mix(z[bad] + _GAMMA)
        bad = z >= _P
    return z


def leaves_colmajor(n_rows: int, n_cols: int, seed: int, stream: int = 0) -> np.ndarray:
    """A column-major leaf matrix as a flat array: element (r, c) at ``c*n_rows + r``."""
    return goldilocks_words(seed, stream, 0, n_rows * n_cols)


def uniform_states(n: int, seed: int, stream: int = 1) -> np.ndarray:
    """``n`` permutation states, ``[n][12]`` row-major, uniform on [0, p)."""
    return goldilocks_words(seed, stream, 0, n * 12).reshape(n, 12)


# Values that exercise carries and the reduction identity 2^64 = 2^32 - 1 (mod p).
EDGE_WORDS = [0, 1, 2, 3, 0xFFFFFFFF, 0x100000000, 0x100000001, 0x7FFFFFFFFFFFFFFF,
              0x8000000000000000, 0xFFFFFFFEFFFFFFFF, GOLDILOCKS_P - 2, GOLDILOCKS_P - 1,
              0xFFFFFFFF, 0xFFFFFFFF00000000]


def edge_states() -> np.ndarray:
    """Hand-picked permutation states: all-zero, all p-1, ramps and edge words."""
    p = GOLDILOCKS_P
    rows = [[0] * 12, [p - 1] * 12, list(range(12)), [1] * 12,
            [0xFFFFFFFF] * 12, [0x100000000] * 12, [0xFFFFFFFF00000000] * 12,
            [(p - 1 - i) for i in range(12)]]
    e = EDGE_WORDS
    for s in range(8):
        rows.append([e[(s * 5 + 3 * i) % len(e)] for i in range(12)])
    return np.array(rows, dtype=np.uint64)


def tree_shapes(seed: int, n_trees: int, lo_log2: float, hi_log2: float, widths,
                stream: int = 0xB47C):
    """Row counts ``floor(2^U)``, U uniform on [lo_log2, hi_log2], and widths drawn
    uniformly from ``widths``: the shape stream of the batched and served workloads."""
    key = stream_key(seed, stream)
    idx = np.arange(1, 2 * n_trees + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = splitmix64_mix(key + idx * _GAMMA)
    u = (z[0::2] >> np.uint64(11)).astype(np.float64) / float(1 << 53)
    rows = np.floor(2.0 ** (lo_log2 + u * (hi_log2 - lo_log2))).astype(np.int64)
    rows = np.clip(rows, int(2 ** lo_log2), int(2 ** hi_log2))
    w = np.asarray(widths, dtype=np.int64)[(z[1::2] % np.uint64(len(widths))).astype(np.int64)]
    return rows, w


def poisson_arrivals(seed: int, n: int, rate_per_s: float, stream: int = 0xA771):
    """Arrival times (seconds) of a Poisson process of the given rate."""
    key = stream_key(seed, stream)
    idx = np.arange(1, n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = splitmix64_mix(key + idx * _GAMMA)
    u = ((z >> np.uint64(11)).astype(np.float64) + 0.5) / float(1 << 53)
    return np.cumsum(-np.log(u) / rate_per_s)
