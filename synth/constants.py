"""Seed-derived instance parameters of Poseidon-12 over Goldilocks.

The paper (Sec. 2.4, Alg. 1) fixes the structure of the permutation: a
12-element state, 4 + 22 + 4 rounds, the x^7 S-box, a 12 x 12 MDS matrix and
"vectors and matrices of constants" C, M, S.  It prints none of their values,
and Table 1's ``mult_72`` / ``mmult_4x12_8`` show the MDS entries fit in
8 bits.  So this module *draws* them, once, from a fixed seed:

* bit generator: numpy ``PCG64(250609505)`` (the arXiv id digits), consumed
  through ``random_raw()`` so the stream does not depend on numpy's
  integer-sampling algorithms;
* round constants ``rc[r][i]`` for r = 0..29, i = 0..11 in row-major order,
  each the next raw 64-bit draw below p (draws >= p are skipped);
* the first row ``m[0..11]`` of the circulant ``M[i][j] = m[(j - i) mod 12]``,
  each ``1 + (raw >> 58)``, i.e. uniform on [1, 64].

``S`` (the sparse partial-round matrices) is not drawn: it is derived from M
by whoever evaluates the fast form of the permutation, so the function stays
the textbook Poseidon defined by ``rc`` and ``M``.

Run ``python -m synth.constants`` to (re)write ``poseidon12.json``; the file
is committed and its SHA-256 is checked by the tests.
"""

from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from .inputs import GOLDILOCKS_P

SEED = 250609505
WIDTH = 12
N_ROUNDS = 30
CONSTANTS_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "poseidon12.json")


def draw_constants(seed: int = SEED):
    bg = np.random.PCG64(seed)
    rc = []
    while len(rc) < N_ROUNDS * WIDTH:
        v = int(bg.random_raw())
        if v < GOLDILOCKS_P:
            rc.append(v)
    m = [1 + (int(bg.random_raw()) >> 58) for _ in range(WIDTH)]
    rc2 = [rc[r * WIDTH:(r + 1) * WIDTH] for r in range(N_ROUNDS)]
    mds = [[m[(j - i) % WIDTH] for j in range(WIDTH)] for i in range(WIDTH)]
    return rc2, m, mds


def build_spec(seed: int = SEED) -> dict:
    rc, m, mds = draw_constants(seed)
    return {
        "name": "poseidon12-goldilocks-seeded",
        "p": str(GOLDILOCKS_P),
        "width": WIDTH,
        "rate": 8,
        "capacity": 4,
        "digest": 4,
        "alpha": 7,
        "full_rounds": 8,
        "partial_rounds": 22,
        "seed": seed,
        "generator": ("numpy PCG64(seed).random_raw(); rc row-major, raw draws >= p skipped; "
                      "then m[k] = 1 + (raw >> 58) for k = 0..11"),
        "mds_convention": "new_state[i] = sum_j mds[i][j] * state[j]; mds[i][j] = m[(j - i) mod 12]",
        "mds_first_row": m,
        "mds": mds,
        "rc": [[str(v) for v in row] for row in rc],
    }


def spec_bytes(spec: dict) -> bytes:
    return (json.dumps(spec, indent=1) + "\n").encode()


def load_constants(path: str = CONSTANTS_PATH):
    """Return ``(rc, mds)`` as Python int lists: rc[30][12], mds[12][12]."""
    with open(path) as f:
        spec = json.load(f)
    rc = [[int(v) for v in row] for row in spec["rc"]]
    mds = [[int(v) for v in row] for row in spec["mds"]]
    return rc, mds


def file_sha256(path: str = CONSTANTS_PATH) -> str:
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


if __name__ == "__main__":
    data = spec_bytes(build_spec())
    with open(CONSTANTS_PATH, "wb") as f:
        f.write(data)
    print(CONSTANTS_PATH, hashlib.sha256(data).hexdigest())
