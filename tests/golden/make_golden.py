"""Writes the regression fixtures in this folder.  Calls only the oracle.

Run: python tests/golden/make_golden.py

These are frozen oracle outputs (not values printed by the paper, which
prints none): the permutation of three fixed states and the root and first
leaf digests of the 2^10 x 8 tree (seed 0).  They guard against accidental
changes to the instance or the oracle; the pins in test_oracle_*.py are what
tie the oracle to the paper.
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth.inputs import leaves_colmajor  # noqa: E402


def main():
    prm = oracle.spec_params()
    p = oracle.P
    states = np.array([[0] * 12, list(range(12)), [p - 1] * 12], dtype=np.uint64)
    perm = oracle.permute(prm, states)
    n, w = 1 << 10, 8
    nodes = oracle.merkle_build(prm, leaves_colmajor(n, w, seed=0), n, w)
    out = {
        "source": "oracle (tests/golden/make_golden.py); instance synth/poseidon12.json",
        "permute": {"inputs": [[str(int(v)) for v in s] for s in states],
                    "outputs": [[str(int(v)) for v in s] for s in perm]},
        "tree_1024x8_seed0": {"root": [str(int(v)) for v in nodes[-1]],
                              "leaf0": [str(int(v)) for v in nodes[0]],
                              "num_nodes": int(nodes.shape[0])},
    }
    with open(os.path.join(HERE, "oracle_vectors.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
