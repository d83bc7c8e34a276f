"""Writes the regression fixtures in this folder.  Calls only the oracle.

Run: python tests/golden/make_golden.py [small] [tree22] [wide21] [batch64] [serve]
(no argument: all of them; the large ones take tens of minutes of CPU).

These are frozen oracle outputs (not values printed by the paper, which
prints none).  They guard against accidental changes to the instance or the
oracle; the pins in test_oracle_*.py are what tie the oracle to the paper.

* ``oracle_vectors.json`` (``small``): the permutation of three fixed states
  and the root and first leaf digest of the 2^10 x 8 tree (seed 0).
* ``fullsize.json``: every node of the paper-scale trees, recorded level by
  level as the SHA-256 of the level's words (each word as 8 little-endian
  bytes, nodes in order, 4 words per node) plus the root's words:
    - ``tree22``: 2^22 leaves x 8 words, seed 1 (the shape of Sec. 4.2);
    - ``wide21``: 2^21 rows x 256 words, column-major, seed 2;
    - ``batch64``: the 64 uneven trees of the batched workload (shapes from
      the shape stream of seed 3, tree k from seed 3, stream k);
    - ``serve``: roots of a stratified sample of the served request stream
      (seed 4, the first 1,100 requests): every request of at most 2^16 rows
      and 8 seeded picks among the larger ones.  Request k's leaves are the
      first n_rows * n_cols words of stream 100 + (k mod 4) of seed 4.
A GPU test that hashes its own levels the same way and finds every digest
equal has matched every node, word for word.
"""

import hashlib
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
from synth.inputs import goldilocks_words, leaves_colmajor, tree_shapes  # noqa: E402

FULLSIZE = os.path.join(HERE, "fullsize.json")

# Workload recipes (shared with the GPU tests that read the fixtures).
TREE22 = dict(n_rows=1 << 22, n_cols=8, seed=1, stream=0)
WIDE21 = dict(n_rows=1 << 21, n_cols=256, seed=2, stream=0)
BATCH64 = dict(seed=3, n_trees=64, lo_log2=10, hi_log2=20, widths=(8, 16, 32, 64, 128))
SERVE = dict(seed=4, n_requests=1100, lo_log2=12, hi_log2=22, widths=(8, 32, 64), small_max_rows=1 << 16,
             n_large=8, pick_seed=20250609, buffers=4, buffer_stream0=100)


def level_digests(nodes: np.ndarray, n_rows: int):
    """[(level size, sha256 hex)] of every level of a level-major node array."""
    nodes = np.ascontiguousarray(nodes, dtype=np.uint64).reshape(-1, 4)
    out, off, n = [], 0, n_rows
    while True:
        out.append({"n": int(n), "sha256": hashlib.sha256(nodes[off:off + n].astype("<u8").tobytes()).hexdigest()})
        off += n
        if n == 1:
            break
        n = (n + 1) // 2
    assert off == nodes.shape[0]
    return out


def tree_record(prm, lv, n, w, **extra):
    t0 = time.time()
    nodes = oracle.merkle_build(prm, lv, n, w)
    rec = dict(extra, n_rows=int(n), n_cols=int(w), levels=level_digests(nodes, n),
               root=[str(int(v)) for v in nodes[-1]])
    print("  %d x %d: %.1f s" % (n, w, time.time() - t0), flush=True)
    return rec


def serve_sample():
    """Indices of the served requests whose roots are recorded."""
    s = SERVE
    rows, _ = tree_shapes(s["seed"], s["n_requests"], s["lo_log2"], s["hi_log2"], s["widths"])
    small = [k for k in range(len(rows)) if rows[k] <= s["small_max_rows"]]
    large = [k for k in range(len(rows)) if rows[k] > s["small_max_rows"]]
    pick = np.random.default_rng(s["pick_seed"]).choice(len(large), s["n_large"], replace=False)
    return sorted(small + [large[i] for i in pick])


def make_small(prm):
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


def make_tree(prm, recipe):
    r = recipe
    lv = leaves_colmajor(r["n_rows"], r["n_cols"], seed=r["seed"], stream=r["stream"])
    return tree_record(prm, lv, r["n_rows"], r["n_cols"], seed=r["seed"], stream=r["stream"])


def make_batch(prm):
    b = BATCH64
    rows, ws = tree_shapes(b["seed"], b["n_trees"], b["lo_log2"], b["hi_log2"], b["widths"])
    trees = []
    for k, (n, w) in enumerate(zip(rows, ws)):
        lv = leaves_colmajor(int(n), int(w), seed=b["seed"], stream=k)
        trees.append(tree_record(prm, lv, int(n), int(w), tree=k, seed=b["seed"], stream=k))
    return dict(b, widths=list(b["widths"]), trees=trees)


def make_serve(prm):
    s = SERVE
    rows, ws = tree_shapes(s["seed"], s["n_requests"], s["lo_log2"], s["hi_log2"], s["widths"])
    reqs = []
    for k in serve_sample():
        n, w = int(rows[k]), int(ws[k])
        lv = goldilocks_words(s["seed"], s["buffer_stream0"] + k % s["buffers"], 0, n * w)
        nodes = oracle.merkle_build(prm, lv, n, w)
        reqs.append({"request": k, "n_rows": n, "n_cols": w, "root": [str(int(v)) for v in nodes[-1]]})
    print("  %d served requests" % len(reqs), flush=True)
    return dict(s, widths=list(s["widths"]), requests=reqs)


def update_fullsize(key, value):
    data = {}
    if os.path.exists(FULLSIZE):
        with open(FULLSIZE) as f:
            data = json.load(f)
    data["source"] = ("oracle (tests/golden/make_golden.py); instance synth/poseidon12.json; level digest = "
                      "SHA-256 of the level's words as 8-byte little-endian integers, nodes in order")
    data[key] = value
    tmp = FULLSIZE + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, FULLSIZE)


def main(argv):
    what = argv or ["small", "tree22", "wide21", "batch64", "serve"]
    prm = oracle.spec_params()
    for name in what:
        print(name, flush=True)
        if name == "small":
            make_small(prm)
        elif name == "tree22":
            update_fullsize("tree22", make_tree(prm, TREE22))
        elif name == "wide21":
            update_fullsize("wide21", make_tree(prm, WIDE21))
        elif name == "batch64":
            update_fullsize("batch64", make_batch(prm))
        elif name == "serve":
            update_fullsize("serve", make_serve(prm))
        else:
            raise SystemExit("unknown fixture %r" % name)


if __name__ == "__main__":
    main(sys.argv[1:])
