"""GPU parity at full size: every node of the paper-scale trees against the
oracle, word for word.

The oracle's nodes are recorded level by level in ``tests/golden/fullsize.json``
by ``tests/golden/make_golden.py`` (which calls only the oracle): the SHA-256
of each level's words and the root.  Here the same trees are built on the GPU
from the same seeded inputs (generated on the device by the twin generator),
every level is hashed the same way, and every digest must be equal.  A
mismatch names the levels that differ; the sampled tests in test_gpu_parity.py
then point at the nodes.

* 2^22 leaves x 8 words, seed 1 (the tree of Sec. 4.2): all 2^23 - 1 nodes;
* 2^21 rows x 256 words, seed 2: all 2^22 - 1 nodes;
* the 64 uneven trees of the batched workload, seed 3, built in one batched
  call (every schedule knob at its default) and as 64 plain builds.
"""

import json
import os

import pytest

import paper_2506_09505_amd as goldi
from synth.inputs import tree_shapes

from .golden.make_golden import BATCH64, TREE22, WIDE21, level_digests
from .gpu_util import banner, to_host

pytestmark = pytest.mark.gpu

FIXTURE = os.path.join(os.path.dirname(__file__), "golden", "fullsize.json")


@pytest.fixture(scope="module")
def golden():
    with open(FIXTURE) as f:
        return json.load(f)


def assert_levels(nodes_dev, n_rows, want, what):
    nodes = to_host(nodes_dev).reshape(-1, 4)
    got = level_digests(nodes, n_rows)
    assert [g["n"] for g in got] == [w["n"] for w in want["levels"]], what
    bad = [k for k, (g, w) in enumerate(zip(got, want["levels"])) if g["sha256"] != w["sha256"]]
    assert not bad, "%s: levels %s differ from the oracle" % (what, bad)
    assert [str(int(v)) for v in nodes[-1]] == want["root"], what


def device_leaves(n, w, seed, stream):
    from synth import fill
    return fill.leaves_colmajor_dev(n, w, seed=seed, stream=stream)


def test_paper_scale_tree_every_node(golden):
    r, want = TREE22, golden["tree22"]
    banner("every node of %dx%d seed %d" % (r["n_rows"], r["n_cols"], r["seed"]))
    lv = device_leaves(r["n_rows"], r["n_cols"], r["seed"], r["stream"])
    nodes = goldi.goldi_merkle_build(lv, r["n_rows"], r["n_cols"])
    assert nodes.shape[0] == 2 * r["n_rows"] - 1
    assert_levels(nodes, r["n_rows"], want, "tree22")


def test_paper_scale_tree_async_every_node(golden):
    # The launch configuration the benchmark times: the asynchronous entry
    # point on torch's current stream, into a reused node buffer.
    import torch
    r, want = TREE22, golden["tree22"]
    banner("every node of %dx%d, async on the current stream" % (r["n_rows"], r["n_cols"]))
    lv = device_leaves(r["n_rows"], r["n_cols"], r["seed"], r["stream"])
    nodes = torch.empty(goldi.goldi_merkle_num_nodes(r["n_rows"]) * 4, dtype=torch.uint64, device="cuda:0")
    status = torch.zeros(1, dtype=torch.int32, device="cuda:0")
    for _ in range(2):
        goldi.goldi_merkle_build_async(lv, r["n_rows"], r["n_cols"], nodes, status)
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    assert_levels(nodes, r["n_rows"], want, "tree22 async")


def test_wide_rows_every_node(golden):
    import torch
    r, want = WIDE21, golden["wide21"]
    banner("every node of %dx%d seed %d" % (r["n_rows"], r["n_cols"], r["seed"]))
    lv = device_leaves(r["n_rows"], r["n_cols"], r["seed"], r["stream"])
    nodes = goldi.goldi_merkle_build(lv, r["n_rows"], r["n_cols"])
    del lv
    torch.cuda.empty_cache()
    assert_levels(nodes, r["n_rows"], want, "wide21")


@pytest.mark.parametrize("batch_mode", [1, 0])
def test_batched_workload_every_node(golden, batch_mode):
    b, want = BATCH64, golden["batch64"]
    rows, ws = tree_shapes(b["seed"], b["n_trees"], b["lo_log2"], b["hi_log2"], b["widths"])
    banner("every node of the %d batched trees, batch_mode %d" % (b["n_trees"], batch_mode))
    trees = [(device_leaves(int(n), int(w), b["seed"], k), int(n), int(w)) for k, (n, w) in enumerate(zip(rows, ws))]
    assert [(t["n_rows"], t["n_cols"]) for t in want["trees"]] == [(n, w) for _, n, w in trees]
    old = goldi.goldi_tune_get("batch_mode")
    try:
        goldi.goldi_tune_set("batch_mode", batch_mode)
        outs = goldi.goldi_merkle_build_many(trees)
    finally:
        goldi.goldi_tune_set("batch_mode", old)
    for k, ((_, n, _), o) in enumerate(zip(trees, outs)):
        assert_levels(o, n, want["trees"][k], "batched tree %d" % k)
