"""GPU: the serving loop.  Each served result must equal the same build done
alone (goldi_merkle_build) and the oracle, whatever else was in the mix;
admission must respect the HBM budget; a bad request fails alone, even inside
a batch; a batch that fails is rebuilt request by request; the watchdog
reports an overrunning batch without freeing memory the device still uses;
destroy never waits on work that cannot start."""

import json
import os
import random
import threading
import time

import numpy as np
import pytest

import oracle
import paper_2506_09505_amd as goldi
from synth.inputs import GOLDILOCKS_P, leaves_colmajor, tree_shapes

from .gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prm():
    return oracle.spec_params()


def make_requests(seed, count, lo, hi, widths):
    import torch
    rows, ws = tree_shapes(seed, count, lo, hi, widths)
    reqs = []
    for k, (n, w) in enumerate(zip(rows, ws)):
        lv = leaves_colmajor(int(n), int(w), seed=seed, stream=k)
        if k % 2 == 0:
            src = torch.from_numpy(lv.view(np.int64)).pin_memory().view(torch.uint64)   # host, pinned
        else:
            src = to_dev(lv)                                                              # device
        reqs.append((int(n), int(w), lv, src))
    return reqs


def blocker():
    """A device-resident request that keeps a single slot busy for about a
    millisecond, so that requests submitted right after it queue up and are
    admitted together."""
    from synth import fill
    n, w = 1 << 18, 64
    return fill.leaves_colmajor_dev(n, w, seed=99, stream=0), n, w


def submit_blocker(srv):
    """Submits the blocker and returns once the server has admitted it as a
    group of its own (a request submitted before that could join its group).
    Returns its id and its leaves, which must outlive the build."""
    import time
    b_lv, b_n, b_w = blocker()
    groups = srv.stats()["groups"]
    rid = srv.submit(b_lv, b_n, b_w)
    t0 = time.monotonic()
    while srv.stats()["groups"] == groups:
        assert time.monotonic() - t0 < 10, "the blocker was not admitted"
        time.sleep(1e-4)
    return rid, b_lv


def test_served_equals_alone_and_oracle(prm):
    banner("serving mix of 40 requests")
    reqs = make_requests(21, 40, 4, 12, (1, 8, 9, 32, 64))
    rnd = random.Random(0)
    with goldi.GoldiServer(256 << 20, n_slots=4, max_group=4) as srv:
        ids = []
        for n, w, lv, src in reqs:
            ids.append(srv.submit(src, n, w))
            time.sleep(rnd.uniform(0, 0.002))
        infos = [srv.wait(i) for i in ids]
        for (n, w, lv, src), rid, info in zip(reqs, ids, infos):
            assert info["status"] == 0
            served = to_host(srv.nodes(rid)).reshape(-1, 4)
            alone = to_host(goldi.goldi_merkle_build(to_dev(lv), n, w)).reshape(-1, 4)
            assert (served == alone).all(), (n, w)
            assert (served == oracle.merkle_build(prm, lv, n, w)).all(), (n, w)
            assert [int(v) for v in served[-1]] == info["root"]
            assert info["t_submit_ns"] <= info["t_admit_ns"] <= info["t_done_ns"]
            srv.release(rid)
        st = srv.stats()
        assert st["admitted"] == 40 and st["peak_bytes"] <= 256 << 20
        assert st["groups"] <= 40


def test_budget_limits_admission(prm):
    banner("serving under a tight budget")
    reqs = make_requests(22, 10, 9, 11, (8, 32))
    biggest = max(goldi.goldi_merkle_num_nodes(n) * 32 + n * w * 8 for n, w, _, _ in reqs)
    budget = 2 * biggest
    with goldi.GoldiServer(budget, n_slots=8, max_group=8) as srv:
        ids = [srv.submit(src, n, w) for n, w, _, src in reqs]
        for (n, w, lv, _), rid in zip(reqs, ids):
            info = srv.wait(rid)
            assert info["status"] == 0
            assert (to_host(srv.nodes(rid)).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all()
            srv.release(rid)
        assert srv.stats()["peak_bytes"] <= budget


def test_oversized_request_rejected():
    import torch
    with goldi.GoldiServer(1 << 20) as srv:
        big = torch.zeros(1 << 18, dtype=torch.uint64, device="cuda:0")
        with pytest.raises(goldi.GoldiError) as e:
            srv.submit(big, 1 << 15, 8)
        assert e.value.code == goldi.GOLDI_ENOMEM


def test_bad_request_fails_alone(prm):
    # One slot, busy with a blocker while the bad request and its neighbours
    # are queued: they are admitted as one batch, and only the bad one fails.
    banner("serving with one non-canonical request inside a batch")
    reqs = make_requests(23, 6, 6, 9, (8, 16))
    bad_lv = leaves_colmajor(100, 8, seed=1)
    bad_lv[17] = np.uint64(GOLDILOCKS_P)
    with goldi.GoldiServer(1 << 30, n_slots=1, max_group=8) as srv:
        first, b_lv = submit_blocker(srv)
        ids = [srv.submit(to_dev(bad_lv), 100, 8)] + [srv.submit(src, n, w) for n, w, _, src in reqs]
        assert srv.wait(first)["status"] == 0
        bad = srv.wait(ids[0])
        assert bad["status"] == goldi.GOLDI_ENONCANON
        assert bad["group_size"] > 1, "the bad request was not batched with others"
        for (n, w, lv, _), rid in zip(reqs, ids[1:]):
            info = srv.wait(rid)
            assert info["status"] == 0, (n, w)
            assert (to_host(srv.nodes(rid)).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all()
        with pytest.raises(goldi.GoldiError):
            srv.nodes(ids[0])


def test_failed_batch_is_rebuilt_alone(prm):
    # The server is told to treat its next batch of two or more requests as
    # failed at launch (forced on the host, nothing reaches the GPU for it);
    # each request must then be rebuilt in a batch of its own and succeed.
    banner("serving: a failed batch is rebuilt request by request")
    reqs = make_requests(24, 5, 6, 10, (8, 32))
    with goldi.GoldiServer(1 << 30, n_slots=1, max_group=8) as srv:
        srv.set("fail_next_batches", 1)
        first, b_lv = submit_blocker(srv)
        ids = [srv.submit(src, n, w) for n, w, _, src in reqs]
        assert srv.wait(first)["status"] == 0
        for (n, w, lv, _), rid in zip(reqs, ids):
            info = srv.wait(rid)
            assert info["status"] == 0, (n, w)
            assert info["group_size"] == 1
            assert (to_host(srv.nodes(rid)).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all()
            srv.release(rid)
        # the blocker, the failed batch, then one batch per request
        assert srv.stats()["groups"] == 2 + len(reqs)


def test_watchdog_reports_and_server_recovers(prm):
    # A 1 us watchdog makes an ordinary ~1 ms build overrun (the kernels run
    # to their normal end): it is reported GOLDI_ETIMEDOUT, its release is
    # deferred until the device work ends, and the server keeps serving.
    banner("serving: watchdog")
    with goldi.GoldiServer(1 << 30, n_slots=2, max_group=4) as srv:
        srv.set("watchdog_us", 1)
        b_lv, b_n, b_w = blocker()
        rid = srv.submit(b_lv, b_n, b_w)
        assert srv.wait(rid)["status"] == goldi.GOLDI_ETIMEDOUT
        srv.release(rid)
        srv.set("watchdog_us", 0)
        n, w = 300, 9
        lv = leaves_colmajor(n, w, seed=5)
        rid = srv.submit(to_dev(lv), n, w)
        info = srv.wait(rid)
        assert info["status"] == 0
        assert (to_host(srv.nodes(rid)).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all()


def test_destroy_returns_with_requests_queued():
    # The budget holds one request; completed requests are never released, so
    # the others can never be admitted.  Destroy must cancel them and return.
    banner("serving: destroy with requests that cannot be admitted")
    n, w = 1 << 10, 8
    need = goldi.goldi_merkle_num_nodes(n) * 32
    srv = goldi.GoldiServer(need + 1024, n_slots=2, max_group=2)
    lv = to_dev(leaves_colmajor(n, w, seed=6))
    ids = [srv.submit(lv, n, w) for _ in range(3)]
    assert srv.wait(ids[0])["status"] == 0
    done = threading.Event()

    def close():
        srv.close()
        done.set()

    th = threading.Thread(target=close, daemon=True)
    th.start()
    assert done.wait(30), "goldi_server_destroy did not return"


def test_served_workload_shapes_vs_alone_and_oracle():
    # The served workload's shapes (rows floor(2^U), U uniform on [12, 22];
    # widths {8, 32, 64}; seed 4; request k reads the first n*w words of
    # stream 100 + k mod 4): the first 24 requests of that stream, admitted
    # by continuous batching.  Every served tree must equal its standalone
    # build word for word, and the roots recorded by the oracle for this
    # stream (tests/golden/fullsize.json) must match.
    import torch
    from synth import fill
    from .golden.make_golden import SERVE
    s = SERVE
    count = 24
    rows, ws = tree_shapes(s["seed"], count, s["lo_log2"], s["hi_log2"], s["widths"])
    banner("served workload shapes: %d requests, %d rows in total" % (count, int(rows.sum())))
    words = int(max(int(n) * int(w) for n, w in zip(rows, ws)))
    bufs = []
    for b in range(s["buffers"]):
        t = torch.empty(words, dtype=torch.uint64, device="cuda:0")
        bufs.append(fill.fill_words(t, s["seed"], s["buffer_stream0"] + b))
    with open(os.path.join(os.path.dirname(__file__), "golden", "fullsize.json")) as f:
        golden_roots = {q["request"]: q["root"] for q in json.load(f)["serve"]["requests"]}
    with goldi.GoldiServer(64 * 10**9, n_slots=8, max_group=8) as srv:
        ids = [srv.submit(bufs[k % 4][: int(n) * int(w)], int(n), int(w)) for k, (n, w) in enumerate(zip(rows, ws))]
        checked = 0
        for k, ((n, w), rid) in enumerate(zip(zip(rows, ws), ids)):
            n, w = int(n), int(w)
            info = srv.wait(rid)
            assert info["status"] == 0, k
            alone = goldi.goldi_merkle_build(bufs[k % 4][: n * w], n, w)
            assert torch.equal(srv.nodes(rid).view(torch.int64), alone.view(torch.int64)), k
            if k in golden_roots:
                assert [str(v) for v in info["root"]] == golden_roots[k], k
                checked += 1
            srv.release(rid)
        assert checked > 0
