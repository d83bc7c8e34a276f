"""GPU: the serving loop.  Each served result must equal the same build done
alone (goldi_merkle_build) and the oracle, whatever else was in the mix;
admission must respect the HBM budget; a bad request fails alone."""

import random
import time

import numpy as np
import pytest

import oracle
import paper_2506_09505_amd as goldi
from synth.inputs import GOLDILOCKS_P, leaves_colmajor, tree_shapes

from .gpu_util import to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def prm():
    return oracle.spec_params()


def banner(msg):
    print("[case] " + msg, flush=True)


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
    banner("serving with one non-canonical request")
    reqs = make_requests(23, 6, 6, 9, (8,))
    bad_lv = leaves_colmajor(100, 8, seed=1)
    bad_lv[17] = np.uint64(GOLDILOCKS_P)
    with goldi.GoldiServer(256 << 20, n_slots=1, max_group=8) as srv:
        # one slot: everything queued behind the bad request
        ids = [srv.submit(to_dev(bad_lv), 100, 8)] + [srv.submit(src, n, w) for n, w, _, src in reqs]
        assert srv.wait(ids[0])["status"] == goldi.GOLDI_ENONCANON
        for (n, w, lv, _), rid in zip(reqs, ids[1:]):
            info = srv.wait(rid)
            # a request built in the same batch as the bad one shares its status word
            if info["status"] == 0:
                assert (to_host(srv.nodes(rid)).reshape(-1, 4) == oracle.merkle_build(prm, lv, n, w)).all()
            else:
                assert info["status"] == goldi.GOLDI_ENONCANON
