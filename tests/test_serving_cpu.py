"""CPU checks of the serving loop's admission rule (no GPU needed): requests
are admitted in arrival order, as the longest prefix of the queue that fits
the HBM budget next to what is already admitted, at most max_group at once."""

import random

import paper_2506_09505_amd as goldi


def plan(*a):
    return goldi.goldi_admission_plan(*a)


def test_fifo_prefix_within_budget():
    assert plan([10, 20, 30], 100, 0, 8) == 3
    assert plan([10, 20, 30], 59, 0, 8) == 2
    assert plan([10, 20, 30], 30, 0, 8) == 2
    assert plan([10, 20, 30], 29, 0, 8) == 1


def test_no_overtaking_when_head_does_not_fit():
    # a small request behind a large one waits: arrival order is kept
    assert plan([90, 1, 1], 100, 20, 8) == 0


def test_group_limit_and_empty_queue():
    assert plan([1] * 10, 100, 0, 4) == 4
    assert plan([], 100, 0, 4) == 0


def test_inflight_counts_against_budget():
    assert plan([10, 10], 100, 85, 8) == 1
    assert plan([10], 100, 100, 8) == 0
    assert plan([10], 100, 150, 8) == 0   # over budget already (never admits more)


def test_randomised_against_definition():
    rnd = random.Random(5)
    for _ in range(2000):
        q = [rnd.randrange(1, 50) for _ in range(rnd.randrange(0, 12))]
        budget, used, g = rnd.randrange(1, 200), rnd.randrange(0, 220), rnd.randrange(1, 6)
        k = 0
        while k < len(q) and k < g and used + sum(q[:k + 1]) <= budget:
            k += 1
        assert plan(q, budget, used, g) == k
