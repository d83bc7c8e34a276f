"""Autotuner for batched Merkle builds.

Every schedule knob of the library (``goldi_tune_set``) changes speed, never
results.  For a batch of trees this module times a small grid of schedules
with the real kernels on the real inputs and keeps the fastest:

* ``batch_mode``: one launch per level across all trees, or tree after tree;
* ``graph``: replay a captured hipGraph of the launch sequence, or launch
  directly;
* ``quad_max_rows`` / ``quad_max_parents`` and ``lane12_max_rows`` /
  ``lane12_max_parents``: where leaf hashing and tree levels switch from one
  lane per state (throughput) to four lanes, then one word per lane (latency).

Results are cached per *shape signature* -- the sorted multiset of
(row-count octave, chunks per row) of the batch -- in a JSON file, so batches
of the same shape class reuse the choice without re-timing.
"""

from __future__ import annotations

import itertools
import json
import math
import os
import threading

from . import goldi_merkle_build_many_async, goldi_tune_get, goldi_tune_set

KNOBS = ("batch_mode", "graph", "quad_max_rows", "quad_max_parents", "lane12_max_rows", "lane12_max_parents")
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "goldi_autotune.json")

_lock = threading.Lock()


def signature(shapes) -> str:
    """Shape class of a batch: sorted (floor(log2 rows), ceil(cols / 8)) pairs."""
    keys = sorted((int(math.log2(max(1, n))), (w + 7) // 8) for n, w in shapes)
    return ";".join("%d:%d" % k for k in keys)


def candidates():
    for bm, gr in ((0, 0), (1, 0), (1, 1)):
        for qr, qp in itertools.product((1 << 14, 1 << 16), (1 << 16, 1 << 17)):
            for l12_rows, l12_par in ((1 << 10, 1 << 10), (1 << 12, 1 << 12), (1 << 13, 1 << 13)):
                yield {"batch_mode": bm, "graph": gr, "quad_max_rows": qr, "quad_max_parents": qp,
                       "lane12_max_rows": l12_rows, "lane12_max_parents": l12_par}


def current():
    return {k: goldi_tune_get(k) for k in KNOBS}


def apply(cfg) -> None:
    for k, v in cfg.items():
        goldi_tune_set(k, int(v))


def _time_cfg(cfg, trees, outs, status, reps: int) -> float:
    import torch
    apply(cfg)
    goldi_merkle_build_many_async(trees, outs, status)      # warm-up (and graph capture)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        goldi_merkle_build_many_async(trees, outs, status)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def tune(trees, outs, status, reps: int = 2, cache_path: str | None = DEFAULT_CACHE, force: bool = False):
    """Pick the fastest schedule for ``trees`` (list of (leaves, n_rows, n_cols))
    writing into ``outs``; applies it and returns ``(cfg, ms, table)``."""
    sig = signature([(n, w) for _, n, w in trees])
    with _lock:
        cache = {}
        if cache_path and os.path.exists(cache_path):
            try:
                with open(cache_path) as f:
                    cache = json.load(f)
            except (OSError, ValueError):
                cache = {}
        if not force and sig in cache:
            apply(cache[sig]["cfg"])
            return cache[sig]["cfg"], cache[sig]["ms"], None
        saved = current()
        table = []
        try:
            for cfg in candidates():
                table.append((_time_cfg(cfg, trees, outs, status, reps), cfg))
        finally:
            apply(saved)
        ms, best = min(table, key=lambda t: t[0])
        apply(best)
        if cache_path:
            cache[sig] = {"cfg": best, "ms": ms}
            os.makedirs(os.path.dirname(cache_path), exist_ok=True)
            tmp = cache_path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(cache, f, indent=1)
            os.replace(tmp, cache_path)
        return best, ms, table
