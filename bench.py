#!/usr/bin/env python3
"""Benchmark of the Poseidon-12 / Goldilocks Merkle build on one MI355X.

One step = one whole Merkle build (leaf hashing with the Poseidon-12 sponge
+ the level-by-level 2-to-1 reduce to the root) of the paper's tree shape
(Sec. 4.2): 2^22 leaves x 8 Goldilocks words, uniform random (seed 1),
column-major, every node written.  Inputs are generated on the device before
the timed region; the timed region holds exactly ``--steps`` builds.

Printed: one JSON line with the headline (permutations per second over the
whole build), the build time, a roofline entry for the dominant kernel
(integer multiply-adds per second against the chip's 32-bit multiply-add
peak, from HIP events recorded on the launch stream during the timed region;
with the committed HBM counters, bytes per launch and the fraction of HBM
peak), the spread of single builds (an untimed pass with one event pair per
build), and the CPU oracle's rate on a bounded sample of the same workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Poseidon-12 perms/s + 2^22-leaf Merkle build ms; batched vs plain, bit-exact"

# Algorithmic work of one permutation, in 32x32->64-bit multiply-adds on
# 32-bit limbs, for the optimised form of the permutation that Alg. 1 (Sec.
# 2.4) describes -- sparse partial rounds after one pre-matrix:
#   full-width field products: 118 S-boxes x 4 products + the pre-matrix's
#     121 + 22 partial rounds x (12 + 11)                 = 1,099, x 4 = 4,396
#   small-entry matrix terms: 8 full rounds x 144 entries  = 1,152, x 2 = 2,304
# total 6,700 per permutation (reductions, carries and additions are not
# counted, the way a flop count leaves out index arithmetic).  This is the
# work of the method, not of the textbook form with the dense matrix in every
# round (DENSE_MULADDS_PER_PERM below, reported only as a labelled secondary
# figure).
MULADDS_PER_PERM = 1099 * 4 + 1152 * 2
OP_TEXT = ("32x32->64-bit multiply-add (v_mad_u64_u32), %d per permutation: the optimised form of Alg. 1 "
           "(1,099 full-width products x 4 limb products + 1,152 small matrix terms x 2)" % MULADDS_PER_PERM)
# The textbook form (dense 12x12 matrix in all 30 rounds):
#   S-boxes 118 x 4 x 4 = 1,888; matrix 30 x 144 x 2 = 8,640.
DENSE_MULADDS_PER_PERM = 1888 + 8640
# gfx950 peak of that operation: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one
# v_mad_u64_u32 per lane per cycle (one wave64 instruction per SIMD every 4
# cycles).  The measured rate of the instruction is in profiles/rates.json.
PEAK_MULADD_PER_S = 256 * 4 * 16 * 2.4e9
# MI355X HBM3E peak, bytes/s (to show how far below it the path runs).
PEAK_HBM_BYTES_PER_S = 8.0e12

WORKLOADS = {
    # name: (n_rows, n_cols, seed, description)
    "tree22": (1 << 22, 8, 1, "plain single tree: 2^22 leaves x 8 Goldilocks words, column-major, seed 1; "
                              "Poseidon-12 sponge leaves + binary 2-to-1 reduce, all 2^23-1 nodes written"),
    "tree10": (1 << 10, 8, 0, "plain single tree: 2^10 leaves x 8 Goldilocks words, column-major, seed 0"),
    "wide21": (1 << 21, 256, 2, "wide-row commitment tree: 2^21 rows x 256 Goldilocks words, column-major, "
                                "seed 2; 32 rate-8 chunks per row, binary reduce"),
    "serve": (None, None, 4, "served: Poisson stream, mean 200 requests/s, rows floor(2^U) with U uniform on "
                             "[12, 22], widths uniform in {8,32,64}, uniform Goldilocks words (seed 4), leaves in "
                             "pinned host memory, 64 GB HBM budget; continuous batching vs one request at a time"),
    "functions": (None, None, 0, "the paper's Table-1 basic functions on gfx950: dependent chains per lane, "
                                 "1M lanes, rate of each function"),
    "batch64": (None, None, 3, "batched: 64 trees, rows floor(2^U) with U uniform on [10, 20], widths uniform "
                               "in {8,16,32,64,128}, uniform Goldilocks words (seed 3); autotuned batched "
                               "schedule vs 64 plain single-tree launches"),
    "rates": (None, None, 0, "per-opcode issue rates of the gfx950 vector ALU for the field layer's integer "
                             "instructions (inline assembly, 8 waves per SIMD; one wave alone for latency)"),
}


def perms_per_build(n_rows: int, n_cols: int) -> int:
    return n_rows * ((n_cols + 7) // 8) + (n_rows - 1)


# The device code of the build kernels (their bodies, block size and
# constants); host-side files do not change what a kernel reads or writes.
DEVICE_SOURCES = ("field.hpp", "field_asm.inc", "poseidon.hpp", "poseidon_quad.hpp", "poseidon_lane12.hpp",
                  "kernels.hpp", "poseidon12_constants.inc")


def source_digest() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2506_09505_amd", "csrc")
    for name in DEVICE_SOURCES:
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def profile_record(name: str, kernel: str, workload: str):
    """A committed rocprofv3 counter summary (profiles/<name>) for one kernel
    and workload, if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", name)
    try:
        with open(path) as f:
            rec = json.load(f).get("%s/%s" % (kernel, workload))
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_digest") != source_digest():
        return None
    return rec


def traffic_from_profiles(kernel: str, workload: str):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, scaled), or None."""
    rec = profile_record("traffic.json", kernel, workload)
    return rec.get("hbm_bytes_per_launch") if rec else None


def host_cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def step_stats(samples_ms):
    """Mean, standard deviation and minimum of per-build times (ms)."""
    n = len(samples_ms)
    mean = sum(samples_ms) / n
    var = sum((x - mean) ** 2 for x in samples_ms) / max(1, n - 1)
    return {"builds": n, "mean_ms": round(mean, 4), "std_ms": round(var ** 0.5, 4), "min_ms": round(min(samples_ms), 4)}


def cpu_baseline(n_rows: int, n_cols: int, seed: int):
    """The oracle (plain textbook C, all host threads) on a bounded sample:
    a 2^18-leaf tree of the same leaf shape (524,287 permutations)."""
    import oracle
    from synth.inputs import leaves_colmajor
    n = 1 << 18
    lv = leaves_colmajor(n, n_cols, seed=seed)
    prm = oracle.spec_params()
    threads = oracle.default_threads()
    oracle.lib()
    t0 = time.perf_counter()
    nodes = oracle.merkle_build(prm, lv, n, n_cols, threads=threads)
    dt = time.perf_counter() - t0
    perms = perms_per_build(n, n_cols)
    # The same oracle on one thread, over a smaller tree of the same shape.
    n1 = 1 << 15
    lv1 = leaves_colmajor(n1, n_cols, seed=seed)
    t1 = time.perf_counter()
    oracle.merkle_build(prm, lv1, n1, n_cols, threads=1)
    dt1 = time.perf_counter() - t1
    return {"value": perms / dt, "unit": "perms/s", "cores": threads, "kind": "oracle",
            "host_cpu": host_cpu_model(), "host_logical_cpus": os.cpu_count(),
            "sample": "one 2^18-leaf x %d-word tree (seed %d, %d permutations) built by the oracle "
                      "in %.2f s" % (n_cols, seed, perms, dt),
            "single_thread_value": perms_per_build(n1, n_cols) / dt1,
            "single_thread_sample": "one 2^15-leaf x %d-word tree on one thread in %.2f s" % (n_cols, dt1)}, \
        (lv, nodes, n)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="tree22", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", default=None,
                    help="measure a test build of the library (paper_2506_09505_amd/_special/libgoldi_<NAME>.so, "
                         "e.g. limb24, sparse, dense) instead of the default one")
    ap.add_argument("--split-parts", type=int, default=None,
                    help="single-tree builds: ranges of rows run on separate streams (library default when unset; "
                         "0 = one stream)")
    ap.add_argument("--no-extras", action="store_true",
                    help="tree22: skip the batched-vs-plain and 2^24-state permutation records")
    ap.add_argument("--requests", type=int, default=1000, help="serve: measured requests (after 100 warm-up)")
    ap.add_argument("--serve-input", default="host", choices=("host", "device"),
                    help="serve: leaves in pinned host memory (copied in by the server) or already in HBM")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device-to-device copy three times (HBM counter "
                         "calibration for rocprofv3 FETCH_SIZE / WRITE_SIZE) and exit")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.calibrate_copy:
        src = torch.ones(1 << 27, dtype=torch.int64, device="cuda:0")   # 1 GiB
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": 1 << 30, "bytes_written": 1 << 30,
                          "launches": 3}), flush=True)
        return 0

    import paper_2506_09505_amd as goldi
    if args.variant:
        from paper_2506_09505_amd import build as pkg_build
        goldi.LIB_PATH = pkg_build.special_lib(args.variant)

    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    if args.workload == "functions":
        return bench_functions(args)
    if args.workload == "rates":
        return bench_rates(args)
    return bench_tree(args, goldi, np, torch)


KINDS = ("leaf_hash", "leaf_hash_quad", "leaf_hash_lane12", "level", "level_quad", "levels_lane12", "top_lane12")
LEVELS_PER_LAUNCH = 5  # one-word-per-lane launches below the top: up to five levels each


def schedule(goldi, n_rows: int, n_cols: int):
    """Permutations and launches per kernel kind of one build on one stream,
    following the library's schedule knobs (an unpaired last node is moved,
    not hashed)."""
    t = {k: goldi.goldi_tune_get(k) for k in ("lane12_max_rows", "quad_max_rows", "lane12_max_parents",
                                               "quad_max_parents", "top_max_parents")}
    perms = dict.fromkeys(KINDS, 0)
    launches = dict.fromkeys(KINDS, 0)
    leaf = ("leaf_hash_lane12" if n_rows <= t["lane12_max_rows"] else
            "leaf_hash_quad" if n_rows <= t["quad_max_rows"] else "leaf_hash")
    perms[leaf] += n_rows * ((n_cols + 7) // 8)
    launches[leaf] += 1
    n = n_rows
    while n > 1:
        par = (n + 1) // 2
        if par <= t["top_max_parents"]:
            kind, levels = "top_lane12", 64
        elif par <= t["lane12_max_parents"]:
            kind, levels = "levels_lane12", LEVELS_PER_LAUNCH
        else:
            kind, levels = ("level_quad" if par <= t["quad_max_parents"] else "level"), 1
        launches[kind] += 1
        for _ in range(levels):
            if n == 1:
                break
            perms[kind] += n // 2
            n = (n + 1) // 2
    return perms, launches


def measured_mad_rate():
    """Throughput of v_mad_u64_u32 as a fraction of the full rate, from the
    committed rate-probe summary, or None."""
    try:
        with open(os.path.join(ROOT, "profiles", "rates.json")) as f:
            return json.load(f)["rates"]["v_mad_u64_u32"]["throughput_frac_of_full_rate"]
    except (OSError, ValueError, KeyError):
        return None


def golden_record(key: str):
    """The oracle's per-level digests and root for a workload, as recorded by
    tests/golden/make_golden.py (which calls only the oracle), or None."""
    try:
        with open(os.path.join(ROOT, "tests", "golden", "fullsize.json")) as f:
            return json.load(f).get(key)
    except (OSError, ValueError):
        return None


def root_words(nodes_dev, torch, np):
    return [str(int(v)) for v in nodes_dev.view(-1, 4)[-1].view(torch.int64).cpu().numpy().view(np.uint64)]


def bench_tree(args, goldi, np, torch) -> int:
    from synth import fill
    n_rows, n_cols, seed, desc = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    leaves = fill.leaves_colmajor_dev(n_rows, n_cols, seed=seed, device=dev)
    nodes = torch.empty(goldi.goldi_merkle_num_nodes(n_rows) * 4, dtype=torch.uint64, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    perms = perms_per_build(n_rows, n_cols)
    sched_perms, sched_launches = schedule(goldi, n_rows, n_cols)
    assert sum(sched_perms.values()) == perms

    def build():
        goldi.goldi_merkle_build_async(leaves, n_rows, n_cols, nodes, status, stream)

    if args.split_parts is not None:
        goldi.goldi_tune_set("split_parts", args.split_parts)
    split_parts = goldi.goldi_tune_get("split_parts")
    for _ in range(args.warmup):
        build()
    torch.cuda.synchronize()

    def timed_builds():
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ev0.record(stream)
        for _ in range(args.steps):
            build()
        ev1.record(stream)
        torch.cuda.synchronize()
        return ev0.elapsed_time(ev1) / args.steps, (time.perf_counter() - t0) * 1e3 / args.steps

    # Kernel figures come from builds on one stream: a split build runs two
    # launches side by side on two streams, so an event span there would
    # include the other stream's work and is no launch duration.
    goldi.goldi_tune_set("split_parts", 0)
    # Untimed breakdown pass: every kernel bracketed (adds a few us per
    # launch); it names the dominant kernel kind, the one with the most time
    # per build.
    goldi.goldi_profile_select(None)
    goldi.goldi_profile_enable(True)
    for _ in range(3):
        build()
    torch.cuda.synchronize()
    goldi.goldi_profile_enable(False)
    breakdown = {k: goldi.goldi_profile_read(k) for k in KINDS}
    dominant = max(KINDS, key=lambda k: breakdown[k][0])

    # Kernel timed region: exactly `steps` one-stream builds; the library
    # brackets each run of launches of the dominant kernel kind with HIP
    # events on the launch stream, the other kernels run unbracketed.
    goldi.goldi_profile_select(dominant)
    goldi.goldi_profile_enable(True)
    ms_one_stream, _ = timed_builds()
    goldi.goldi_profile_enable(False)
    goldi.goldi_profile_select(None)
    dom_ms, dom_launches = goldi.goldi_profile_read(dominant)

    # Build timed region (the headline): exactly `steps` builds as the
    # library runs them by default (split when the tree is large enough), no
    # per-kernel events.
    goldi.goldi_tune_set("split_parts", split_parts)
    for _ in range(2):
        build()
    ms_per_step, wall_ms_per_step = timed_builds()

    # Untimed pass for the spread: one event pair around each build.
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        build()
        b.record(stream)
    torch.cuda.synchronize()
    per_build = step_stats([a.elapsed_time(b) for a, b in evs])
    if int(status.item()) != 0:
        print("device status %d: non-canonical input" % int(status.item()), file=sys.stderr)
        return 1

    # Roofline of the dominant kind: its algorithmic multiply-adds per launch
    # over its average launch duration, both from the kernel timed region.
    mad_frac = measured_mad_rate()

    def fracs(work_per_s):
        f = {"frac": round(work_per_s / PEAK_MULADD_PER_S, 4)}
        if mad_frac:
            f["frac_of_measured_mad_rate"] = round(work_per_s / (PEAK_MULADD_PER_S * mad_frac), 4)
        return f

    runs = max(1, args.steps)
    dom_launch_ms = dom_ms / max(1, dom_launches)
    dom_perms_per_launch = sched_perms[dominant] / max(1, sched_launches[dominant])
    achieved = dom_perms_per_launch * MULADDS_PER_PERM / (dom_launch_ms * 1e-3)
    roofline = {"bound": "alu", "kernel": "k_" + dominant,
                "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_MULADD_PER_S / 1e12, 3),
                "unit": "Tops/s"}
    roofline.update(fracs(achieved))
    roofline.update({
        "op": OP_TEXT,
        "kernel_ms_per_launch": round(dom_launch_ms, 4),
        "kernel_timing": "HIP events around the launches on their stream, in %d one-stream builds (the build "
                         "timed region runs the default schedule)" % args.steps,
        "launches_per_build": round(dom_launches / runs, 2),
        "perms_per_launch": dom_perms_per_launch,
        "traffic": traffic_from_profiles("k_" + dominant, args.workload)})
    # Every kernel kind and the whole build on the same scale (the kinds from
    # the untimed one-stream breakdown pass, the build from the build timed
    # region).
    per_kind = {}
    for k in KINDS:
        ms_k = breakdown[k][0] / 3
        if breakdown[k][1] and sched_perms[k]:
            rate = sched_perms[k] * MULADDS_PER_PERM / (ms_k * 1e-3)
            per_kind["k_" + k] = dict(ms_per_build=round(ms_k, 4), perms_per_build=sched_perms[k],
                                      launches_per_build=breakdown[k][1] // 3, **fracs(rate))
    whole = perms * MULADDS_PER_PERM / (ms_per_step * 1e-3)
    roofline["per_kernel"] = per_kind
    roofline["whole_build"] = dict(achieved=round(whole / 1e12, 3), **fracs(whole))
    roofline["dense_equivalent"] = {
        "note": "the same times counted with the textbook form's %d multiply-adds per permutation (dense matrix "
                "in every round), which the kernels do not execute" % DENSE_MULADDS_PER_PERM,
        "kernel_frac": round(dom_perms_per_launch * DENSE_MULADDS_PER_PERM / (dom_launch_ms * 1e-3)
                             / PEAK_MULADD_PER_S, 4),
        "whole_build_frac": round(perms * DENSE_MULADDS_PER_PERM / (ms_per_step * 1e-3) / PEAK_MULADD_PER_S, 4)}
    if mad_frac:
        roofline["measured_mad_rate"] = {"frac_of_full_rate": mad_frac, "source": "profiles/rates.json"}
    valu = profile_record("valu.json", "k_" + dominant, args.workload)
    if valu and dominant in ("leaf_hash", "level"):
        # One state per lane: a wave runs 64 permutations.  Issued VALU
        # instructions per SIMD per cycle at 2.4 GHz (0.25 = one wave64
        # instruction every 4 cycles; some 32-bit instructions issue faster).
        per_perm = valu["valu_instructions_per_permutation"]
        rate = dom_perms_per_launch / 64 * per_perm / (dom_launch_ms * 1e-3)
        roofline["valu_issue"] = {"instructions_per_permutation": per_perm,
                                  "instructions_per_simd_per_cycle": round(rate / (256 * 4 * 2.4e9), 4),
                                  "source": "profiles/valu.json (SQ_INSTS_VALU / SQ_WAVES) with the live kernel time"}
    if roofline["traffic"]:
        hbm = roofline["traffic"] / (dom_launch_ms * 1e-3)
        roofline["hbm_gb_per_s"] = round(hbm / 1e9, 1)
        roofline["hbm_frac"] = round(hbm / PEAK_HBM_BYTES_PER_S, 4)

    config = {"workload": desc, "n_rows": n_rows, "n_cols": n_cols, "seed": seed, "library": os.path.basename(goldi.LIB_PATH),
              "perms_per_step": perms, "build_ms": round(ms_per_step, 4),
              "wall_ms_per_step": round(wall_ms_per_step, 4),
              "split_parts": split_parts,
              "build_ms_one_stream": round(ms_one_stream, 4),
              "build_ms_each": per_build,
              "breakdown_ms_per_build": {k: round(v[0] / 3, 4) for k, v in breakdown.items()},
              "breakdown_launches_per_build": {k: v[1] // 3 for k, v in breakdown.items()}}
    gold = golden_record(args.workload)
    if gold:
        config["root_equals_oracle"] = root_words(nodes, torch, np) == gold["root"]
    out = {
        "metric": METRIC,
        "value": perms / (ms_per_step * 1e-3),
        "unit": "perms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": config,
        "roofline": roofline,
    }
    del leaves, nodes
    torch.cuda.empty_cache()
    if args.workload == "tree22" and not args.no_extras:
        out["batched"] = batched_vs_plain(args, goldi, np, torch)
        out["permute"] = permute_rate(args, goldi, torch)
    if not args.no_cpu_baseline:
        base, (lv, want, n_s) = cpu_baseline(n_rows, n_cols, seed)
        # The same sample on the GPU must agree word for word.
        got = goldi.goldi_merkle_build(torch.from_numpy(lv.view(np.int64)).to(dev).view(torch.uint64), n_s, n_cols)
        base["bit_exact_vs_gpu"] = bool((got.view(torch.int64).cpu().numpy().view(np.uint64).reshape(-1, 4)
                                         == want).all())
        out["cpu_baseline"] = base
    print(json.dumps(out), flush=True)
    return 0


def batched_vs_plain(args, goldi, np, torch):
    """The batched workload (64 uneven trees, seed 3) built by one
    goldi_merkle_build_many call under the default schedule, against the same
    64 trees built one after another with the plain single-tree kernels; both
    outputs compared word for word, and the 64 roots with the oracle's."""
    from synth import fill
    from synth.inputs import tree_shapes
    dev = torch.device("cuda:0")
    rows, ws = tree_shapes(3, 64, 10, 20, (8, 16, 32, 64, 128))
    trees = [(fill.leaves_colmajor_dev(int(n), int(w), seed=3, stream=k, device=dev), int(n), int(w))
             for k, (n, w) in enumerate(zip(rows, ws))]
    outs = [torch.empty(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device=dev) for _, n, _ in trees]
    plain = [torch.empty_like(o) for o in outs]
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    perms = sum(perms_per_build(n, w) for _, n, w in trees)
    steps = max(3, args.steps // 4)

    def timed(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def run_plain():
        for (lv, n, w), o in zip(trees, plain):
            goldi.goldi_merkle_build_async(lv, n, w, o, status, stream)

    def run_many():
        goldi.goldi_merkle_build_many_async(trees, outs, status, stream)

    plain_ms = timed(run_plain)
    many_ms = timed(run_many)
    exact = all(torch.equal(a.view(torch.int64), b.view(torch.int64)) for a, b in zip(outs, plain))
    rec = {"workload": WORKLOADS["batch64"][3].replace("autotuned batched schedule", "default batched schedule"),
           "trees": 64, "perms": perms, "plain_64_builds_ms": round(plain_ms, 4), "batched_ms": round(many_ms, 4),
           "speedup_vs_plain": round(plain_ms / many_ms, 3), "batched_perms_per_s": perms / (many_ms * 1e-3),
           "trees_per_s": 64 / (many_ms * 1e-3), "bit_exact_vs_plain": bool(exact),
           "status_ok": int(status.item()) == 0, "steps": steps}
    gold = golden_record("batch64")
    if gold:
        rec["roots_equal_oracle"] = all(root_words(o, torch, np) == t["root"] for o, t in zip(outs, gold["trees"]))
    del trees, outs, plain
    torch.cuda.empty_cache()
    return rec


def permute_rate(args, goldi, torch):
    """goldi_poseidon_permute on 2^24 uniform states (1.5 GiB), in place."""
    from synth import fill
    n = 1 << 24
    dev = torch.device("cuda:0")
    states = torch.empty(n * 12, dtype=torch.uint64, device=dev)
    fill.fill_words(states, 8, 1)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    steps = max(3, args.steps // 4)
    goldi.goldi_poseidon_permute_async(states, status, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(steps):
        goldi.goldi_poseidon_permute_async(states, status, stream)
    b.record(stream)
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    rate = n / (ms * 1e-3)
    del states
    torch.cuda.empty_cache()
    return {"states": n, "ms": round(ms, 4), "perms_per_s": rate, "status_ok": int(status.item()) == 0,
            "frac": round(rate * MULADDS_PER_PERM / PEAK_MULADD_PER_S, 4), "steps": steps}


def bench_rates(args) -> int:
    import torch

    from paper_2506_09505_amd import fieldbench
    torch.cuda.set_device(0)
    t0 = time.perf_counter()
    rows = fieldbench.rates()
    out = {"metric": "gfx950 VALU issue rate per opcode", "value": rows["v_mad_u64_u32"]["throughput_frac_of_full_rate"],
           "unit": "fraction of one wave64 instruction per SIMD per 4 cycles at 2.4 GHz (v_mad_u64_u32)",
           "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": (time.perf_counter() - t0) * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
           "config": {"workload": WORKLOADS["rates"][3]}, "rates": rows}
    print(json.dumps(out), flush=True)
    return 0


def bench_batch(args) -> int:
    """64 trees of uneven shapes: plain (one build after another) vs the
    batched many-tree build under the autotuned schedule; bit-exact check."""
    import torch

    import paper_2506_09505_amd as goldi
    from paper_2506_09505_amd import autotune
    from synth import fill
    from synth.inputs import tree_shapes

    _, _, seed, desc = WORKLOADS["batch64"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rows, ws = tree_shapes(seed, 64, 10, 20, (8, 16, 32, 64, 128))
    trees = [(fill.leaves_colmajor_dev(int(n), int(w), seed=seed, stream=k, device=dev), int(n), int(w))
             for k, (n, w) in enumerate(zip(rows, ws))]
    outs = [torch.empty(goldi.goldi_merkle_num_nodes(n) * 4, dtype=torch.uint64, device=dev) for _, n, _ in trees]
    plain = [torch.empty_like(o) for o in outs]
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream()
    perms = sum(perms_per_build(n, w) for _, n, w in trees)
    leaf_perms = sum(n * ((w + 7) // 8) for _, n, w in trees)

    def timed(fn, steps):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    def run_plain():
        for (lv, n, w), o in zip(trees, plain):
            goldi.goldi_merkle_build_async(lv, n, w, o, status, stream)

    def run_many():
        goldi.goldi_merkle_build_many_async(trees, outs, status, stream)

    saved = autotune.current()
    goldi.goldi_tune_set("batch_mode", 0)
    goldi.goldi_tune_set("graph", 0)
    plain_ms = timed(run_plain, max(2, args.steps // 4))
    autotune.apply(saved)
    default_ms = timed(run_many, max(2, args.steps // 4))
    cfg, _, _ = autotune.tune(trees, outs, status, cache_path=None)
    goldi.goldi_profile_select("leaf_hash")
    goldi.goldi_profile_enable(True)
    ms = timed(run_many, args.steps)
    goldi.goldi_profile_enable(False)
    leaf_tot, leaf_cnt = goldi.goldi_profile_read("leaf_hash")
    leaf_note = "timed inside the measured builds"
    if leaf_cnt == 0:
        # A replayed hipGraph records no per-kernel events: time the dominant
        # kernel in the same schedule launched directly.
        goldi.goldi_tune_set("graph", 0)
        goldi.goldi_profile_enable(True)
        timed(run_many, max(2, args.steps // 2))
        goldi.goldi_profile_enable(False)
        leaf_tot, leaf_cnt = goldi.goldi_profile_read("leaf_hash")
        leaf_note = "tuned schedule replays a hipGraph; kernel timed in the same schedule launched directly"
    goldi.goldi_profile_select(None)
    exact = all(torch.equal(a.view(torch.int64), b.view(torch.int64)) for a, b in zip(outs, plain))
    autotune.apply(saved)
    if int(status.item()) != 0:
        print("device status %d" % int(status.item()), file=sys.stderr)
        return 1
    leaf_ms = leaf_tot / max(1, leaf_cnt)
    achieved = leaf_perms * MULADDS_PER_PERM / (leaf_ms * 1e-3)
    out = {
        "metric": METRIC, "value": perms / (ms * 1e-3), "unit": "perms/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": desc, "trees": 64, "rows_total": int(rows.sum()), "perms_per_step": perms,
                   "trees_per_s": 64 / (ms * 1e-3), "plain_64_launches_ms": round(plain_ms, 4),
                   "batched_default_ms": round(default_ms, 4), "batched_tuned_ms": round(ms, 4),
                   "speedup_vs_plain": round(plain_ms / ms, 3), "tuned_schedule": cfg,
                   "bit_exact_vs_plain": bool(exact)},
        "roofline": {"bound": "alu", "kernel": "k_leaf_hash_batch",
                     "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_MULADD_PER_S / 1e12, 3),
                     "unit": "Tops/s", "frac": round(achieved / PEAK_MULADD_PER_S, 4),
                     "op": OP_TEXT,
                     "kernel_ms": round(leaf_ms, 4), "kernel_timing": leaf_note, "traffic": None},
    }
    print(json.dumps(out), flush=True)
    return 0 if exact else 1


def serve_run(srv_args, shapes, arrivals, bufs, warm):
    """Submits every request at its arrival time; a waiter thread collects
    results and releases them.  Returns per-request records."""
    import threading

    import paper_2506_09505_amd as goldi

    out = [None] * len(shapes)
    with goldi.GoldiServer(*srv_args) as srv:
        ids = [None] * len(shapes)
        ready = threading.Semaphore(0)

        def waiter():
            for k in range(len(shapes)):
                ready.acquire()
                info = srv.wait(ids[k])
                srv.release(ids[k])
                out[k] = info

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.monotonic()
        for k, ((n, w), t_arr) in enumerate(zip(shapes, arrivals)):
            delay = t0 + t_arr - time.monotonic()
            if delay > 0:
                time.sleep(delay)
            ids[k] = srv.submit(bufs[k % len(bufs)][: n * w], n, w)
            ready.release()
        th.join()
        stats = srv.stats()
    return out, stats


# VALU instructions per call of each function in the timed loops, counted
# from this repository's own gfx950 code object (hipcc -S of fieldbench.hip).
def bench_functions(args) -> int:
    import torch

    from paper_2506_09505_amd import count_valu, fieldbench
    torch.cuda.set_device(0)
    valu = count_valu.read()  # written at build time from the library's own code object
    rows = {}
    for name in fieldbench.OPS:
        iters = 8 if name == "mmult_12x12_full" else 64
        rate, ms = fieldbench.throughput(name, threads=256 * 4096, iters=iters)
        instr = valu[name]
        rows[name] = {"ops_per_s": rate, "kernel_ms": round(ms, 4), "valu_per_op": instr,
                      "valu_instr_per_s_per_lane_slot": rate * instr / PEAK_MULADD_PER_S}
    out = {"metric": "Table-1 basic functions on gfx950 (ops/s)", "value": rows["mult_128"]["ops_per_s"],
           "unit": "mult_128/s", "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": rows["mult_128"]["kernel_ms"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
           "config": {"workload": WORKLOADS["functions"][3], "functions": rows}}
    print(json.dumps(out), flush=True)
    return 0


def bench_serve(args) -> int:
    import numpy as np
    import torch

    import paper_2506_09505_amd as goldi
    from synth import fill
    from synth.inputs import poisson_arrivals, tree_shapes

    _, _, seed, desc = WORKLOADS["serve"]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    warm, total = 100, 100 + args.requests
    rows, ws = tree_shapes(seed, total, 12, 22, (8, 32, 64))
    arrivals = poisson_arrivals(seed, total, 200.0)
    shapes = [(int(n), int(w)) for n, w in zip(rows, ws)]
    words = max(n * w for n, w in shapes)
    # Four distinct pinned host matrices; request k reads the first n*w words
    # of matrix k mod 4 as its column-major leaves.
    bufs = []
    for b in range(4):
        d = torch.empty(words, dtype=torch.uint64, device=dev)
        fill.fill_words(d, seed, 100 + b)
        if args.serve_input == "device":
            bufs.append(d)
            continue
        h = torch.empty(words, dtype=torch.int64, pin_memory=True)
        h.copy_(d.view(torch.int64))
        bufs.append(h.view(torch.uint64))
        del d
    torch.cuda.synchronize()
    budget = 64 * 10**9
    runs = {}
    for name, srv_args in (("continuous", (budget, 8, 8)), ("one_at_a_time", (budget, 1, 1))):
        recs, stats = serve_run(srv_args, shapes, arrivals, bufs, warm)
        m = recs[warm:]
        lat = np.array([(r["t_done_ns"] - r["t_submit_ns"]) / 1e6 for r in m])
        wait = np.array([(r["t_admit_ns"] - r["t_submit_ns"]) / 1e6 for r in m])
        span = (max(r["t_done_ns"] for r in m) - min(r["t_submit_ns"] for r in m)) / 1e9
        perms = sum(perms_per_build(n, w) for n, w in shapes[warm:])
        runs[name] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                      "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                      "admission_wait_p99_ms": float(np.percentile(wait, 99)),
                      "trees_per_s": len(m) / span, "perms_per_s": perms / span,
                      "statuses_ok": all(r["status"] == 0 for r in recs),
                      "batches": stats["groups"], "requests": stats["admitted"],
                      "peak_admitted_bytes": stats["peak_bytes"], "roots": [r["root"] for r in recs]}
    # Every served root must equal the same build done alone, and the roots
    # the oracle recorded for a stratified sample of this request stream
    # (every request of at most 2^16 rows and 8 larger ones) must match.
    exact = True
    for k, (n, w) in enumerate(shapes):
        lv = bufs[k % 4][: n * w].to(dev)
        alone = goldi.goldi_merkle_build(lv, n, w)[-1].view(torch.int64).cpu().numpy().view(np.uint64)
        a = [int(v) for v in alone]
        exact &= runs["continuous"]["roots"][k] == a and runs["one_at_a_time"]["roots"][k] == a
    gold = golden_record("serve") or {"requests": []}
    sample = [q for q in gold["requests"] if q["request"] < len(shapes)]
    oracle_ok = all([str(v) for v in runs["continuous"]["roots"][q["request"]]] == q["root"] and
                    [str(v) for v in runs["one_at_a_time"]["roots"][q["request"]]] == q["root"] for q in sample)
    for r in runs.values():
        del r["roots"]
    c = runs["continuous"]
    offered = sum(perms_per_build(n, w) for n, w in shapes[warm:]) / (arrivals[-1] - arrivals[warm])
    out = {
        "metric": METRIC, "value": c["perms_per_s"], "unit": "perms/s", "n_gpus": 1, "steps": args.requests,
        "warmup": warm, "ms_per_step": c["mean_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": desc if args.serve_input == "host" else
                   desc.replace("leaves in pinned host memory", "leaves already in HBM"),
                   "requests_measured": args.requests, "offered_perms_per_s": offered,
                   "offered_requests_per_s": 200.0, "hbm_budget_bytes": budget,
                   "continuous_batching": runs["continuous"], "one_at_a_time": runs["one_at_a_time"],
                   "bit_exact_roots_vs_alone": bool(exact),
                   "bit_exact_roots_vs_oracle_sample": bool(oracle_ok) if sample else None,
                   "oracle_sample_requests": len(sample)},
    }
    print(json.dumps(out), flush=True)
    return 0 if exact and (oracle_ok or not sample) and c["statuses_ok"] else 1


if __name__ == "__main__":
    sys.exit(main())
