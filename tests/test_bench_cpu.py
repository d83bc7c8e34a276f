"""Host-side checks of bench.py that need no GPU: the work count, the
refusal of several GPUs, the spread statistics, and that committed counter
summaries are used only while they match the kernels' device sources (else
the bench reports null for them)."""

import json
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_work_count():
    # The optimised form of Alg. 1: full-width products are the S-boxes'
    # (8 full rounds x 12 + 22 partial) x 4, the pre-matrix's 11 x 11 and the
    # 22 sparse partial matrices' 12 + 11 each, at 4 limb products each; the
    # 8 full rounds' 12 x 12 small-entry matrices take 2 limb products per
    # entry.
    full = (8 * 12 + 22) * 4 + 11 * 11 + 22 * (12 + 11)
    assert full == 1099
    assert bench.MULADDS_PER_PERM == full * 4 + 8 * 144 * 2 == 6700
    # The textbook form: the dense matrix in all 30 rounds.
    assert bench.DENSE_MULADDS_PER_PERM == (8 * 12 + 22) * 4 * 4 + 30 * 144 * 2
    assert bench.perms_per_build(1 << 22, 8) == (1 << 23) - 1
    assert bench.perms_per_build(1 << 21, 256) == (1 << 21) * 32 + (1 << 21) - 1


class _Knobs:
    def __init__(self, **kw):
        self.v = dict(lane12_max_rows=1 << 13, quad_max_rows=1 << 14, lane12_max_parents=1 << 13,
                      quad_max_parents=1 << 16, top_max_parents=16)
        self.v.update(kw)

    def goldi_tune_get(self, k):
        return self.v[k]


def test_schedule_of_the_paper_scale_tree():
    perms, launches = bench.schedule(_Knobs(), 1 << 22, 8)
    assert sum(perms.values()) == bench.perms_per_build(1 << 22, 8)
    # levels of 2^13 .. 2^9 parents in one launch, then 2^8 .. 2^4, then 8 .. 1
    assert launches == {"leaf_hash": 1, "leaf_hash_quad": 0, "leaf_hash_lane12": 0, "level": 5,
                        "level_quad": 3, "levels_lane12": 2, "top_lane12": 1}
    assert perms["level"] == sum(1 << k for k in range(17, 22))
    assert perms["levels_lane12"] == sum(1 << k for k in range(4, 14))
    assert perms["top_lane12"] == 8 + 4 + 2 + 1


def test_schedule_ragged_and_tiny():
    for n in (1, 2, 3, 17, 1000, 4097, (1 << 20) + 3):
        for w in (1, 8, 9, 64):
            perms, launches = bench.schedule(_Knobs(), n, w)
            assert sum(perms.values()) == bench.perms_per_build(n, w)
            assert sum(launches.values()) >= 1
    perms, launches = bench.schedule(_Knobs(top_max_parents=0), 1000, 8)
    assert launches["top_lane12"] == 0 and perms["top_lane12"] == 0


def test_several_gpus_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_step_stats():
    st = bench.step_stats([3.0, 1.0, 2.0])
    assert st == {"builds": 3, "mean_ms": 2.0, "std_ms": 1.0, "min_ms": 1.0}


def test_profile_records_follow_the_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"k_leaf_hash/tree22": {"source_digest": bench.source_digest(), "hbm_bytes_per_launch": 123}}
    (prof / "traffic.json").write_text(json.dumps(rec))
    digest = bench.source_digest()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "source_digest", lambda: digest)
    assert bench.traffic_from_profiles("k_leaf_hash", "tree22") == 123
    assert bench.traffic_from_profiles("k_leaf_hash", "wide21") is None
    rec["k_leaf_hash/tree22"]["source_digest"] = "0" * 16
    (prof / "traffic.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profiles("k_leaf_hash", "tree22") is None


def test_function_instruction_counts_from_the_build():
    # The Table-1 instruction counts come from the library's own code object
    # (count_valu.py, run by the build): every function is counted, and the
    # parser takes the innermost loop of each chain kernel.
    from paper_2506_09505_amd import count_valu
    counts = count_valu.read()
    assert set(counts) == set(count_valu.OPS)
    assert all(v > 0 for v in counts.values())
    assert counts["sbox"] == 4 * counts["mult_128"]   # x^7 is four products
    text = "\n".join(["_ZN1x10k_fb_chainILi%dEEvv:" % op + "\n v_mov_b32 v0, 0\n.LBB0_1: ; =>This Inner Loop Header: Depth=1\n"
                      + " v_add_u32 v1, v1, v2\n" * (8 if op < 7 else 3) + " s_cbranch_scc1 .LBB0_1\n v_mov_b32 v3, 0\n s_endpgm"
                      for op in range(len(count_valu.OPS))])
    got = count_valu.counts_from_asm(text)
    assert got["add"] == 1 and got["mmult_12x12_full"] == 3
