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


def test_textbook_work_count():
    # (8 full rounds x 12 + 22 partial) S-boxes x 4 products x 4 limb
    # products, plus 30 dense 12 x 12 matrices x 2 limbs.
    assert bench.MULADDS_PER_PERM == (8 * 12 + 22) * 4 * 4 + 30 * 144 * 2
    assert bench.perms_per_build(1 << 22, 8) == (1 << 23) - 1
    assert bench.perms_per_build(1 << 21, 256) == (1 << 21) * 32 + (1 << 21) - 1


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
