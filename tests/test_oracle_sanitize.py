"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc, host code only) runs every entry point on small ragged shapes without
a report: no out-of-bounds access, no bad shift, no leak."""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = tmp_path / "oracle_sanitized"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-pthread", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=all", os.path.join(ROOT, "oracle", "oracle.c"),
                           os.path.join(HERE, "oracle_sanitize_main.c"), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    assert "sanitized oracle ok" in r.stdout
