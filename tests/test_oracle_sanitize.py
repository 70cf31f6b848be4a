"""The FP64 oracle built with gcc's AddressSanitizer, LeakSanitizer and
UndefinedBehaviorSanitizer and driven through every entry point by
tests/oracle_sanitize_driver.c (walls, a moving wall, a body converting cells
every step, a free squirmer, population round trip, a runaway body): the run
must exit cleanly with no sanitizer report.  Host code only."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def test_oracle_is_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_sanitized"
    build = ["gcc", "-O1", "-g", "-std=c11", "-D_GNU_SOURCE", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
             str(ROOT / "tests" / "oracle_sanitize_driver.c"), str(ROOT / "oracle" / "lbsq_oracle.c"),
             "-lm", "-o", str(exe)]
    b = subprocess.run(build, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr
    assert "conversions" in r.stdout, r.stdout
