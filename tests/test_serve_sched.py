"""The serving policy (queue, admission by slots and memory, chunks,
retirement, cancellation) run on the host against a fake backend:
tests/serve_sched_test.cpp, built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer.  The same policy drives the GPU server, whose own
tests are in test_gpu_serving.py."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


def test_serving_policy_with_a_fake_backend(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "serve_sched_test"
    build = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
             str(ROOT / "tests" / "serve_sched_test.cpp"), "-o", str(exe)]
    b = subprocess.run(build, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout, r.stdout
