"""The serving scheduler on the CPU: built with g++ (no HIP) against a fake
executor, under ThreadSanitizer and AddressSanitizer, and run. Covers
per-stream ordering, history reset, budget admission, queue-full,
resolution mismatch, close/destroy cancellation, injected device failures and
concurrent clients."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "tests", "serve_core_test.cpp"),
       os.path.join(ROOT, "paper_1609_05344_amd", "csrc", "serve_core.cpp")]


@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_scheduler_under_sanitizer(tmp_path, sanitizer):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path / "serve_core_test"
    cmd = [gxx, "-std=c++17", "-O1", "-g", f"-fsanitize={sanitizer}", "-fno-omit-frame-pointer",
           *SRC, "-o", str(exe), "-lpthread"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
