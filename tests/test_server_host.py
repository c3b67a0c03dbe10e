"""Scheduling logic of the native request server, built for the host against a HIP stand-in and a
reference table (tests/native), run plainly, under ThreadSanitizer, and under AddressSanitizer with
UndefinedBehaviorSanitizer: results equal a sequential
replay in submission order, caps hold, every ticket completes once, nothing leaks."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "native", "server_host_test.cpp")


def _build_and_run(tmp_path, extra):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "server_host_test")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-pthread",
           "-I", os.path.join(HERE, "native", "mock_hip"), "-I", os.path.join(ROOT, "include"),
           SRC, "-o", exe] + extra
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and extra:
        pytest.skip(f"sanitizer build unavailable: {b.stderr[-300:]}")
    assert b.returncode == 0, b.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "server host test passed" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr, r.stderr[-2000:]


def test_server_scheduling_on_host(tmp_path):
    _build_and_run(tmp_path, [])


def test_server_scheduling_under_thread_sanitizer(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"])


def test_server_scheduling_under_address_and_undefined_sanitizers(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
