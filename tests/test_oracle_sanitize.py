"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code, gcc): every
entry point of oracle.c and partitioned.c on random batches over several table shapes, the
invariant checker clean after every batch and tripped by every planted corruption, no leak at
exit (tests/native/oracle_sanitize.c)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRCS = [os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(ROOT, "oracle", "partitioned.c"),
        os.path.join(HERE, "native", "oracle_sanitize.c")]


def _run(tmp_path, flags):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize")
    b = subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-Wall", "-pthread", *SRCS, "-o", exe, *flags],
                       capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and flags:
        pytest.skip(f"sanitizer build unavailable: {b.stderr[-300:]}")
    assert b.returncode == 0, b.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert "oracle sanitize run passed" in r.stdout


def test_oracle_entry_points_plain(tmp_path):
    _run(tmp_path, [])


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    _run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"])
