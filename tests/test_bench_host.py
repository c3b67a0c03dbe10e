"""Host-side pieces of bench.py (no GPU): the refusal of more than one GPU, and the serving leg's
child-process handling (its JSON line is read back; a child that fails or overruns its time
gives an error entry and the rest of the line still prints)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def _child(code):
    return subprocess.Popen([sys.executable, "-c", code], stdin=subprocess.PIPE,
                            stdout=subprocess.PIPE, text=True)


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2 and "one GPU" in p.stderr


def test_served_leg_reads_the_child_line():
    res = {"saturated_Mkeys_s": 1.0, "points": []}
    code = ("import sys, json\n"
            "assert sys.stdin.readline() == 'go\\n'\n"
            f"print('log line'); print(json.dumps({res!r}))")
    assert bench.served_leg(_child(code), 30.0) == res


def test_served_leg_reports_failure_and_overrun():
    assert "error" in bench.served_leg(_child("import sys; sys.exit(3)"), 30.0)
    slow = _child("import sys, time; sys.stdin.readline(); time.sleep(60)")
    out = bench.served_leg(slow, 1.0)
    assert "did not finish" in out["error"] and slow.poll() is not None


def test_serving_child_exits_at_end_of_input():
    p = subprocess.run([sys.executable, "-m", "paper_1908_05936_amd.bench_serve", "--wait-stdin"],
                       cwd=ROOT, input="", capture_output=True, text=True, timeout=300)
    assert p.returncode == 0 and p.stdout == ""
