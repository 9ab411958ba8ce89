"""Host code under sanitizers, on the CPU.

* The serving scheduler (hfr_sched.h) with a fake backend that answers each request with the CPU
  oracle's greedy loop, built with AddressSanitizer + UndefinedBehaviorSanitizer and, separately,
  with ThreadSanitizer (the scheduler is multi-threaded: slots, submitters, cancellation).
* The oracle itself under AddressSanitizer + UndefinedBehaviorSanitizer, on the brute-force-pinned
  paths (Simulate with and without blocked pairs, reach, the greedy loop) through that same driver.

Both are compiled with g++/gcc here (no GPU code is involved) and must exit cleanly.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "sched_cpu_test.cpp")
ORACLE = os.path.join(ROOT, "oracle", "hfr_oracle.c")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def _build_and_run(tmp_path, flags, name):
    obj = tmp_path / f"oracle_{name}.o"
    exe = tmp_path / f"sched_{name}"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", *flags, "-c", ORACLE, "-o", str(obj)])
    subprocess.check_call(["g++", "-O1", "-g", "-std=c++17", *flags, SRC, str(obj), "-o", str(exe), "-lpthread", "-lm"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "sched ok" in r.stdout
    return r


def test_scheduler_and_oracle_asan_ubsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                              "-fno-omit-frame-pointer"], "asan")


def test_scheduler_tsan(tmp_path):
    _build_and_run(tmp_path, ["-fsanitize=thread"], "tsan")
