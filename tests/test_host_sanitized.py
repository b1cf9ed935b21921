"""Host-side code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/host/sched_harness.cpp drives the request server's scheduling core (csrc/scp_sched.hpp)
against a simulated executor and clock (admission, budget, workgroup cap, sessions, warm starts,
eviction, staging back-pressure, timeouts, cancellation, the done list, latency quantiles) and the
batch planner (csrc/scp_plan.cpp) on seeded random descriptions.  Both sources are free of device
code, so the harness is built with the host compiler and both sanitizers, and any report or failed
check fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_scheduler_and_planner_under_asan_ubsan(tmp_path):
    exe = tmp_path / "sched_harness"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I" + os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "sched_harness.cpp"),
           os.path.join(ROOT, "paper_2603_10711_amd", "csrc", "scp_plan.cpp"), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([str(exe), "600"], capture_output=True, text=True, env=env, timeout=300)
    print(run.stdout)
    assert run.returncode == 0, run.stdout[-4000:] + run.stderr[-4000:]
    assert "ALL OK" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
