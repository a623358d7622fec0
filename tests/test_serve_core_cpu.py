"""The serving scheduler (paper_2112_09017_amd/csrc/serve_core.h) on the CPU,
against the scripted executor of tests/serve_core_test.cpp: admission by arena
footprint, slots and per-tick staging capacity, FIFO order, the stop test
against an independent model of the scalar iteration, request isolation,
non-finite inputs, the step cap, queue-full, device errors in a tick and in
the finish step, a failing device bind, many submitting and polling threads,
and shutdown with requests in flight.  Built with g++ under ThreadSanitizer
and under AddressSanitizer + UndefinedBehaviorSanitizer; either reporting an
error fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "serve_core_test.cpp")
INC = os.path.join(ROOT, "paper_2112_09017_amd", "csrc")

SANITIZERS = {
    "tsan": ["-fsanitize=thread"],
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
}


@pytest.mark.parametrize("san", sorted(SANITIZERS))
def test_serve_core_under_sanitizer(tmp_path, san):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / f"serve_core_{san}")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-Wall", "-Werror", *SANITIZERS[san], "-I", INC, SRC,
           "-o", exe, "-pthread"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    env = dict(os.environ)
    env["TSAN_OPTIONS"] = "halt_on_error=1 second_deadlock_stack=1"
    env["ASAN_OPTIONS"] = "detect_leaks=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ALL OK" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr
    assert "runtime error" not in r.stderr
