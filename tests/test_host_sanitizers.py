"""The library's host code (assembly, topology, tree, partition checks,
factorisation plan) under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/plan_check.cpp drives the host sources through assembly and
the factorisation plan and runs the plan's task lists on the CPU (the same
program as test_host_plan.py); here it is built with g++ and both
sanitizers (CPU code only, no GPU sources), and any report fails the test.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "paper_2501_04340_amd", "csrc", "host")


@pytest.fixture(scope="module")
def plan_check_sanitized(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan_check_san") / "plan_check")
    srcs = [os.path.join(ROOT, "tests", "native", "plan_check.cpp")]
    srcs += sorted(os.path.join(HOST, f) for f in os.listdir(HOST) if f.endswith(".cpp"))
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]
    cmd = [cxx, *flags, "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_2501_04340_amd", "csrc"), "-o", exe, *srcs, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


@pytest.mark.parametrize("cfg", [
    (2, 2, 2, 2, 4, 8),   # eight one-patch subdomains
    (3, 2, 2, 2, 3, 3),   # uneven subdomains of four patches
])
def test_host_code_is_clean_under_sanitizers(plan_check_sanitized, cfg):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([plan_check_sanitized, *map(str, cfg)], capture_output=True, text=True,
                         timeout=600, env=env)
    out = res.stdout + res.stderr
    assert res.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out and "LeakSanitizer" not in out, out[-4000:]
