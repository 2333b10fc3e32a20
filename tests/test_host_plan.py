"""The factorisation schedule on the CPU: tests/native/plan_check.cpp builds
the library's plan (host sources compiled with g++) and runs its task lists
in plain loops, then checks every tile against the definition of the partial
Cholesky factorisation of the augmented matrix (A = L L^T on the r columns,
trailing blocks A - L L^T, the S_rIrI copy as the Schur complement after the
r_V columns), offsets inside the pool, and that no update launch writes a
tile twice or writes a tile that it also reads.

The configurations reach both deferral thresholds (8 pending contributions
before a subdomain's dense r_I tail, 4 inside it) and the deadlines of the
level schedule (a target's column level, the S_rIrI copy, the subdomain's
last level); a deadline taken one level late or a missing S copy deadline
fails the check.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "paper_2501_04340_amd", "csrc", "host")


@pytest.fixture(scope="module")
def plan_check(tmp_path_factory):
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("plan_check") / "plan_check")
    srcs = [os.path.join(ROOT, "tests", "native", "plan_check.cpp")]
    srcs += sorted(os.path.join(HOST, f) for f in os.listdir(HOST) if f.endswith(".cpp"))
    cmd = [cxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_2501_04340_amd", "csrc"), "-o", exe, *srcs, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    return exe


@pytest.mark.parametrize("cfg", [
    (2, 2, 2, 2, 4, 8),   # eight one-patch subdomains (the smallest box workload)
    (3, 2, 2, 2, 5, 3),   # uneven subdomains of four patches
    (2, 2, 2, 3, 6, 2),   # deep nested dissection: targets with more than 8 contributions
    (2, 2, 2, 3, 6, 2, 2, 1),    # the autotuner's extreme thresholds: every contribution early ...
    (2, 2, 2, 3, 6, 2, 16, 8),   # ... or most of them at their deadline
])
def test_factor_schedule_matches_definition(plan_check, cfg):
    res = subprocess.run([plan_check, *map(str, cfg)], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    m = re.search(r"factor residual ([0-9.e+-]+) S residual ([0-9.e+-]+)", res.stdout)
    assert m and float(m.group(1)) < 1e-12 and float(m.group(2)) < 1e-12, res.stdout


def test_coarse_tile_plan_matches_definition(tmp_path):
    """The coarse problem's tile plan (tests/native/coarse_check.cpp): its
    task lists run in plain loops give L_c L_c^T = S_c, H L_c^T = G and
    L_c^T U = I for problems with n_gp = 0, 1, 3, 64, 65, 150 and row counts
    that are and are not multiples of the tile size."""
    cxx = shutil.which("g++")
    if cxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / "coarse_check")
    srcs = [os.path.join(ROOT, "tests", "native", "coarse_check.cpp")]
    srcs += sorted(os.path.join(HOST, f) for f in os.listdir(HOST) if f.endswith(".cpp"))
    cmd = [cxx, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I",
           os.path.join(ROOT, "paper_2501_04340_amd", "csrc"), "-o", exe, *srcs, "-lpthread"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert res.returncode == 0, res.stderr[-4000:]
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "pivots ok" in res.stdout
