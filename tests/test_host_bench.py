"""Host-side logic of bench.py: the one-GPU guard and how the measured HBM
traffic is taken from the committed PMC summary (only for the workload the
counters were taken on, and dropped once the kernel source or the task-list
builder has changed since)."""
import hashlib
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stdout
    assert "{" not in r.stdout  # no JSON line


def _write_sources(tmp_path, texts):
    files = []
    for i, t in enumerate(texts):
        p = tmp_path / f"src{i}.txt"
        p.write_bytes(t)
        files.append(str(p))
    return files


def test_sources_hash_covers_every_file_in_order(tmp_path, monkeypatch):
    files = _write_sources(tmp_path, [b"kernel source", b"plan source"])
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", files)
    want = hashlib.sha256(b"kernel source" + b"plan source").hexdigest()
    assert bench.sources_sha256() == want
    (tmp_path / "src1.txt").write_bytes(b"plan source, changed")
    assert bench.sources_sha256() != want


def test_traffic_read_only_for_matching_sources(tmp_path, monkeypatch):
    files = _write_sources(tmp_path, [b"a", b"b"])
    monkeypatch.setattr(bench, "TRAFFIC_SOURCES", files)
    sha = bench.sources_sha256()
    prof = tmp_path / "traffic.md"
    prof.write_text(
        "header\n"
        f"traffic_per_launch k_update_multi: workload=cube64 params=8,4,2048 fetch_bytes=10 write_bytes=5 "
        f"total_bytes=15 sources_sha256={sha}\n"
        f"traffic_per_launch k_update_multi: workload=cube256 params=8,4,2048 fetch_bytes=20 write_bytes=5 "
        f"total_bytes=25 sources_sha256={sha}\n"
        f"traffic_per_launch k_update_multi: workload=stream256[0..63] params=8,8,2048 fetch_bytes=30 "
        f"write_bytes=5 total_bytes=35 sources_sha256={sha}\n"
        f"traffic_per_launch k_gemv_sym<double>: workload=cube64 fetch_bytes=7 write_bytes=1 total_bytes=8 "
        f"sources_sha256={sha}\n"
        "traffic_per_launch k_gemv<double>: workload=cube64 fetch_bytes=7 write_bytes=1 total_bytes=9 "
        "sources_sha256=" + "0" * 64 + "\n")
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", [str(prof)])
    assert bench.measured_traffic("k_update_multi", "cube64", (8, 4, 2048)) == 15.0
    assert bench.measured_traffic("k_update_multi", "cube256", (8, 4, 2048)) == 25.0
    assert bench.measured_traffic("k_update_multi", "stream256[0..63]", (8, 8, 2048)) == 35.0
    # the tile update's launches depend on the schedule parameters
    assert bench.measured_traffic("k_update_multi", "cube64", (8, 4, 1024)) is None
    assert bench.measured_traffic("k_update_multi", "cube64") is None
    assert bench.measured_traffic("k_update_multi", "stream256[64..127]", (8, 8, 2048)) is None
    # the GEMV's do not
    assert bench.measured_traffic("k_gemv_sym<double>", "cube64") == 8.0
    # a workload the counters were not taken on
    assert bench.measured_traffic("k_gemv_sym<double>", "cube256") is None
    # stale hash, and a kernel the summary does not hold
    assert bench.measured_traffic("k_gemv<double>", "cube64") is None
    assert bench.measured_traffic("k_trsm_inv", "cube64") is None
    # any change to the sources invalidates every figure
    (tmp_path / "src0.txt").write_bytes(b"a2")
    assert bench.measured_traffic("k_update_multi", "cube64", (8, 4, 2048)) is None


def test_traffic_missing_profile(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "TRAFFIC_PROFILES", [str(tmp_path / "absent.md")])
    assert bench.measured_traffic("k_update_multi", "cube64") is None


def test_committed_summary_parses():
    """Each committed summary carries figures for the kernels bench.py reports
    on its workload (the tile update with its schedule parameters), each with
    a 64-digit source hash."""
    import re
    want = {"stream256_batch64": ("stream256[0..63]", ("k_update_multi", "k_gemv_sym<float>")),
            "cube64_": ("cube64", ("k_update_multi", "k_gemv_sym<double>")),
            "cube256_": ("cube256", ("k_update_multi", "k_gemv_sym<double>"))}
    assert len(bench.TRAFFIC_PROFILES) == len(want)
    for f in bench.TRAFFIC_PROFILES:
        key = next(k for k in want if os.path.basename(f).startswith(k))
        workload, kernels = want[key]
        text = open(f).read()
        for k in kernels:
            params = r"params=\d+,\d+,\d+ " if k == "k_update_multi" else ""
            m = re.search(r"traffic_per_launch " + re.escape(k) + r": workload=" + re.escape(workload) + " "
                          + params + r".*total_bytes=(\d+) sources_sha256=([0-9a-f]{64})", text)
            assert m, (f, k)
            assert int(m.group(1)) > 0


if __name__ == "__main__":
    sys.exit(pytest.main([__file__, "-q"]))
