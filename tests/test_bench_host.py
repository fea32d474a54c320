"""Host-side logic of bench.py: the roofline arithmetic, the source hash that
ties a committed traffic record to the sources it was measured on, and the
single-GPU guard.  No GPU is used."""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_kernel_table_dominant_kernel_and_rates():
    # two kernels over 4 steps; "b" has the larger total time
    prof = {
        "a": {"launches": 8, "total_ms": 2.0, "alg_bytes": 8e9},
        "b": {"launches": 4, "total_ms": 6.0, "alg_bytes": 12e9},
    }
    roofline, kernels = bench.kernel_table(prof, 4)
    assert roofline["kernel"] == "b"
    # 12 GB in 6 ms = 2000 GB/s, a quarter of the 8 TB/s peak
    assert roofline["achieved"] == pytest.approx(2000.0)
    assert roofline["frac"] == pytest.approx(0.25)
    assert roofline["alg_bytes_per_launch"] == 3_000_000_000
    assert roofline["avg_launch_us"] == pytest.approx(1500.0)
    assert roofline["traffic"] is None
    assert list(kernels) == ["b", "a"]                       # by time, largest first
    assert kernels["a"]["launches_per_step"] == 2
    assert kernels["a"]["ms_per_step"] == pytest.approx(0.5)
    assert kernels["a"]["alg_GBs"] == pytest.approx(4000.0)
    assert kernels["b"]["share"] == pytest.approx(0.75)
    assert bench.kernel_table({}, 4) == (None, {})


def test_source_hash_covers_every_library_source(tmp_path, monkeypatch):
    csrc = os.path.join(ROOT, "paper_2211_00120_amd", "csrc")
    listed = {os.path.basename(p) for p in bench.KERNEL_SOURCES}
    on_disk = {f for f in os.listdir(csrc) if f.endswith((".hip", ".h", ".cpp"))}
    assert listed == on_disk
    # a copy of the sources hashes the same; any edit changes the hash
    dst = tmp_path / "paper_2211_00120_amd" / "csrc"
    shutil.copytree(csrc, dst)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    same = bench.kernel_source_sha()
    monkeypatch.setattr(bench, "ROOT", ROOT)
    assert same == bench.kernel_source_sha()
    victim = sorted(on_disk)[0]
    with open(dst / victim, "a") as f:
        f.write("\n// edit\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.kernel_source_sha() != same


def test_committed_traffic_only_for_matching_sources(tmp_path, monkeypatch):
    rec = {"kernel": "k_x", "workload": "w", "kernel_source_sha": "abc", "hbm_bytes_per_launch": 123}
    (tmp_path / "traffic_k_x_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    assert bench.committed_traffic("k_x", "w", "abc")["hbm_bytes_per_launch"] == 123
    assert bench.committed_traffic("k_x", "w", "def") is None      # taken on other sources
    assert bench.committed_traffic("k_y", "w", "abc") is None      # none committed


def test_committed_records_name_their_kernel_and_workload():
    prof = os.path.join(ROOT, "profiles")
    for f in os.listdir(prof):
        if f.startswith("traffic_") and f.endswith(".json"):
            with open(os.path.join(prof, f)) as fh:
                rec = json.load(fh)
            assert f == f"traffic_{rec['kernel']}_{rec['workload']}.json"
            # each figure is rounded to whole bytes on its own
            assert abs(rec["hbm_bytes_per_launch"] - rec["fetch_bytes_per_launch"]
                       - rec["write_bytes_per_launch"]) <= 1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
