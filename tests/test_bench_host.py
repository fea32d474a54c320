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
        "a": {"launches": 8, "total_ms": 2.0, "alg_bytes": 8e9, "method_bytes": 0.0},
        "b": {"launches": 4, "total_ms": 6.0, "alg_bytes": 12e9, "method_bytes": 24e9},
    }
    roofline, kernels = bench.kernel_table(prof, 4)
    assert roofline["kernel"] == "b"
    # method bytes: 24 GB in 6 ms = 4000 GB/s, half the 8 TB/s peak
    assert roofline["achieved"] == pytest.approx(4000.0)
    assert roofline["frac"] == pytest.approx(0.5)
    assert roofline["bytes_per_launch"] == 6_000_000_000
    # the implementation's own bytes: 12 GB in 6 ms
    assert roofline["impl_achieved"] == pytest.approx(2000.0)
    assert roofline["impl_frac"] == pytest.approx(0.25)
    assert roofline["impl_bytes_per_launch"] == 3_000_000_000
    assert roofline["avg_launch_us"] == pytest.approx(1500.0)
    assert roofline["traffic"] is None
    assert list(kernels) == ["b", "a"]                       # by time, largest first
    assert kernels["a"]["launches_per_step"] == 2
    assert kernels["a"]["ms_per_step"] == pytest.approx(0.5)
    assert kernels["a"]["impl_GBs"] == pytest.approx(4000.0)
    assert kernels["a"]["method_GBs"] == 0.0
    assert kernels["b"]["share"] == pytest.approx(0.75)
    assert bench.kernel_table({}, 4) == (None, {})


def test_method_bytes_per_build_closed_form():
    """The per-build method bytes the library reports are the formula
    sum_{l=0}^{L-2} 8(k+1)(N - F(l)) + 8kN, split over the kernels that do
    each iteration; here the formula itself against a direct count."""
    def formula(n, k):
        L = n.bit_length()
        return sum(8 * (k + 1) * (n - (2 ** l - 1)) for l in range(L - 1)) + 8 * k * n
    # N = 10, k = 2: iterations l = 0, 1, 2 with 10, 9, 7 live points
    assert formula(10, 2) == 24 * (10 + 9 + 7) + 16 * 10
    # cfg 3 of the survey: 104.5 GB for 1e8 points, k = 4
    assert formula(100_000_000, 4) / 1e9 == pytest.approx(104.5, abs=0.1)


def test_build_rates_use_committed_counts(tmp_path, monkeypatch):
    prof = {"a": {"launches": 2, "total_ms": 1.0, "alg_bytes": 4e9, "method_bytes": 2e9}}
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    r = bench.build_rates(prof, 2, 2.0, "w")
    assert r["method_GB"] == pytest.approx(1.0) and r["method_GBs"] == pytest.approx(500.0)
    assert r["impl_GB"] == pytest.approx(2.0)
    assert r["counted_GBs"] is None
    rec = {"workload": "w", "kernel_source_sha": bench.kernel_source_sha(), "build_hbm_bytes": 8e9,
           "kernels": {"a": {"hbm_bytes_per_launch": 4e9}}}
    (tmp_path / "traffic_w.json").write_text(json.dumps(rec))
    r = bench.build_rates(prof, 2, 2.0, "w")
    assert r["counted_GBs"] == pytest.approx(4000.0) and r["counted_frac"] == pytest.approx(0.5)
    assert bench.dominant_traffic({"kernel": "a"}, "w") == 4e9
    assert bench.dominant_traffic({"kernel": "b"}, "w") is None


def test_strided_sample_keeps_the_mix():
    import numpy as np
    x = np.concatenate([np.zeros(900), np.ones(100)]).reshape(-1, 1)
    y = bench.strided_sample(x, 100)
    assert 95 <= y.shape[0] <= 105 and abs(float(y.mean()) - 0.1) < 0.02


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
    rec = {"workload": "w", "kernel_source_sha": "abc", "build_hbm_bytes": 5,
           "kernels": {"k_x": {"hbm_bytes_per_launch": 123}}}
    (tmp_path / "traffic_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "PROFILE_DIR", str(tmp_path))
    assert bench.committed_traffic("w", "abc")["kernels"]["k_x"]["hbm_bytes_per_launch"] == 123
    assert bench.committed_traffic("w", "def") is None      # taken on other sources
    assert bench.committed_traffic("v", "abc") is None      # none committed


def test_committed_records_name_their_workload():
    prof = os.path.join(ROOT, "profiles")
    for f in os.listdir(prof):
        if f.startswith("traffic_") and f.endswith(".json"):
            with open(os.path.join(prof, f)) as fh:
                rec = json.load(fh)
            assert f == f"traffic_{rec['workload']}.json"
            total = 0
            for k in rec["kernels"].values():
                # each figure is rounded to whole bytes on its own
                assert abs(k["hbm_bytes_per_launch"] - k["fetch_bytes_per_launch"]
                           - k["write_bytes_per_launch"]) <= 1
                total += k["hbm_bytes_per_launch"] * k["launches_per_build"]
            assert abs(total - rec["build_hbm_bytes"]) <= 1e-6 * rec["build_hbm_bytes"] + 64


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
