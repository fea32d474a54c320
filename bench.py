"""Benchmark of the left-balanced k-d tree build on one MI355X.

One step = one complete build (kdt_build_ws: key prep, presorts, every
iteration's sort and tag update, placement) of the workload's points, which
are resident in HBM before timing starts; outputs and workspace are
preallocated.  Prints one JSON line:

  value       whole-job build throughput in Mpoints/s (N * steps / time)
  roofline    the kernel with the largest share of build time, its
              algorithmic bytes / its HIP-event-measured time against the
              8 TB/s HBM peak, and (when counters for the current kernel
              sources are committed) its measured HBM traffic per launch
  cpu_baseline  the CPU oracle timed on a bounded sample of the workload
  bit_exact   the GPU tree passes the oracle's full-tree checker (which, the
              tree being unique, is equality with the oracle's tree)

Workloads (--workload):
  mixture10m   N=10M 3D, half uniform, half 8-component Gaussian mixture, on
               the 2^-16 grid (heavy ties), round robin  [default]
  cluster100m  N=100M 4D uniform plus a 2^20-point cluster, split-widest
  small1024    N=1024 3D uniform, round robin
  uniform      --n points, --k dims, uniform [0,1)^k, round robin (the
               paper's Table 1 workload with k=4)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_2211_00120_amd/csrc/kdt_kernels.hip", "paper_2211_00120_amd/csrc/kdt_tail.hip",
                  "paper_2211_00120_amd/csrc/kdt_common.h", "paper_2211_00120_amd/csrc/kdt_device.h",
                  "paper_2211_00120_amd/csrc/kdt_layout.h", "paper_2211_00120_amd/csrc/kdt_kernels.h"]


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def make_workload(name: str, n: int, k: int):
    from paper_2211_00120_amd import kdt, workloads
    if name == "mixture10m":
        pts = workloads.cfg_mixture(n=n or 10_000_000, seed=2)
        return pts, kdt.ROUND_ROBIN, {"workload": "mixture10m", "n": int(pts.shape[0]), "k": 3,
                                      "dim_mode": "round_robin",
                                      "distribution": "half uniform [0,1)^3, half 8-Gaussian mixture sigma 0.01, "
                                                      "2^-16 grid", "seed": 2}
    if name == "cluster100m":
        pts = workloads.cfg_cluster4d(n=n or 100_000_000, seed=3)
        return pts, kdt.WIDEST, {"workload": "cluster100m", "n": int(pts.shape[0]), "k": 4,
                                 "dim_mode": "widest",
                                 "distribution": "uniform [0,1)^4 plus 2^20-point Gaussian cluster sigma 2^-10",
                                 "seed": 3}
    if name == "small1024":
        pts = workloads.cfg_small(1)
        return pts, kdt.ROUND_ROBIN, {"workload": "small1024", "n": 1024, "k": 3, "dim_mode": "round_robin",
                                      "distribution": "uniform [0,1)^3", "seed": 1}
    if name == "uniform":
        pts = workloads.uniform(n or 10_000_000, k, seed=7)
        return pts, kdt.ROUND_ROBIN, {"workload": f"uniform{k}d", "n": int(pts.shape[0]), "k": k,
                                      "dim_mode": "round_robin", "distribution": f"uniform [0,1)^{k}", "seed": 7}
    raise SystemExit(f"unknown workload {name}")


def committed_traffic(kernel: str, workload: str, sha: str):
    """Counter-derived HBM bytes per launch of `kernel`, if committed for the
    current kernel sources."""
    path = os.path.join(PROFILE_DIR, f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != sha:
        return None
    return rec


def cpu_baseline(pts, mode, target_s: float):
    """Time the oracle (single-threaded C) on a prefix of the workload sized to
    take roughly target_s seconds."""
    import oracle
    omode = oracle.WIDEST if mode == 1 else oracle.RR
    m = min(pts.shape[0], 200_000)
    t0 = time.perf_counter()
    oracle.build(pts[:m], omode)
    dt = time.perf_counter() - t0
    rate = m / max(dt, 1e-9)
    m2 = int(min(pts.shape[0], max(m, rate * target_s)))
    if m2 > m:
        t0 = time.perf_counter()
        oracle.build(pts[:m2], omode)
        dt = time.perf_counter() - t0
        m = m2
    return {"value": round(m / dt / 1e6, 4), "unit": "Mpoints/s", "cores": 1, "kind": "oracle",
            "sample": f"first {m} points of the same workload (same distribution), one build, "
                      f"{dt:.1f} s on one host core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="mixture10m")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--no-check", action="store_true", help="skip the full-tree bit-exactness check")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="before warmup, run one device-to-device copy of this many MiB (a reference kernel "
                         "of known traffic for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2211_00120_amd import kdt

    pts, mode, cfg = make_workload(args.workload, args.n, args.k)
    n, k = pts.shape
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d_pts = torch.from_numpy(pts).to(dev)
    tree = torch.empty((n, k), dtype=torch.float32, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    dim = torch.empty(n, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(kdt.workspace_bytes(n, k, mode), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()

    if args.calibrate_copy_mib:
        src = torch.ones(args.calibrate_copy_mib * (1 << 18), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        kdt.build_ws(d_pts, mode, tree=tree, perm=perm, dim=dim, status=status, workspace=ws, stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"# warmup done: n={n} k={k} mode={mode}", file=sys.stderr, flush=True)

    if not args.no_profile:
        kdt.profile_enable(True)
        kdt.profile_collect()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = {}
    if not args.no_profile:
        prof = kdt.profile_collect()
        kdt.profile_enable(False)
    st = int(status.item())
    print(f"# timed {args.steps} steps in {elapsed:.3f} s, status {st}", file=sys.stderr, flush=True)

    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed / 1e6

    roofline = None
    kernels = {}
    if prof:
        total_kernel_ms = sum(v["total_ms"] for v in prof.values())
        for name, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"]):
            kernels[name] = {
                "launches_per_step": v["launches"] / args.steps,
                "ms_per_step": round(v["total_ms"] / args.steps, 4),
                "avg_launch_us": round(v["total_ms"] * 1e3 / max(v["launches"], 1), 3),
                "share": round(v["total_ms"] / max(total_kernel_ms, 1e-12), 4),
                "alg_GBs": round(v["alg_bytes"] / max(v["total_ms"], 1e-12) / 1e6, 1),
            }
        dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
        achieved = dom["alg_bytes"] / dom["total_ms"] / 1e6   # GB/s
        sha = kernel_source_sha()
        tr = committed_traffic(dom_name, cfg["workload"], sha)
        roofline = {
            "bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "alg_bytes_per_launch": round(dom["alg_bytes"] / dom["launches"]),
            "avg_launch_us": round(dom["total_ms"] * 1e3 / dom["launches"], 3),
            "traffic": (tr["hbm_bytes_per_launch"] if tr else None),
        }
        build_alg = sum(v["alg_bytes"] for v in prof.values()) / args.steps
        roofline["build_alg_GBs"] = round(build_alg / (ms_per_step * 1e6), 1)

    bit_exact = None
    if not args.no_check:
        import oracle
        code, node = oracle.check(pts, perm.cpu().numpy().astype(np.uint32), dim.cpu().numpy(),
                                  oracle.WIDEST if mode == kdt.WIDEST else oracle.RR)
        same_tree = np.array_equal(tree.cpu().numpy(), pts[perm.cpu().numpy()])
        bit_exact = bool(code == 0 and same_tree and st == 0)
        print(f"# checker code {code} node {node}, tree gather {same_tree}", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu else cpu_baseline(pts, mode, args.cpu_seconds)

    out = {
        "metric": "k-d build Mpoints/s + achieved HBM GB/s; batched vs per-cloud, bit-exact",
        "value": round(value, 3),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 in, u32 ranks",
        "data": "synthetic",
        "config": cfg,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "bit_exact": bit_exact,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
