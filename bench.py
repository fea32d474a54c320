"""Benchmark of the left-balanced k-d tree build on one MI355X.

One step = one complete build (kdt_build_ws: key prep, presorts, every
iteration's sort and tag update, placement) of the workload's points, which
are resident in HBM before timing starts; outputs and workspace are
preallocated.  Prints one JSON line:

  value       whole-job build throughput in Mpoints/s (N * steps / time)
  roofline    the kernel with the largest share of build time: the bytes the
              paper's method moves for the work that kernel completes (each
              iteration reads and writes every live point's k coordinates and
              32-bit tag once, 8(k+1) B per live point; the final placement
              8k B per point) over its HIP-event-measured time, against the
              8 TB/s HBM peak; the same with this implementation's own byte
              model ("impl_*"); and (when counters for the current kernel
              sources are committed) its measured HBM traffic per launch
  build       the whole build: method bytes per build and, from the committed
              counters, counted HBM bytes per build, each over the build time
  cpu_baseline  the CPU oracle (OpenMP tasks on every host core) timed on a
              bounded, evenly strided sample of the workload, with the core
              count, the CPU model and the single-core rate
  bit_exact   the GPU tree passes the oracle's full-tree checker (which, the
              tree being unique, is equality with the oracle's tree), the
              tree's coordinates equal points[perm] byte for byte, and the
              device status word is 0

Workloads (--workload):
  cluster100m  N=100M 4D uniform plus a 2^20-point cluster, split-widest
               [default]
  mixture10m   N=10M 3D, half uniform, half 8-component Gaussian mixture, on
               the 2^-16 grid (heavy ties), round robin
  small1024    N=1024 3D uniform, round robin
  uniform      --n points, --k dims, uniform [0,1)^k, round robin (the
               paper's Table 1 workload with k=4)
  int1         --n int32 points (default 1e8) with k = 1, uniform over all
               int32 values, round robin (Table 1's int1 rows; the paper does
               not state their distribution)
  batched4096  4096 independent 3D clouds, sizes log-uniform in [64, 262144],
               each uniform in its own random box, round robin: one step is
               one kdt_build_batched of all clouds, captured once into a HIP
               graph and replayed; the line also carries the same clouds built
               one kdt_build_ws call after another on one stream
               ("per_cloud"), and whether both give identical bytes
  serving      an open-loop request trace (Poisson arrivals, 2000 per second;
               each request k uniform in {2,3,4}, N log-uniform in [1e3, 4e6],
               points uniform in [0,1)^k) replayed into the build server
               (64 GiB pool): value is served points per second, with p50/p99
               latency from the scheduled arrival, beside the same trace built
               one request at a time in arrival order ("fifo"); --requests
               sets the trace length
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE_DIR = os.path.join(ROOT, "profiles")
# every library source: kernels, tile constants, planner and launch sequence
# all shape what a kernel moves
KERNEL_SOURCES = sorted(os.path.join("paper_2211_00120_amd", "csrc", f)
                        for f in os.listdir(os.path.join(ROOT, "paper_2211_00120_amd", "csrc"))
                        if f.endswith((".hip", ".h", ".cpp")))
METRIC = "k-d build Mpoints/s + achieved HBM GB/s; batched vs per-cloud, bit-exact"


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
    if name == "batched4096":
        pts, offsets = workloads.cfg_batched()
        cfg = {"workload": "batched4096", "clouds": int(len(offsets) - 1), "n": int(pts.shape[0]), "k": 3,
               "dim_mode": "round_robin",
               "distribution": "4096 clouds, sizes log-uniform in [64, 262144], each uniform in a random box "
                               "(corner in [-1000,1000)^3, extents log-uniform in [1e-2, 1e2])", "seed": 4}
        return (pts, offsets), kdt.ROUND_ROBIN, cfg
    if name == "uniform":
        pts = workloads.uniform(n or 10_000_000, k, seed=7)
        return pts, kdt.ROUND_ROBIN, {"workload": f"uniform{k}d", "n": int(pts.shape[0]), "k": k,
                                      "dim_mode": "round_robin", "distribution": f"uniform [0,1)^{k}", "seed": 7}
    if name == "int1":
        pts = workloads.int_uniform(n or 100_000_000, 1, seed=11)
        return pts, kdt.ROUND_ROBIN, {"workload": "int1", "n": int(pts.shape[0]), "k": 1,
                                      "dim_mode": "round_robin", "coords": "int32",
                                      "distribution": "uniform over all int32 values", "seed": 11}
    raise SystemExit(f"unknown workload {name}")


def committed_traffic(workload: str, sha: str):
    """The counter-derived HBM traffic record of `workload`
    (profiles/traffic_<workload>.json: bytes per launch of every kernel and
    per build), if it was taken on the current kernel sources."""
    path = os.path.join(PROFILE_DIR, f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha") != sha:
        return None
    return rec


def host_cpu():
    """(threads this process may run on, CPU model name)."""
    try:
        threads = len(os.sched_getaffinity(0))
    except AttributeError:
        threads = os.cpu_count() or 1
    model = platform.processor() or "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return threads, model


def strided_sample(pts, m):
    """About m points taken at an even stride, so that a workload built as a
    concatenation of parts (uniform then cluster, uniform then mixture)
    keeps its mix."""
    step = max(1, -(-pts.shape[0] // m))
    return pts[::step]


def cpu_baseline(pts, mode, target_s: float):
    """Time the oracle on an evenly strided sample of the workload sized to
    take roughly target_s seconds on every host core (OpenMP tasks), and the
    single-threaded oracle on a smaller sample."""
    import numpy as np
    import oracle
    omode = oracle.WIDEST if mode == 1 else oracle.RR
    threads, model = host_cpu()
    # single core: a sample of ~target_s / 4
    m = min(pts.shape[0], 100_000)
    t0 = time.perf_counter()
    oracle.build(strided_sample(pts, m), omode)
    rate1 = m / max(time.perf_counter() - t0, 1e-9)
    m1 = int(min(pts.shape[0], max(m, rate1 * target_s / 4)))
    x = np.ascontiguousarray(strided_sample(pts, m1))
    t0 = time.perf_counter()
    oracle.build(x, omode)
    dt1 = time.perf_counter() - t0
    rate1 = x.shape[0] / dt1
    # every core: a sample of ~target_s, from the single-core rate times the cores
    mp = int(min(pts.shape[0], max(m1, rate1 * max(1, threads // 2) * target_s)))
    xp = np.ascontiguousarray(strided_sample(pts, mp))
    t0 = time.perf_counter()
    oracle.build(xp, omode, threads=threads)
    dtp = time.perf_counter() - t0
    return {"value": round(xp.shape[0] / dtp / 1e6, 4), "unit": "Mpoints/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "nproc": os.cpu_count(),
            "single_core": {"value": round(rate1 / 1e6, 4), "unit": "Mpoints/s",
                            "sample": f"{x.shape[0]} points, {dt1:.1f} s"},
            "sample": f"{xp.shape[0]} points of the same workload taken at an even stride (same mix of its "
                      f"parts), one build by the oracle's recursion with subtrees as OpenMP tasks on {threads} "
                      f"threads, {dtp:.1f} s"}


def kernel_table(prof, steps):
    """Per-kernel summary and the roofline object of the dominant kernel (the
    one with the largest share of event-measured time)."""
    kernels = {}
    if not prof:
        return None, kernels
    total_kernel_ms = sum(v["total_ms"] for v in prof.values())
    for name, v in sorted(prof.items(), key=lambda kv: -kv[1]["total_ms"]):
        t = max(v["total_ms"], 1e-12)
        kernels[name] = {
            "launches_per_step": v["launches"] / steps,
            "ms_per_step": round(v["total_ms"] / steps, 4),
            "avg_launch_us": round(v["total_ms"] * 1e3 / max(v["launches"], 1), 3),
            "share": round(v["total_ms"] / max(total_kernel_ms, 1e-12), 4),
            "method_GBs": round(v.get("method_bytes", 0.0) / t / 1e6, 1),
            "impl_GBs": round(v["alg_bytes"] / t / 1e6, 1),
        }
    dom_name, dom = max(prof.items(), key=lambda kv: kv[1]["total_ms"])
    mb = dom.get("method_bytes", 0.0)
    achieved = mb / dom["total_ms"] / 1e6                  # GB/s
    impl = dom["alg_bytes"] / dom["total_ms"] / 1e6
    roofline = {
        "bound": "hbm", "kernel": dom_name, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
        "bytes": "paper method: 8(k+1) B per live point per iteration completed, 8k B per point placed",
        "bytes_per_launch": round(mb / dom["launches"]),
        "avg_launch_us": round(dom["total_ms"] * 1e3 / dom["launches"], 3),
        "impl_achieved": round(impl, 1), "impl_frac": round(impl / HBM_PEAK_GBS, 4),
        "impl_bytes_per_launch": round(dom["alg_bytes"] / dom["launches"]),
        "traffic": None,
    }
    return roofline, kernels


def build_rates(prof, steps, ms_per_step, workload):
    """Whole-build GB/s: the paper method's bytes per build, and (from the
    committed counters, when they match the sources) the counted HBM bytes
    per build, each over the un-profiled build time."""
    out = {"ms": round(ms_per_step, 4)}
    if prof:
        mb = sum(v.get("method_bytes", 0.0) for v in prof.values()) / steps
        ib = sum(v["alg_bytes"] for v in prof.values()) / steps
        out["method_GB"] = round(mb / 1e9, 3)
        out["method_GBs"] = round(mb / (ms_per_step * 1e6), 1)
        out["method_frac"] = round(mb / (ms_per_step * 1e6) / HBM_PEAK_GBS, 4)
        out["impl_GB"] = round(ib / 1e9, 3)
        out["impl_GBs"] = round(ib / (ms_per_step * 1e6), 1)
    tr = committed_traffic(workload, kernel_source_sha())
    if tr:
        out["counted_GB"] = round(tr["build_hbm_bytes"] / 1e9, 3)
        out["counted_GBs"] = round(tr["build_hbm_bytes"] / (ms_per_step * 1e6), 1)
        out["counted_frac"] = round(tr["build_hbm_bytes"] / (ms_per_step * 1e6) / HBM_PEAK_GBS, 4)
    else:
        out["counted_GB"] = out["counted_GBs"] = out["counted_frac"] = None
    return out


def dominant_traffic(roofline, workload):
    """Counted HBM bytes per launch of the roofline's kernel, or None."""
    tr = committed_traffic(workload, kernel_source_sha())
    if not tr or not roofline:
        return None
    k = tr.get("kernels", {}).get(roofline["kernel"])
    return k["hbm_bytes_per_launch"] if k else None


def calibration_copy(args, dev):
    """One device-to-device copy of a known size, for scaling rocprofv3's
    FETCH_SIZE / WRITE_SIZE counters of the same run."""
    import torch
    if args.calibrate_copy_mib:
        src = torch.ones(args.calibrate_copy_mib * (1 << 18), dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def run_batched(args, data, mode, cfg):
    """One step = one graph replay of kdt_build_batched over every cloud."""
    import numpy as np
    import torch

    from paper_2211_00120_amd import kdt

    pts, offsets = data
    n, k = pts.shape
    C = len(offsets) - 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d_pts = torch.from_numpy(pts).to(dev)
    tree = torch.empty((n, k), dtype=torch.float32, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    dim = torch.empty(n, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(kdt.batched_workspace_bytes(offsets, k, mode), dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream()
    calibration_copy(args, dev)

    def build_eager():
        kdt.build_batched(d_pts, offsets, mode, tree=tree, perm=perm, dim=dim, status=status, workspace=ws,
                          stream=stream)

    if args.autotune:
        rb, items, pdims, tms = kdt.tune_batched(d_pts, offsets, mode, reps=2, workspace=ws, stream=stream)
        cfg["tuned"] = {"radix_bits": rb, "level_items": items, "presort_dims": pdims}
        print(f"# autotune: radix {rb} items {items} presort dims {pdims} ({tms:.3f} ms)", file=sys.stderr, flush=True)
    # per-kernel breakdown from profiled eager builds on the side stream
    with torch.cuda.stream(stream):
        for _ in range(max(args.warmup, 1)):
            build_eager()
        torch.cuda.synchronize()
        psteps = max(1, min(args.steps, 5))
        kdt.profile_enable(True)
        kdt.profile_collect()
        for _ in range(psteps):
            build_eager()
        prof = kdt.profile_collect()
        kdt.profile_enable(False)
    roofline, kernels = kernel_table(prof, psteps)
    print(f"# batched: {C} clouds, n={n}; profiled {psteps} eager builds", file=sys.stderr, flush=True)

    # the timed steps: graph replays
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=stream):
            build_eager()
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g.replay()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    st = int(status.item())
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed / 1e6
    if roofline:
        roofline["traffic"] = dominant_traffic(roofline, cfg["workload"])
    build = build_rates(prof, psteps, ms_per_step, cfg["workload"])
    print(f"# batched graph: {ms_per_step:.3f} ms per build, status {st}", file=sys.stderr, flush=True)

    if args.no_per_cloud:
        return {"value": round(value, 3), "ms_per_step": round(ms_per_step, 4), "roofline": roofline,
                "build": build, "kernels": kernels, "bit_exact": None, "cpu_baseline": None, "per_cloud": None,
                "batched_vs_per_cloud": None}
    # the same clouds as one kdt_build_ws call each, one after another on one
    # stream, preallocated, no host synchronisation between calls
    nmax = int(np.max(np.diff(offsets.astype(np.int64))))
    ws1 = torch.empty(kdt.workspace_bytes(nmax, k, mode), dtype=torch.uint8, device=dev)
    tree1 = torch.empty_like(tree)
    perm1 = torch.empty_like(perm)
    dim1 = torch.empty_like(dim)
    st1 = torch.zeros(1, dtype=torch.int32, device=dev)
    bounds = [(int(offsets[c]), int(offsets[c + 1])) for c in range(C)]
    views = [(d_pts[a:b], tree1[a:b], perm1[a:b], dim1[a:b]) for a, b in bounds]

    def per_cloud():
        for p_, t_, q_, d_ in views:
            kdt.build_ws(p_, mode, tree=t_, perm=q_, dim=d_, status=st1, workspace=ws1, stream=stream)

    with torch.cuda.stream(stream):
        per_cloud()
        torch.cuda.synchronize()
        reps = max(1, min(args.steps, 3))
        t0 = time.perf_counter()
        for _ in range(reps):
            per_cloud()
        torch.cuda.synchronize()
        pc_elapsed = time.perf_counter() - t0
    pc_ms = pc_elapsed * 1e3 / reps
    same = bool(torch.equal(tree, tree1) and torch.equal(perm, perm1) and torch.equal(dim, dim1))
    print(f"# per-cloud: {pc_ms:.3f} ms per pass, identical to batched: {same}", file=sys.stderr, flush=True)

    bit_exact = None
    if not args.no_check:
        import oracle
        pb = perm.cpu().numpy().astype(np.uint32)
        db = dim.cpu().numpy()
        tb = tree.cpu().numpy()
        ok = st == 0 and same
        for a, b in bounds:
            code, _ = oracle.check(pts[a:b], pb[a:b], db[a:b], oracle.RR)
            ok = ok and code == 0 and np.array_equal(tb[a:b], pts[a:b][pb[a:b]])
        bit_exact = bool(ok)
        print(f"# checker over all clouds: {bit_exact}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_clouds(pts, offsets, args.cpu_seconds)

    return {
        "value": round(value, 3), "ms_per_step": round(ms_per_step, 4), "roofline": roofline, "build": build,
        "kernels": kernels, "bit_exact": bit_exact, "cpu_baseline": cpu,
        "per_cloud": {"value": round(n / pc_elapsed * reps / 1e6, 3), "unit": "Mpoints/s",
                      "ms_per_pass": round(pc_ms, 3), "calls": C, "identical_to_batched": same},
        "batched_vs_per_cloud": round(pc_ms / ms_per_step, 3),
    }


def run_serving(args):
    """Replay the request trace into kdt_server_* and, for comparison, build
    the same requests one at a time in arrival order."""
    import threading

    import numpy as np
    import torch

    from paper_2211_00120_amd import kdt, workloads

    arrivals, ks, ns, _ = workloads.cfg_serving_trace(requests=args.requests, seed=5)
    R = len(arrivals)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    # request points: views into a few pinned host buffers of uniform points
    # (request i reads buffer i mod B), so the trace needs no per-request
    # generation while it is replayed
    nbuf = 8
    nmax = int(ns.max())
    gen = torch.Generator().manual_seed(5)
    bufs = [torch.rand(nmax * 4, generator=gen, dtype=torch.float32).pin_memory() for _ in range(nbuf)]
    views = [bufs[i % nbuf][: int(ns[i]) * int(ks[i])].view(int(ns[i]), int(ks[i])) for i in range(R)]
    total_pts = int(ns.sum())
    print(f"# serving: {R} requests, {total_pts} points, offered {total_pts / arrivals[-1] / 1e6:.0f} Mpts/s",
          file=sys.stderr, flush=True)

    def replay(srv):
        tickets = [None] * R
        done = {}
        lock = threading.Lock()
        submitted = [0]

        def reaper():
            nxt = 0
            while len(done) < R:
                with lock:
                    hi = submitted[0]
                progressed = False
                for i in range(nxt, hi):
                    if i in done:
                        continue
                    r = srv.poll(tickets[i])
                    if r is None:
                        continue
                    done[i] = (r.status, r.t_admit, r.t_done, r.device_ms, r.batch_requests)
                    srv.release(tickets[i])
                    progressed = True
                while nxt in done:
                    nxt += 1
                if not progressed:
                    time.sleep(50e-6)

        th = threading.Thread(target=reaper)
        th.start()
        t0 = kdt.clock() + 0.05
        for i in range(R):
            target = t0 + float(arrivals[i])
            while True:
                dt = target - kdt.clock()
                if dt <= 0:
                    break
                if dt > 300e-6:
                    time.sleep(dt - 200e-6)
            tickets[i] = srv.submit(views[i], kdt.ROUND_ROBIN)
            with lock:
                submitted[0] = i + 1
        th.join()
        return t0, done

    with kdt.Server(64 << 30, max_inflight=args.inflight, max_batch_requests=64, max_batch_points=1 << 26) as srv:
        # warm-up: one request of each k, small and large, before the replay
        warm = [srv.submit(bufs[0][: n * k].view(n, k), kdt.ROUND_ROBIN) for k in (2, 3, 4) for n in (1000, nmax)]
        for t in warm:
            srv.wait(t)
            srv.release(t)
        t0, done = replay(srv)
    lat = np.array([done[i][2] - (t0 + arrivals[i]) for i in range(R)]) * 1e3
    dev_ms = np.array([done[i][3] for i in range(R)])
    bsz = np.array([done[i][4] for i in range(R)])
    statuses = {done[i][0] for i in range(R)}
    makespan = max(done[i][2] for i in range(R)) - t0
    served = total_pts / makespan / 1e6
    print(f"# served: {served:.1f} Mpts/s, p50 {np.percentile(lat, 50):.2f} ms, p99 {np.percentile(lat, 99):.2f} ms,"
          f" statuses {statuses}", file=sys.stderr, flush=True)

    # the same requests one at a time in arrival order (kdt_build_ws with a
    # preallocated workspace; copy-in included, as for the server)
    stream = torch.cuda.current_stream()
    d_in = torch.empty(nmax * 4, dtype=torch.float32, device=dev)
    tree = torch.empty(nmax * 4, dtype=torch.float32, device=dev)
    perm = torch.empty(nmax, dtype=torch.int32, device=dev)
    dim = torch.empty(nmax, dtype=torch.uint8, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = torch.empty(max(kdt.workspace_bytes(nmax, k, 0) for k in (2, 3, 4)), dtype=torch.uint8, device=dev)
    dur = np.zeros(R)
    for i in range(R):
        n, k = int(ns[i]), int(ks[i])
        torch.cuda.synchronize()
        a = time.perf_counter()
        x = d_in[: n * k].view(n, k)
        x.copy_(views[i], non_blocking=True)
        kdt.build_ws(x, kdt.ROUND_ROBIN, tree=tree[: n * k].view(n, k), perm=perm[:n], dim=dim[:n], status=st,
                     workspace=ws, stream=stream)
        torch.cuda.synchronize()
        dur[i] = time.perf_counter() - a
    fin = np.zeros(R)
    t = 0.0
    for i in range(R):
        t = max(t, float(arrivals[i])) + dur[i]
        fin[i] = t
    fifo_lat = (fin - arrivals) * 1e3
    fifo = {"value": round(total_pts / fin[-1] / 1e6, 3), "unit": "Mpoints/s",
            "p50_ms": round(float(np.percentile(fifo_lat, 50)), 3),
            "p99_ms": round(float(np.percentile(fifo_lat, 99)), 3),
            "busy_s": round(float(dur.sum()), 3)}
    print(f"# fifo: {fifo}", file=sys.stderr, flush=True)

    # each result in the mix equals the request built alone: a sample
    same = True
    with kdt.Server(8 << 30, max_inflight=args.inflight, max_batch_requests=64) as srv:
        pick = list(range(0, R, max(1, R // 24)))[:24]
        tks = [srv.submit(views[i], kdt.ROUND_ROBIN) for i in pick]
        for i, t in zip(pick, tks):
            n, k = int(ns[i]), int(ks[i])
            t_tree, t_perm, t_dim = srv.fetch(t)
            x = views[i].to(dev)
            a_tree, a_perm, a_dim, _ = kdt.build_ws(x, kdt.ROUND_ROBIN)
            torch.cuda.synchronize()
            same = same and bool(torch.equal(t_tree, a_tree) and torch.equal(t_perm, a_perm)
                                 and torch.equal(t_dim, a_dim))
            srv.release(t)
    return {
        "value": round(served, 3), "makespan_s": round(makespan, 4),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)), 3),
                       "p99": round(float(np.percentile(lat, 99)), 3),
                       "mean": round(float(lat.mean()), 3)},
        "device_ms_per_batch": {"p50": round(float(np.percentile(dev_ms, 50)), 3),
                                "p99": round(float(np.percentile(dev_ms, 99)), 3)},
        "mean_batch_requests": round(float(bsz.mean()), 2),
        "offered_Mpts_s": round(total_pts / float(arrivals[-1]) / 1e6, 1),
        "statuses_ok": statuses == {0},
        "fifo": fifo,
        "mix_equals_alone": same,
        "requests": R,
        "points": total_pts,
    }


def cpu_baseline_clouds(pts, offsets, target_s: float):
    """The oracle over whole clouds, in order, until about target_s seconds:
    one cloud per host thread at a time (clouds are independent), and on one
    core for comparison."""
    from concurrent.futures import ThreadPoolExecutor

    import oracle
    threads, model = host_cpu()
    bounds = [(int(offsets[c]), int(offsets[c + 1])) for c in range(len(offsets) - 1)]
    t0 = time.perf_counter()
    done1 = 0
    for a, b in bounds:
        oracle.build(pts[a:b], oracle.RR)
        done1 += b - a
        if time.perf_counter() - t0 > target_s / 4:
            break
    dt1 = time.perf_counter() - t0
    # the C oracle releases the GIL (ctypes), so a thread pool runs clouds in parallel
    t0 = time.perf_counter()
    done = clouds = 0
    with ThreadPoolExecutor(threads) as ex:
        while clouds < len(bounds) and time.perf_counter() - t0 < target_s:
            chunk = bounds[clouds:clouds + 4 * threads]
            list(ex.map(lambda ab: oracle.build(pts[ab[0]:ab[1]], oracle.RR), chunk))
            done += sum(b - a for a, b in chunk)
            clouds += len(chunk)
    dt = time.perf_counter() - t0
    return {"value": round(done / dt / 1e6, 4), "unit": "Mpoints/s", "cores": threads, "kind": "oracle",
            "cpu_model": model, "nproc": os.cpu_count(),
            "single_core": {"value": round(done1 / dt1 / 1e6, 4), "unit": "Mpoints/s",
                            "sample": f"{done1} points of the first clouds, {dt1:.1f} s"},
            "sample": f"the first {clouds} clouds ({done} points) of the same batch, one build each, "
                      f"{threads} clouds at a time on {threads} threads, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="cluster100m")
    ap.add_argument("--n", type=int, default=0)
    ap.add_argument("--k", type=int, default=4)
    ap.add_argument("--variant", choices=["ws", "inplace"], default="ws",
                    help="ws: kdt_build_ws (default); inplace: the low-memory in-place build kdt_build_inplace "
                         "(one int per point; each step first restores the input with a device copy, which "
                         "HIP events leave out of the timed build)")
    ap.add_argument("--no-check", action="store_true", help="skip the full-tree bit-exactness check")
    ap.add_argument("--no-per-cloud", action="store_true",
                    help="batched: skip the comparison with one single build per cloud (for counter runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-profile", action="store_true", help="time without per-kernel events")
    ap.add_argument("--autotune", action="store_true",
                    help="before warm-up, let kdt_tune_batched pick the digit width, tile size and presort grouping for this input")
    ap.add_argument("--requests", type=int, default=2000, help="serving: trace length")
    ap.add_argument("--inflight", type=int, default=4, help="serving: batches on the device at once")
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

    if args.workload == "serving":
        r = run_serving(args)
        cfg = {"workload": "serving", "requests": r["requests"], "points": r["points"],
               "arrivals": "Poisson 2000/s", "k": "uniform {2,3,4}", "n": "log-uniform [1e3, 4e6]",
               "dim_mode": "round_robin", "hbm_budget_GiB": 64, "max_inflight": args.inflight, "seed": 5}
        out = {"metric": METRIC, "value": r["value"], "unit": "Mpoints/s", "n_gpus": 1, "steps": 1,
               "warmup": 0, "ms_per_step": round(r["makespan_s"] * 1e3, 3), "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32 in, u32 ranks", "data": "synthetic",
               "config": cfg, "roofline": None, "cpu_baseline": None, "latency_ms": r["latency_ms"],
               "device_ms_per_batch": r["device_ms_per_batch"], "mean_batch_requests": r["mean_batch_requests"],
               "offered_Mpts_s": r["offered_Mpts_s"], "fifo": r["fifo"], "mix_equals_alone": r["mix_equals_alone"],
               "statuses_ok": r["statuses_ok"]}
        print(json.dumps(out), flush=True)
        return
    pts, mode, cfg = make_workload(args.workload, args.n, args.k)
    if args.workload == "batched4096":
        r = run_batched(args, pts, mode, cfg)
        out = {"metric": METRIC, "value": r["value"], "unit": "Mpoints/s", "n_gpus": 1, "steps": args.steps,
               "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f32 in, u32 ranks", "data": "synthetic",
               "config": cfg, "roofline": r["roofline"], "build": r["build"], "cpu_baseline": r["cpu_baseline"],
               "bit_exact": r["bit_exact"], "per_cloud": r["per_cloud"],
               "batched_vs_per_cloud": r["batched_vs_per_cloud"], "kernels": r["kernels"]}
        print(json.dumps(out), flush=True)
        return
    n, k = pts.shape
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    d_pts = torch.from_numpy(pts).to(dev)
    inplace = args.variant == "inplace"
    tree = torch.empty((n, k), dtype=d_pts.dtype, device=dev)
    perm = torch.empty(n, dtype=torch.int32, device=dev)
    dim = torch.empty(n, dtype=torch.uint8, device=dev)
    status = torch.zeros(1, dtype=torch.int32, device=dev)
    if inplace:
        ws = torch.empty(max(kdt.inplace_workspace_bytes(n, k, mode), 1), dtype=torch.uint8, device=dev)
        cfg["variant"] = "inplace (kdt_build_inplace: one int per point, swap-only)"
        cfg["workspace_bytes"] = int(ws.numel())
    else:
        ws = torch.empty(kdt.workspace_bytes(n, k, mode), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    i32 = pts.dtype == np.int32

    calibration_copy(args, dev)

    if inplace:
        ev = []

        def step():
            tree.copy_(d_pts)                       # restore the input; not part of the timed build
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            kdt.build_inplace(tree, mode, perm=perm, dim=dim, status=status, workspace=ws, stream=stream)
            b.record(stream)
            ev.append((a, b))
    else:
        def step():
            kdt.build_ws(d_pts, mode, tree=tree, perm=perm, dim=dim, status=status, workspace=ws, stream=stream)

    if args.autotune and not inplace:
        import numpy as np
        rb, items, pdims, tms = kdt.tune_batched(d_pts, np.array([0, n], np.uint32), mode, reps=3, workspace=ws)
        cfg["tuned"] = {"radix_bits": rb, "level_items": items, "presort_dims": pdims}
        print(f"# autotune: radix {rb} items {items} presort dims {pdims} ({tms:.3f} ms)", file=sys.stderr, flush=True)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"# warmup done: n={n} k={k} mode={mode}", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    if inplace:
        ev.clear()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if inplace:
        # the builds alone, by the events around each (the restore copies between them excluded)
        elapsed = sum(a.elapsed_time(b) for a, b in ev) / 1e3
    st = int(status.item())
    print(f"# timed {args.steps} steps in {elapsed:.3f} s, status {st}", file=sys.stderr, flush=True)
    ms_per_step = elapsed * 1e3 / args.steps
    value = n * args.steps / elapsed / 1e6

    # the same K steps again with a pair of HIP events around every kernel
    # on the build's stream (per-kernel durations for the roofline); the
    # events add a few microseconds between kernels, so `value` comes from
    # the pass above
    prof = {}
    if not args.no_profile:
        kdt.profile_enable(True)
        kdt.profile_collect()
        for _ in range(args.steps):
            step()
        prof = kdt.profile_collect()
        kdt.profile_enable(False)

    roofline, kernels = kernel_table(prof, args.steps)
    if roofline:
        roofline["traffic"] = dominant_traffic(roofline, cfg["workload"])
    build = build_rates(prof, args.steps, ms_per_step, cfg["workload"])

    bit_exact = None
    if not args.no_check:
        import oracle
        h_perm = perm.cpu().numpy().view(np.uint32)
        t0 = time.perf_counter()
        code, node = oracle.check(pts, h_perm, dim.cpu().numpy(), oracle.WIDEST if mode == kdt.WIDEST else oracle.RR)
        print(f"# checker code {code} node {node} ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
        # the tree's coordinates are the points in perm order, byte for byte
        same_tree = tree.cpu().numpy().tobytes() == np.ascontiguousarray(pts[h_perm]).tobytes()
        bit_exact = bool(code == 0 and same_tree and st == 0)
        print(f"# tree bytes equal points[perm]: {same_tree}", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu else cpu_baseline(pts, mode, args.cpu_seconds)

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32 in, u32 ranks" if i32 else "f32 in, u32 ranks",
        "data": "synthetic",
        "config": cfg,
        "roofline": roofline,
        "build": build,
        "cpu_baseline": cpu,
        "bit_exact": bit_exact,
        "kernels": kernels,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
