"""Compile the gfx950 HIP sources into the in-tree libkdt.so."""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["kdt_kernels.hip", "kdt_tail.hip", "kdt_level_k1.hip", "kdt_level_k2.hip", "kdt_level_k3.hip",
           "kdt_level_k4.hip", "kdt_api.hip", "kdt_plan.cpp", "kdt_server.hip", "kdt_inplace.hip"]
LIB = os.path.join(HERE, "libkdt.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    # no packed-FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # float32 subnormals are ordered by value: no flush to zero
    "-fno-gpu-flush-denormals-to-zero",
    "-Wall",
]


def build_library(verbose: bool = False, out: str = LIB, defines=(), sources_dir: str = CSRC, jobs: int = 0) -> str:
    """Compile every source to an object in parallel, then link the shared
    library.  `defines` are extra -D tuning knobs (e.g. "KDT_LB_WINDOW=8"),
    `out` the path of the shared object."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tag = hashlib.sha256(("|".join(defines) + out).encode()).hexdigest()[:10]
    objdir = os.path.join(tempfile.gettempdir(), f"kdt_build_{os.getpid()}_{tag}")
    os.makedirs(objdir, exist_ok=True)
    dflags = [f"-D{d}" for d in defines]
    cmds = []
    objs = []
    for s in SOURCES:
        obj = os.path.join(objdir, s + ".o")
        objs.append(obj)
        cmds.append([hipcc, *HIPCC_FLAGS, *dflags, "-c", os.path.join(sources_dir, s), "-o", obj])
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 1)))
    with ThreadPoolExecutor(jobs) as ex:
        for cmd, r in zip(cmds, ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds)):
            if verbose:
                print(" ".join(cmd), flush=True)
            if r.returncode != 0:
                sys.stderr.write(r.stdout + r.stderr)
                raise subprocess.CalledProcessError(r.returncode, cmd)
            if r.stderr.strip():
                sys.stderr.write(r.stderr)
    tmp = out + ".tmp"
    link = [hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, out)
    shutil.rmtree(objdir, ignore_errors=True)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
