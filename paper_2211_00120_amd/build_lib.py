"""Compile the gfx950 HIP sources into the in-tree libkdt.so."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
SOURCES = ["kdt_kernels.hip", "kdt_tail.hip", "kdt_api.hip"]
LIB = os.path.join(HERE, "libkdt.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed-FP32 instructions in any generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # float32 subnormals are ordered by value: no flush to zero
    "-fno-gpu-flush-denormals-to-zero",
    "-Wall",
]


def build_library(verbose: bool = False, out: str = LIB, defines=(), sources_dir: str = CSRC) -> str:
    """Compile the library; `defines` are extra -D tuning knobs (e.g.
    "KDT_LEVEL_ITEMS=12"), `out` the path of the shared object."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = out + ".tmp"
    cmd = [hipcc, *HIPCC_FLAGS, *[f"-D{d}" for d in defines], *[os.path.join(sources_dir, s) for s in SOURCES],
           "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build_library(verbose=True))
