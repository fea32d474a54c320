"""CPU oracle for the left-balanced k-d tree build (arXiv 2211.00120).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check in
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The product
library (``paper_2211_00120_amd``) never imports, links or runs anything here,
and nothing here imports the product package.

The arithmetic lives in ``kdt_oracle.c`` (plain C, compiled with gcc into
``libkdt_oracle.so``); this module only marshals numpy arrays through ctypes.
See the header of ``kdt_oracle.c`` for the definition being implemented and
the paper passages it follows (Obs. 2.1, Sec. 2, Sec. 3.1, Sec. 6).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kdt_oracle.c")
_LIB = os.path.join(_HERE, "libkdt_oracle.so")

RR = 0
WIDEST = 1

_lib = None


def build_oracle() -> str:
    """Compile kdt_oracle.c with gcc (no fast-math: float32 compares and the
    float32 extent subtraction must be exact IEEE)."""
    tmp = _LIB + ".tmp"
    subprocess.run(
        ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
         "-ffp-contract=off", "-Wall", "-Wextra", "-o", tmp, _SRC],
        check=True,
    )
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build_oracle()
    lib = ctypes.CDLL(_LIB)
    build_args = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_void_p]
    check_args = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, ctypes.c_void_p,
                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]
    for suffix in ("", "_i32"):
        f = getattr(lib, "kdt_oracle_build" + suffix)
        f.restype, f.argtypes = ctypes.c_int, build_args
        f = getattr(lib, "kdt_oracle_build_par" + suffix)
        f.restype, f.argtypes = ctypes.c_int, build_args + [ctypes.c_int]
        f = getattr(lib, "kdt_oracle_check" + suffix)
        f.restype, f.argtypes = ctypes.c_int, check_args
    lib.kdt_oracle_subtree_size.restype = ctypes.c_uint64
    lib.kdt_oracle_subtree_size.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    _lib = lib
    return lib


def _points(points):
    """The points as a C-contiguous (N, k) array, and the suffix of the C
    functions for their type: float32 (""), int32 ("_i32")."""
    p = np.asarray(points)
    if p.dtype == np.int32:
        p, suffix = np.ascontiguousarray(p), "_i32"
    else:
        p, suffix = np.ascontiguousarray(p, dtype=np.float32), ""
    if p.ndim != 2 or not (1 <= p.shape[1] <= 4):
        raise ValueError("points must be an (N, k) float32 or int32 array with 1 <= k <= 4")
    return p, suffix


def build(points, mode: int = RR, threads: int = 1):
    """Return (perm, dim): perm[s] is the original index of the point at
    level-order node s, dim[s] its split dimension.  The tree's points are
    points[perm].  points: float32 or int32.  threads > 1 runs the same
    recursion with subtrees as OpenMP tasks (same output)."""
    p, suffix = _points(points)
    n, k = p.shape
    perm = np.zeros(n, dtype=np.uint32)
    dim = np.zeros(n, dtype=np.uint8)
    lib = _load()
    if threads > 1:
        rc = getattr(lib, "kdt_oracle_build_par" + suffix)(p.ctypes.data, n, k, int(mode), perm.ctypes.data,
                                                          dim.ctypes.data, int(threads))
    else:
        rc = getattr(lib, "kdt_oracle_build" + suffix)(p.ctypes.data, n, k, int(mode), perm.ctypes.data,
                                                      dim.ctypes.data)
    if rc != 0:
        raise RuntimeError(f"kdt_oracle_build failed with code {rc}")
    return perm, dim


def check(points, perm, dim, mode: int = RR):
    """Verify (perm, dim) against the split rule and the k-d order at every
    node/ancestor pair.  Returns (code, node); code 0 means it is the tree.
    Large inputs are checked on every host core (OpenMP)."""
    p, suffix = _points(points)
    n, k = p.shape
    perm = np.ascontiguousarray(perm, dtype=np.uint32)
    dim = np.ascontiguousarray(dim, dtype=np.uint8)
    if perm.shape != (n,) or dim.shape != (n,):
        raise ValueError("perm and dim must have N entries")
    bad = ctypes.c_uint64(0)
    rc = getattr(_load(), "kdt_oracle_check" + suffix)(p.ctypes.data, n, k, int(mode), perm.ctypes.data,
                                                       dim.ctypes.data, ctypes.byref(bad))
    if rc < 0:
        raise RuntimeError(f"kdt_oracle_check failed with code {rc}")
    return rc, int(bad.value)


def subtree_size(s: int, n: int) -> int:
    """Direct-count subtree size used inside the oracle."""
    return int(_load().kdt_oracle_subtree_size(s, n))
