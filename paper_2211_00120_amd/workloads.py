"""Seeded synthetic inputs for the k-d tree build.

This module only draws random numbers; it contains none of the build's
arithmetic, so both the GPU path's tests/benchmark and the CPU oracle may use
it.  Every generator uses numpy's PCG64 with an explicit seed and a fixed draw
order, so the same seed always yields the same float32 bytes.

The paper measures on uniformly distributed random points in [0,1]^4
(Sec. 7.1, Table 1); the workloads below follow that and add the duplicate-
heavy, clustered, batched and served mixes the benchmark configurations name.
"""
from __future__ import annotations

import math

import numpy as np


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform(n: int, k: int, seed: int) -> np.ndarray:
    """n points i.i.d. uniform in [0,1)^k, float32."""
    return _rng(seed).random((n, k), dtype=np.float32)


def grid(n: int, k: int, seed: int, levels: int = 8) -> np.ndarray:
    """n points with coordinates drawn from a small integer grid (heavy ties)."""
    return _rng(seed).integers(0, levels, size=(n, k)).astype(np.float32)


def signed_mix(n: int, k: int, seed: int) -> np.ndarray:
    """Values of mixed sign and magnitude, including -0.0, +0.0, subnormals and
    the float32 extremes, to exercise the order-preserving key transform."""
    r = _rng(seed)
    base = r.standard_normal((n, k)).astype(np.float32) * np.float32(1e3)
    specials = np.array([0.0, -0.0, 1e-45, -1e-45, 1.17549435e-38, -1.17549435e-38,
                         3.4028235e38, -3.4028235e38, 1.0, -1.0], dtype=np.float32)
    mask = r.random((n, k)) < 0.3
    picks = specials[r.integers(0, len(specials), size=(n, k))]
    return np.where(mask, picks, base).astype(np.float32)


def int_uniform(n: int, k: int, seed: int) -> np.ndarray:
    """n points i.i.d. uniform over all int32 values (Table 1's int1 rows:
    the paper does not state their distribution), int32."""
    return _rng(seed).integers(-(2 ** 31), 2 ** 31, size=(n, k), dtype=np.int64).astype(np.int32)


def int_grid(n: int, k: int, seed: int, levels: int = 8) -> np.ndarray:
    """int32 points from a small range around 0 (heavy ties, both signs)."""
    return (_rng(seed).integers(0, levels, size=(n, k)) - levels // 2).astype(np.int32)


def int_extremes(n: int, k: int, seed: int) -> np.ndarray:
    """int32 values with the extremes, 0 and -1 mixed into uniform ones, so
    that the key transform and exact extents see both ends of the range."""
    r = _rng(seed)
    base = r.integers(-(2 ** 31), 2 ** 31, size=(n, k), dtype=np.int64)
    specials = np.array([-(2 ** 31), 2 ** 31 - 1, 0, -1, 1, -(2 ** 31) + 1, 2 ** 31 - 2], dtype=np.int64)
    mask = r.random((n, k)) < 0.3
    return np.where(mask, specials[r.integers(0, len(specials), size=(n, k))], base).astype(np.int32)


def cfg_small(seed: int = 1) -> np.ndarray:
    """N=1024 3D points uniform in [0,1)^3 (single build, round robin)."""
    return uniform(1024, 3, seed)


def cfg_mixture(n: int = 10_000_000, seed: int = 2) -> np.ndarray:
    """Half uniform in [0,1)^3, half from an 8-component isotropic Gaussian
    mixture (sigma 0.01), all coordinates rounded to the 2^-16 grid so that
    many coordinate values repeat."""
    r = _rng(seed)
    h = n // 2
    u = r.random((h, 3), dtype=np.float32).astype(np.float64)
    centres = r.uniform(0.1, 0.9, (8, 3))
    comp = r.integers(0, 8, n - h)
    g = centres[comp] + r.normal(0.0, 0.01, (n - h, 3))
    x = np.concatenate([u, g], axis=0)
    x = np.rint(x * 65536.0) / 65536.0
    return x.astype(np.float32)


def cfg_cluster4d(n: int = 100_000_000, seed: int = 3, cluster: int = 1 << 20) -> np.ndarray:
    """N points in 4D: n - cluster uniform in [0,1)^4 plus a dense cluster of
    `cluster` points (Gaussian, sigma 2^-10, centre uniform in [0.25,0.75)^4).
    Used with the split-widest-dimension rule."""
    r = _rng(seed)
    m = max(n - cluster, 0)
    c = min(cluster, n)
    out = np.empty((n, 4), dtype=np.float32)
    out[:m] = r.random((m, 4), dtype=np.float32)
    centre = r.uniform(0.25, 0.75, 4)
    out[m:] = (centre + r.normal(0.0, 2.0 ** -10, (c, 4))).astype(np.float32)
    return out


def cfg_batched_sizes(clouds: int = 4096, seed: int = 4, lo: int = 64, hi: int = 262144) -> np.ndarray:
    """Cloud sizes log-uniform in [lo, hi]."""
    r = _rng(seed)
    n = np.floor(np.exp(r.uniform(math.log(lo), math.log(hi), clouds))).astype(np.int64)
    return np.clip(n, lo, hi)


def cfg_batched(clouds: int = 4096, seed: int = 4, lo: int = 64, hi: int = 262144, k: int = 3):
    """`clouds` independent 3D clouds concatenated; returns (points, offsets)
    with offsets[c]..offsets[c+1] the rows of cloud c.  Each cloud is uniform
    in its own random box (corner in [-1000,1000)^3, extents log-uniform in
    [1e-2, 1e2])."""
    r = _rng(seed)
    n = np.floor(np.exp(r.uniform(math.log(lo), math.log(hi), clouds))).astype(np.int64)
    n = np.clip(n, lo, hi)
    offsets = np.zeros(clouds + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(n)
    pts = np.empty((int(offsets[-1]), k), dtype=np.float32)
    for c in range(clouds):
        corner = r.uniform(-1000.0, 1000.0, k)
        ext = np.exp(r.uniform(math.log(1e-2), math.log(1e2), k))
        a, b = int(offsets[c]), int(offsets[c + 1])
        pts[a:b] = (corner + ext * r.random((b - a, k))).astype(np.float32)
    return pts, offsets


def cfg_serving_trace(requests: int = 20000, seed: int = 5, rate: float = 2000.0,
                      nmin: int = 1000, nmax: int = 4_000_000):
    """Open-loop request trace: Poisson arrivals at `rate` per second, each
    request with k uniform in {2,3,4} and N log-uniform in [nmin, nmax].
    Returns (arrival_seconds, k, n, point_seeds); the points of request i are
    uniform(n[i], k[i], point_seeds[i])."""
    r = _rng(seed)
    arrivals = np.cumsum(r.exponential(1.0 / rate, requests))
    ks = r.integers(2, 5, requests)
    ns = np.floor(np.exp(r.uniform(math.log(nmin), math.log(nmax), requests))).astype(np.int64)
    seeds = r.integers(0, 2**31 - 1, requests)
    return arrivals, ks, ns, seeds
