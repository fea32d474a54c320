"""GPU parity: the HIP build through the C ABI against the CPU oracle.

The build is integer/permutation work on float32 inputs, so the bar is bit
equality of perm, dim and the tree's coordinates with the oracle.  At sizes
the oracle builds in seconds the comparison is element by element; at the
full benchmark sizes the oracle's checker verifies the GPU tree at every node
(k-d order against every ancestor, split rule, permutation), which by the
uniqueness of the tree under the (coordinate, index) order is the same as
equality with the oracle's tree.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2211_00120_amd import kdt, workloads  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _gpu_build(pts, mode):
    t = torch.from_numpy(np.ascontiguousarray(pts)).to(DEV)
    tree, perm, dim, status = kdt.build_ws(t, mode)
    torch.cuda.synchronize()
    return (tree.cpu().numpy(), perm.cpu().numpy().astype(np.uint32), dim.cpu().numpy(),
            int(status.item()))


def _omode(mode):
    return oracle.WIDEST if mode == kdt.WIDEST else oracle.RR


def _assert_same(pts, mode, label):
    _say(f"case {label}: n={pts.shape[0]} k={pts.shape[1]} mode={mode}")
    tree, perm, dim, status = _gpu_build(pts, mode)
    assert status == kdt.OK, f"{label}: device status {status:#x}"
    perm_o, dim_o = oracle.build(pts, _omode(mode))
    bad = np.flatnonzero(perm != perm_o)
    assert bad.size == 0, f"{label}: perm differs at {bad.size} nodes, first {bad[:5]}"
    assert np.array_equal(dim, dim_o), f"{label}: dim differs"
    assert tree.tobytes() == np.ascontiguousarray(pts[perm_o]).tobytes(), f"{label}: tree bytes differ"


GENS = {
    "uniform": lambda n, k, s: workloads.uniform(n, k, s),
    "grid": lambda n, k, s: workloads.grid(n, k, s, levels=7),
    "signed": lambda n, k, s: workloads.signed_mix(n, k, s),
}

SMALL_N = [1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 15, 16, 17, 31, 32, 33, 63, 64, 100, 127, 128, 129, 255, 256, 257,
           1000, 1023, 1024, 1025]
MID_N = [2047, 2048, 2049, 4095, 4096, 4097, 6000, 8191, 8192, 12345, 65535, 65536, 65537, 100003]
BIG_N = [300000, 1048575, 1048576, 2000001]


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("n", SMALL_N)
def test_small_sweep(n, k, mode):
    gen = ["uniform", "grid", "signed"][(n + k) % 3]
    _assert_same(GENS[gen](n, k, 1000 + n * 7 + k), mode, f"small-{gen}")


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
@pytest.mark.parametrize("k", [2, 3, 4])
@pytest.mark.parametrize("n", MID_N)
def test_mid_sweep(n, k, mode):
    gen = ["uniform", "grid", "signed"][(n + k) % 3]
    _assert_same(GENS[gen](n, k, 2000 + n + k), mode, f"mid-{gen}")


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
@pytest.mark.parametrize("n", BIG_N)
def test_big_sweep(n, mode):
    k = 3 if mode == kdt.ROUND_ROBIN else 4
    gen = "grid" if n % 2 else "uniform"
    _assert_same(GENS[gen](n, k, 3000 + n), mode, f"big-{gen}")


def test_config_small_1024():
    _assert_same(workloads.cfg_small(1), kdt.ROUND_ROBIN, "cfg-1024")


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
def test_identical_points(mode):
    pts = np.full((5000, 3), 0.25, np.float32)
    _assert_same(pts, mode, "identical")


def _digit_pattern_points(n, seed):
    """Four coordinates whose order-preserving keys differ in chosen bytes
    only: powers of four (only the top byte varies), 1 + m * 2^-15 (only
    byte 1 varies), a constant, and uniform values (every byte varies), so
    that the presort skips different digit passes in each dimension."""
    r = np.random.default_rng(seed)
    pts = np.empty((n, 4), np.float32)
    pts[:, 0] = np.float32(4.0) ** r.integers(-6, 7, n).astype(np.float32)
    pts[:, 1] = np.float32(1.0) + r.integers(0, 256, n).astype(np.float32) * np.float32(2.0 ** -15)
    pts[:, 2] = np.float32(0.75)
    pts[:, 3] = r.random(n, dtype=np.float32)
    return pts


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
def test_constant_digit_passes(mode):
    pts = _digit_pattern_points(100003, 31)
    for cols in ([0, 1, 2, 3], [2, 0, 1], [1, 2]):
        _assert_same(np.ascontiguousarray(pts[:, cols]), mode, f"digit-pattern-{cols}")


@pytest.mark.parametrize("pdims", [0, 1, 2])
@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
@pytest.mark.parametrize("k", [2, 3, 4])
def test_rank_layouts(pdims, layout, mode, k):
    """Both rank-table layouts (the last presort passes scatter point-major
    records; or per-role arrays by root position, the root's role sorted
    first) build the oracle's tree, whatever number of dimensions share a
    presort launch (0: the planner's, all of them).  The planner picks the
    layout by the table's size, so each is forced through the tuning table
    of this size class."""
    n = 150_001
    bits = (n - 1).bit_length()
    pts = workloads.grid(n, k, 300 + k, levels=9)
    kdt.tuning_clear()
    try:
        kdt.tuning_set(k, mode, bits, 0, 0, layout, pdims)
        assert kdt.tuning_get(k, mode, bits) == (0, 0, layout, pdims)
        _assert_same(pts, mode, f"rank-layout-{layout}-presort-dims-{pdims}")
    finally:
        kdt.tuning_clear()


@pytest.mark.parametrize("pdims", [0, 1])
@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("k", [2, 3, 4])
def test_rank_layouts_widest_root_not_first(pdims, layout, k):
    """Split-widest with the root splitting in the last dimension (stretched
    points): presort role 0 is that dimension and the other roles map past
    it; both layouts build the oracle's tree."""
    n = 150_001
    bits = (n - 1).bit_length()
    pts = workloads.uniform(n, k, 700 + k)
    pts[:, k - 1] *= np.float32(2.5)
    kdt.tuning_clear()
    try:
        kdt.tuning_set(k, kdt.WIDEST, bits, 0, 0, layout, pdims)
        _assert_same(pts, kdt.WIDEST, f"rank-layout-{layout}-root-dim-{k - 1}")
    finally:
        kdt.tuning_clear()


def test_k1_widest_and_rr_equal():
    pts = workloads.grid(7777, 1, 5, levels=50)
    _assert_same(pts, kdt.ROUND_ROBIN, "k1-rr")
    _assert_same(pts, kdt.WIDEST, "k1-widest")


def test_nonfinite_sets_status():
    pts = workloads.uniform(5000, 3, 8)
    pts[1234, 1] = np.nan
    _say("case nonfinite")
    *_, status = _gpu_build(pts, kdt.ROUND_ROBIN)
    assert status & kdt.ENONFINITE
    pts[1234, 1] = np.inf
    *_, status = _gpu_build(pts, kdt.WIDEST)
    assert status & kdt.ENONFINITE


def test_empty_input():
    _say("case empty")
    t = torch.zeros((0, 3), dtype=torch.float32, device=DEV)
    tree, perm, dim, status = kdt.build_ws(t, kdt.ROUND_ROBIN)
    torch.cuda.synchronize()
    assert tree.numel() == 0 and perm.numel() == 0 and int(status.item()) == 0


def test_deterministic_repeats():
    pts = workloads.cfg_mixture(n=400000, seed=2)
    _say("case repeats")
    t = torch.from_numpy(pts).to(DEV)
    ws = torch.empty(kdt.workspace_bytes(*pts.shape, kdt.ROUND_ROBIN), dtype=torch.uint8, device=DEV)
    ref = None
    for _ in range(10):
        tree, perm, dim, status = kdt.build_ws(t, kdt.ROUND_ROBIN, workspace=ws)
        torch.cuda.synchronize()
        assert int(status.item()) == 0
        cur = perm.cpu().numpy()
        if ref is None:
            ref = cur
        assert np.array_equal(cur, ref)
    perm_o, _ = oracle.build(pts, oracle.RR)
    assert np.array_equal(ref.astype(np.uint32), perm_o)


def test_in_place_build_matches():
    pts = workloads.uniform(123457, 4, 12)
    _say("case in-place")
    t = torch.from_numpy(pts).to(DEV)
    kdt.build(t, kdt.WIDEST)
    torch.cuda.synchronize()
    perm_o, _ = oracle.build(pts, oracle.WIDEST)
    assert t.cpu().numpy().tobytes() == pts[perm_o].tobytes()


def test_optional_outputs():
    pts = workloads.uniform(50000, 3, 13)
    _say("case optional outputs")
    t = torch.from_numpy(pts).to(DEV)
    perm_o, dim_o = oracle.build(pts, oracle.WIDEST)
    tree, perm, dim, status = kdt.build_ws(t, kdt.WIDEST, want_tree=False, want_dim=False)
    torch.cuda.synchronize()
    assert tree is None and dim is None
    assert np.array_equal(perm.cpu().numpy().astype(np.uint32), perm_o)
    tree, perm, dim, status = kdt.build_ws(t, kdt.WIDEST, want_perm=False)
    torch.cuda.synchronize()
    assert tree.cpu().numpy().tobytes() == pts[perm_o].tobytes()
    assert np.array_equal(dim.cpu().numpy(), dim_o)


def _check_full(pts, mode, label):
    """Full-size parity: the oracle's checker on every node (k-d order against
    every ancestor, split rule, permutation), which by the uniqueness of the
    tree is equality with the oracle's tree, and the tree's coordinates
    compared byte for byte with the points in perm order."""
    _say(f"case {label}: n={pts.shape[0]} k={pts.shape[1]} mode={mode} (checker)")
    tree, perm, dim, status = _gpu_build(pts, mode)
    assert status == kdt.OK, f"device status {status:#x}"
    code, node = oracle.check(pts, perm, dim, _omode(mode))
    assert code == 0, f"{label}: checker code {code} at node {node}"
    assert tree.tobytes() == np.ascontiguousarray(pts[perm]).tobytes(), f"{label}: tree bytes differ"


def test_config_mixture_10m():
    _check_full(workloads.cfg_mixture(), kdt.ROUND_ROBIN, "cfg-10M-mixture")


@pytest.mark.skipif(os.environ.get("KDT_SKIP_100M") == "1", reason="100M case disabled by KDT_SKIP_100M")
def test_config_cluster_100m_widest():
    _check_full(workloads.cfg_cluster4d(), kdt.WIDEST, "cfg-100M-widest")


@pytest.mark.parametrize("n", [1_000_000, 10_000_000,
                               pytest.param(100_000_000, marks=pytest.mark.skipif(
                                   os.environ.get("KDT_SKIP_100M") == "1",
                                   reason="100M case disabled by KDT_SKIP_100M"))])
def test_uniform4d_round_robin_table1(n):
    """The workload of the paper's Table 1 (uniform points in [0,1)^4, round
    robin) at 1e6, 1e7 and 1e8 points."""
    _check_full(workloads.uniform(n, 4, seed=7), kdt.ROUND_ROBIN, f"uniform4d-{n}")


_RUN_1E9 = os.environ.get("KDT_RUN_1E9") == "1"


@pytest.mark.skipif(not _RUN_1E9, reason="1e9-point builds take minutes of host time: set KDT_RUN_1E9=1")
@pytest.mark.parametrize("kind", ["float4", "int1"])
def test_one_billion_points(kind):
    """Table 1's last column: 10^9 points, round robin (uniform [0,1)^4
    float32, and int32 with k = 1).  Checked by the oracle's checker on every
    node and the tree's bytes against the points in perm order."""
    n = 1_000_000_000
    if kind == "float4":
        pts = workloads.uniform(n, 4, seed=7)
    else:
        pts = workloads.int_uniform(n, 1, seed=11)
    _check_full(pts, kdt.ROUND_ROBIN, f"1e9-{kind}")
