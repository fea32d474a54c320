"""GPU parity for int32 coordinates (Table 1's int1 rows; Sec. 7.2's point
type) and for the payload permutation, through the C ABI, against the CPU
oracle's int32 build: perm, dim and the tree's words compared bytewise at
sizes the oracle builds quickly, the oracle's checker plus a full byte
compare of the tree at the Table 1 sizes."""
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


def _omode(mode):
    return oracle.WIDEST if mode == kdt.WIDEST else oracle.RR


def _gpu(pts, mode):
    t = torch.from_numpy(np.ascontiguousarray(pts)).to(DEV)
    tree, perm, dim, status = kdt.build_ws(t, mode)
    torch.cuda.synchronize()
    return tree.cpu().numpy(), perm.cpu().numpy().view(np.uint32), dim.cpu().numpy(), int(status.item())


def _same(pts, mode, label):
    _say(f"case {label}: n={pts.shape[0]} k={pts.shape[1]} mode={mode}")
    tree, perm, dim, status = _gpu(pts, mode)
    assert status == kdt.OK, f"{label}: status {status:#x}"
    assert tree.dtype == np.int32
    perm_o, dim_o = oracle.build(pts, _omode(mode))
    bad = np.flatnonzero(perm != perm_o)
    assert bad.size == 0, f"{label}: perm differs at {bad.size} nodes, first {bad[:5]}"
    assert np.array_equal(dim, dim_o), f"{label}: dim differs"
    assert tree.tobytes() == np.ascontiguousarray(pts[perm_o]).tobytes(), f"{label}: tree differs"


GENS = {
    "uniform": lambda n, k, s: workloads.int_uniform(n, k, s),
    "grid": lambda n, k, s: workloads.int_grid(n, k, s, levels=9),
    "extremes": lambda n, k, s: workloads.int_extremes(n, k, s),
}


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 100, 1023, 2047, 2048, 2049, 6000, 65537, 300001])
def test_i32_sweep(n, k, mode):
    gen = ["uniform", "grid", "extremes"][(n + k) % 3]
    _same(GENS[gen](n, k, 700 + n + k), mode, f"i32-{gen}")


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
def test_i32_identical_and_extreme_boxes(mode):
    _same(np.full((5000, 3), -7, np.int32), mode, "i32-identical")
    # x spans all of int32 (an int32 subtraction would wrap), y 2^24 + 1, z 2^24
    r = np.random.default_rng(3)
    pts = np.stack([r.integers(-(2 ** 31), 2 ** 31, 40000), r.integers(0, 2 ** 24 + 2, 40000),
                    r.integers(0, 2 ** 24 + 1, 40000)], axis=1).astype(np.int32)
    pts[0] = [-(2 ** 31), 0, 0]
    pts[1] = [2 ** 31 - 1, 2 ** 24 + 1, 2 ** 24]
    _same(pts, mode, "i32-extreme-extents")


def test_i32_batched_equals_oracle():
    sizes = [0, 1, 5, 2000, 2049, 9000, 70000, 3]
    clouds = [workloads.int_extremes(n, 3, 900 + i) if i % 2 else workloads.int_grid(n, 3, 900 + i, levels=33)
              for i, n in enumerate(sizes)]
    pts = np.ascontiguousarray(np.concatenate(clouds, axis=0))
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.uint32)
    for mode in (kdt.ROUND_ROBIN, kdt.WIDEST):
        _say(f"case i32-batched mode={mode}")
        t = torch.from_numpy(pts).to(DEV)
        tree, perm, dim, status = kdt.build_batched(t, offsets, mode)
        torch.cuda.synchronize()
        assert int(status.item()) == kdt.OK
        tree, perm, dim = tree.cpu().numpy(), perm.cpu().numpy().view(np.uint32), dim.cpu().numpy()
        for c, (a, b) in enumerate(zip(offsets[:-1], offsets[1:])):
            p_o, d_o = oracle.build(pts[a:b], _omode(mode))
            assert np.array_equal(perm[a:b], p_o) and np.array_equal(dim[a:b], d_o), f"cloud {c}"
            assert tree[a:b].tobytes() == pts[a:b][p_o].tobytes(), f"cloud {c}"


@pytest.mark.parametrize("stride", [1, 3, 4, 12, 16, 48, 7])
def test_payload_follows_the_tree(stride):
    """A per-point payload of any record size lands in tree order."""
    n = 100_003
    pts = workloads.uniform(n, 3, 31)
    _say(f"case payload stride={stride}")
    t = torch.from_numpy(pts).to(DEV)
    _, perm, _, status = kdt.build_ws(t, kdt.WIDEST)
    payload = np.random.default_rng(stride).integers(0, 256, size=(n, stride), dtype=np.uint8)
    out = kdt.permute_payload(perm, torch.from_numpy(payload).to(DEV), status=status)
    torch.cuda.synchronize()
    assert int(status.item()) == kdt.OK
    h_perm = perm.cpu().numpy().view(np.uint32)
    assert out.cpu().numpy().tobytes() == payload[h_perm].tobytes()


def test_payload_out_of_range_index_is_flagged():
    perm = torch.tensor([2, 0, 7, 1], dtype=torch.int32, device=DEV)     # 7 >= n
    payload = torch.arange(16, dtype=torch.float32, device=DEV).view(4, 4)
    out = torch.full((4, 4), -1.0, device=DEV)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    kdt.permute_payload(perm, payload, out=out, status=status)
    torch.cuda.synchronize()
    assert int(status.item()) & kdt.STATUS_INTERNAL_BIT
    got = out.cpu().numpy()
    assert np.array_equal(got[[0, 1, 3]], payload.cpu().numpy()[[2, 0, 1]])
    assert (got[2] == -1.0).all()                                         # left unwritten


@pytest.mark.parametrize("n", [1_000_000, 10_000_000,
                               pytest.param(100_000_000, marks=pytest.mark.skipif(
                                   os.environ.get("KDT_SKIP_100M") == "1",
                                   reason="100M case disabled by KDT_SKIP_100M"))])
def test_int1_table1(n):
    """Table 1's int1 workload (k = 1): the checker on every node plus a byte
    compare of the tree."""
    pts = workloads.int_uniform(n, 1, seed=8)
    _say(f"case int1: n={n}")
    tree, perm, dim, status = _gpu(pts, kdt.ROUND_ROBIN)
    assert status == kdt.OK
    code, node = oracle.check(pts, perm, dim, oracle.RR)
    assert code == 0, f"checker code {code} at node {node}"
    assert tree.tobytes() == np.ascontiguousarray(pts[perm]).tobytes()
