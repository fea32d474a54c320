"""kdt_build_static (the entry point that allocates nothing: its workspace is
the library's fixed per-device array) against kdt_build_ws on the same
inputs, through the C ABI: two calls in a row, the second on a smaller
input, so the second reuses the array after the first left it dirty; both
split rules; sizes beyond the array are refused on the host."""
import ctypes
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


def _host(*ts):
    torch.cuda.synchronize()
    return [t.cpu().numpy() for t in ts]


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
@pytest.mark.parametrize("k", [1, 3, 4])
def test_static_equals_workspace_build_twice(k, mode):
    # the largest n whose workspace fits, then a smaller one (ragged sizes)
    lib = kdt.lib()
    lo, hi = 0, 1 << 22
    while lo < hi:
        m = (lo + hi + 1) // 2
        if lib.kdt_workspace_bytes(m, k, mode) <= kdt.STATIC_WS_BYTES:
            lo = m
        else:
            hi = m - 1
    for n, seed in ((lo, 41 + k), (100_003, 42 + k)):
        _say(f"case static: n={n} k={k} mode={mode}")
        pts = workloads.grid(n, k, seed, levels=300) if seed % 2 else workloads.uniform(n, k, seed)
        t = torch.from_numpy(pts).to(DEV)
        ref = _host(*kdt.build_ws(t, mode))
        got = _host(*kdt.build_static(t, mode))
        assert int(got[3][0]) == kdt.OK and int(ref[3][0]) == kdt.OK
        assert np.array_equal(got[1], ref[1]), "perm differs from kdt_build_ws"
        assert np.array_equal(got[2], ref[2]), "dim differs from kdt_build_ws"
        assert got[0].tobytes() == ref[0].tobytes(), "tree differs from kdt_build_ws"
    # the last one also against the oracle
    perm_o, dim_o = oracle.build(pts, oracle.WIDEST if mode == kdt.WIDEST else oracle.RR)
    assert np.array_equal(got[1].view(np.uint32), perm_o) and np.array_equal(got[2], dim_o)


def test_static_small_and_status():
    """Trees built whole in one workgroup, N = 0 and 1, and the non-finite
    flag, each right after a larger build."""
    for n in (5000, 0, 1, 2047, 3):
        _say(f"case static-small: n={n}")
        pts = workloads.uniform(n, 3, 50 + n)
        t = torch.from_numpy(pts).to(DEV)
        ref = _host(*kdt.build_ws(t, kdt.ROUND_ROBIN))
        got = _host(*kdt.build_static(t, kdt.ROUND_ROBIN))
        assert int(got[3][0]) == kdt.OK
        assert np.array_equal(got[1], ref[1]) and got[0].tobytes() == ref[0].tobytes()
    pts = workloads.uniform(30000, 3, 60)
    pts[123, 0] = np.inf
    *_, st = _host(*kdt.build_static(torch.from_numpy(pts).to(DEV), kdt.WIDEST))
    assert int(st[0]) & kdt.ENONFINITE


def test_static_rejects_sizes_beyond_the_array():
    lib = kdt.lib()
    fake = ctypes.c_void_p(0x1000)
    n = 4_000_000
    assert lib.kdt_workspace_bytes(n, 4, 0) > kdt.STATIC_WS_BYTES
    assert lib.kdt_build_static(fake, n, 4, 0, None, None, None, None, None) == kdt.EINVAL
    assert "static" in kdt.last_error()
    assert lib.kdt_build_static(fake, 10, 5, 0, None, None, None, None, None) == kdt.EINVAL
