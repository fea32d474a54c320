"""GPU parity of the batched build (kdt_build_batched) through the C ABI.

Each cloud of a batch must come out exactly as the oracle builds it alone
(perm local to the cloud, dim, tree bytes); at the full 4096-cloud size every
cloud is compared with its own single build on the GPU and checked at every
node by the oracle's checker, and a sample of clouds is compared with the
oracle directly.  A HIP-graph capture of the batched call is replayed with new
inputs and each replay is compared with the oracle.
"""
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


def _concat(clouds):
    k = clouds[0].shape[1]
    offsets = np.zeros(len(clouds) + 1, np.uint64)
    offsets[1:] = np.cumsum([c.shape[0] for c in clouds])
    pts = np.concatenate(clouds, axis=0) if offsets[-1] else np.zeros((0, k), np.float32)
    return np.ascontiguousarray(pts, dtype=np.float32), offsets


def _run_batched(pts, offsets, mode):
    t = torch.from_numpy(pts).to(DEV)
    tree, perm, dim, status = kdt.build_batched(t, offsets, mode)
    torch.cuda.synchronize()
    return (tree.cpu().numpy(), perm.cpu().numpy().astype(np.uint32), dim.cpu().numpy(), int(status.item()))


def _assert_cloud(pts, offsets, c, tree, perm, dim, mode, label):
    a, b = int(offsets[c]), int(offsets[c + 1])
    if a == b:
        return
    cp = pts[a:b]
    perm_o, dim_o = oracle.build(cp, _omode(mode))
    bad = np.flatnonzero(perm[a:b] != perm_o)
    assert bad.size == 0, f"{label}: cloud {c} (n={b - a}) perm differs at {bad.size} nodes, first {bad[:5]}"
    assert np.array_equal(dim[a:b], dim_o), f"{label}: cloud {c} dim differs"
    assert tree[a:b].tobytes() == cp[perm_o].tobytes(), f"{label}: cloud {c} tree bytes differ"


MIXED_SIZES = [0, 1, 2, 3, 100, 2047, 2048, 2049, 0, 5000, 70001, 1, 4096, 300000, 17, 65536, 12345, 2]


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_batched_mixed_sizes(k, mode):
    rng = np.random.default_rng(10 + k)
    clouds = []
    for i, n in enumerate(MIXED_SIZES):
        gen = [workloads.uniform, workloads.signed_mix, lambda n_, k_, s_: workloads.grid(n_, k_, s_, levels=9)][i % 3]
        clouds.append(gen(n, k, int(rng.integers(1 << 30))))
    pts, offsets = _concat(clouds)
    _say(f"case batched-mixed k={k} mode={mode} clouds={len(clouds)} n={pts.shape[0]}")
    tree, perm, dim, status = _run_batched(pts, offsets, mode)
    assert status == kdt.OK
    for c in range(len(clouds)):
        _assert_cloud(pts, offsets, c, tree, perm, dim, mode, "mixed")


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
def test_batched_single_cloud_equals_single_build(mode):
    pts = workloads.cfg_mixture(n=200003, seed=21)
    offsets = np.array([0, pts.shape[0]], np.uint64)
    _say(f"case batched-one-cloud mode={mode}")
    tree, perm, dim, status = _run_batched(pts, offsets, mode)
    assert status == kdt.OK
    _assert_cloud(pts, offsets, 0, tree, perm, dim, mode, "one-cloud")


def test_batched_constant_digit_passes():
    """Clouds whose keys leave different presort digits constant (powers of
    four, 1 + m * 2^-15, a constant coordinate) beside uniform clouds: each
    cloud skips its own passes and still equals the oracle's build."""
    r = np.random.default_rng(33)
    clouds = []
    for i, n in enumerate([70000, 3000, 150000, 9000, 40000, 2500]):
        c = r.random((n, 3), dtype=np.float32)
        if i % 3 == 0:
            c[:, 0] = np.float32(4.0) ** r.integers(-6, 7, n).astype(np.float32)
        if i % 3 == 1:
            c[:, 1] = np.float32(1.0) + r.integers(0, 256, n).astype(np.float32) * np.float32(2.0 ** -15)
            c[:, 2] = np.float32(-3.5)
        clouds.append(c)
    pts, offsets = _concat(clouds)
    for mode in (kdt.ROUND_ROBIN, kdt.WIDEST):
        _say(f"case batched-digit-patterns mode={mode}")
        tree, perm, dim, status = _run_batched(pts, offsets, mode)
        assert status == kdt.OK
        for c in range(len(clouds)):
            _assert_cloud(pts, offsets, c, tree, perm, dim, mode, "digit-patterns")


def test_batched_only_small_clouds():
    clouds = [workloads.uniform(n, 3, 50 + n) for n in (1, 5, 64, 700, 2048, 1999, 3)]
    pts, offsets = _concat(clouds)
    _say("case batched-small-only")
    tree, perm, dim, status = _run_batched(pts, offsets, kdt.WIDEST)
    assert status == kdt.OK
    for c in range(len(clouds)):
        _assert_cloud(pts, offsets, c, tree, perm, dim, kdt.WIDEST, "small-only")


def test_batched_all_empty():
    _say("case batched-empty")
    t = torch.zeros((0, 3), dtype=torch.float32, device=DEV)
    tree, perm, dim, status = kdt.build_batched(t, np.zeros(5, np.uint64), kdt.ROUND_ROBIN)
    torch.cuda.synchronize()
    assert int(status.item()) == kdt.OK and perm.numel() == 0


def test_batched_nonfinite_status():
    clouds = [workloads.uniform(n, 3, 60 + n) for n in (100, 9000, 3000)]
    clouds[2][17, 0] = np.inf
    pts, offsets = _concat(clouds)
    _say("case batched-nonfinite")
    *_, status = _run_batched(pts, offsets, kdt.ROUND_ROBIN)
    assert status & kdt.ENONFINITE
    clouds[2][17, 0] = 0.5
    clouds[0][3, 2] = np.nan
    pts, offsets = _concat(clouds)
    *_, status = _run_batched(pts, offsets, kdt.WIDEST)
    assert status & kdt.ENONFINITE


def test_batched_graph_replay():
    """Capture one batched build into a HIP graph; replay it on three inputs
    of the same shape (eager work and synchronisations between replays) and
    compare every replay with the oracle."""
    sizes = [3000, 64, 100000, 2500, 0, 40000, 700]
    k, mode = 3, kdt.ROUND_ROBIN
    offsets = np.zeros(len(sizes) + 1, np.uint64)
    offsets[1:] = np.cumsum(sizes)
    n = int(offsets[-1])
    static_in = torch.empty((n, k), dtype=torch.float32, device=DEV)
    tree = torch.empty((n, k), dtype=torch.float32, device=DEV)
    perm = torch.empty(n, dtype=torch.int32, device=DEV)
    dim = torch.empty(n, dtype=torch.uint8, device=DEV)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    ws = torch.empty(kdt.batched_workspace_bytes(offsets, k, mode), dtype=torch.uint8, device=DEV)
    inputs = [workloads.uniform(n, k, 70 + i) for i in range(3)]
    static_in.copy_(torch.from_numpy(inputs[0]))
    _say("case batched-graph: warm-up")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        kdt.build_batched(static_in, offsets, mode, tree=tree, perm=perm, dim=dim, status=status, workspace=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        kdt.build_batched(static_in, offsets, mode, tree=tree, perm=perm, dim=dim, status=status, workspace=ws)
    torch.cuda.synchronize()
    for i, x in enumerate(inputs):
        _say(f"case batched-graph: replay {i}")
        static_in.copy_(torch.from_numpy(x))
        tree.fill_(-1.0)
        perm.fill_(-1)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(status.item()) == kdt.OK
        tr, pe, di = tree.cpu().numpy(), perm.cpu().numpy().astype(np.uint32), dim.cpu().numpy()
        for c in range(len(sizes)):
            _assert_cloud(x, offsets, c, tr, pe, di, mode, f"graph-replay-{i}")
    del g


def test_batched_full_4096_clouds():
    """The 4096-cloud configuration: batched output equals each cloud's own
    single build on the GPU byte for byte, the checker accepts every cloud,
    and sampled clouds equal the oracle's build."""
    pts, offsets = workloads.cfg_batched()
    C = len(offsets) - 1
    k, mode = 3, kdt.ROUND_ROBIN
    _say(f"case batched-4096: n={pts.shape[0]}")
    t = torch.from_numpy(pts).to(DEV)
    tree, perm, dim, status = kdt.build_batched(t, offsets, mode)
    torch.cuda.synchronize()
    assert int(status.item()) == kdt.OK
    perm_b = perm.cpu().numpy().astype(np.uint32)
    tree_b = tree.cpu().numpy()
    dim_b = dim.cpu().numpy()
    # per-cloud single builds into the same layout
    nmax = int(np.max(np.diff(offsets.astype(np.int64))))
    ws = torch.empty(kdt.workspace_bytes(nmax, k, mode), dtype=torch.uint8, device=DEV)
    tree_s = torch.empty_like(tree)
    perm_s = torch.empty_like(perm)
    dim_s = torch.empty_like(dim)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    _say("case batched-4096: per-cloud builds")
    for c in range(C):
        a, b = int(offsets[c]), int(offsets[c + 1])
        kdt.build_ws(t[a:b], mode, tree=tree_s[a:b], perm=perm_s[a:b], dim=dim_s[a:b], status=st, workspace=ws)
    torch.cuda.synchronize()
    assert int(st.item()) == kdt.OK
    assert np.array_equal(perm_s.cpu().numpy().astype(np.uint32), perm_b)
    assert np.array_equal(dim_s.cpu().numpy(), dim_b)
    assert tree_s.cpu().numpy().tobytes() == tree_b.tobytes()
    _say("case batched-4096: checker on every cloud")
    for c in range(C):
        a, b = int(offsets[c]), int(offsets[c + 1])
        code, node = oracle.check(pts[a:b], perm_b[a:b], dim_b[a:b], oracle.RR)
        assert code == 0, f"cloud {c}: checker code {code} at node {node}"
        assert np.array_equal(tree_b[a:b], pts[a:b][perm_b[a:b]])
    _say("case batched-4096: oracle on sampled clouds")
    for c in np.random.default_rng(4).choice(C, 48, replace=False):
        _assert_cloud(pts, offsets, int(c), tree_b, perm_b, dim_b, mode, "batched-4096")


@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
def test_batched_rank_layouts(mode):
    """A batch built with per-role rank arrays (by root position) equals the
    same batch built with the point-major scatter, and every cloud is the
    oracle's tree."""
    sizes = [70000, 3000, 0, 130000, 9000, 1500, 40000, 2049]
    clouds = [workloads.grid(n, 4, 140 + i, levels=11) for i, n in enumerate(sizes)]
    pts, offsets = _concat(clouds)
    bits = int(max(sizes) - 1).bit_length()
    kdt.tuning_clear()
    try:
        got = {}
        for layout in (1, 2):
            _say(f"case batched rank layout {layout} mode {mode}")
            kdt.tuning_set(4, mode, bits, 0, 0, layout)
            got[layout] = _run_batched(pts, offsets, mode)
            assert got[layout][3] == kdt.OK
        assert got[1][0].tobytes() == got[2][0].tobytes()
        assert np.array_equal(got[1][1], got[2][1]) and np.array_equal(got[1][2], got[2][2])
        for c in range(len(sizes)):
            _assert_cloud(pts, offsets, c, *got[2][:3], mode, "rank-layout-2")
    finally:
        kdt.tuning_clear()


@pytest.mark.parametrize("layout", [1, 2])
@pytest.mark.parametrize("k", [2, 3, 4])
def test_batched_widest_root_dims_differ(k, layout):
    """Split-widest clouds whose roots split in different dimensions (cloud i
    stretched along dimension i mod k) in one batch: the presort roles map
    to other dimensions in every cloud, and with per-role rank arrays the
    root's role runs first and the others carry root ranks.  Every cloud is
    the oracle's tree, with either rank layout."""
    sizes = [60000, 9000, 2500, 33333, 70001, 4100, 12000, 2049]
    clouds = []
    for i, n in enumerate(sizes):
        c = workloads.uniform(n, k, 900 + 10 * k + i)
        c[:, i % k] *= np.float32(3.0)
        clouds.append(c)
    pts, offsets = _concat(clouds)
    bits = int(max(sizes) - 1).bit_length()
    kdt.tuning_clear()
    try:
        kdt.tuning_set(k, kdt.WIDEST, bits, 0, 0, layout)
        _say(f"case batched widest root dims k={k} layout {layout}")
        tree, perm, dim, status = _run_batched(pts, offsets, kdt.WIDEST)
        assert status == kdt.OK
        for c in range(len(sizes)):
            a = int(offsets[c])
            assert dim[a] == c % k, f"cloud {c}: root dimension {dim[a]}"
            _assert_cloud(pts, offsets, c, tree, perm, dim, kdt.WIDEST, f"widest-roots-layout-{layout}")
    finally:
        kdt.tuning_clear()


@pytest.mark.parametrize("layout", [0, 2])
@pytest.mark.parametrize("mode", [kdt.ROUND_ROBIN, kdt.WIDEST])
def test_batched_many_large_clouds(mode, layout):
    """Enough clouds of more than 2048 points that the presort takes its
    tiles from per-XCD queues (whole clouds per queue): every cloud is still
    the oracle's tree, with either rank layout (0: the planner's, which for
    these sizes is the point-major scatter; 2: per-dimension arrays written
    through index windows)."""
    rng = np.random.default_rng(77)
    sizes = [int(x) for x in np.exp(rng.uniform(np.log(2100), np.log(40000), 24))] + [5, 700, 2048, 0]
    clouds = [workloads.grid(n, 3, 400 + i, levels=10) for i, n in enumerate(sizes)]
    pts, offsets = _concat(clouds)
    bits = int(max(sizes) - 1).bit_length()
    kdt.tuning_clear()
    try:
        if layout:
            kdt.tuning_set(3, mode, bits, 0, 0, layout)
        _say(f"case many large clouds: mode {mode} layout {layout} n={pts.shape[0]}")
        got = _run_batched(pts, offsets, mode)
        assert got[3] == kdt.OK
        for c in range(len(sizes)):
            _assert_cloud(pts, offsets, c, *got[:3], mode, f"many-large-{layout}")
    finally:
        kdt.tuning_clear()


def test_tuner_choices_give_identical_trees():
    """Every digit-width / tile choice the tuner may record builds the same
    trees; kdt_tune_batched records one of them for the batch's class."""
    sizes = [70000, 3000, 0, 250000, 9000, 1500, 40000]
    clouds = [workloads.grid(n, 3, 90 + i, levels=17) for i, n in enumerate(sizes)]
    pts, offsets = _concat(clouds)
    _say("case tuner: reference build")
    kdt.tuning_clear()
    try:
        ref = _run_batched(pts, offsets, kdt.ROUND_ROBIN)
        bits = int(np.ceil(np.log2(max(sizes))))
        for rb in (8, 9, 10):
            for items in (4, 10):
                for pdims in (1, 2, 4):
                    _say(f"case tuner: radix {rb} items {items} presort dims {pdims}")
                    kdt.tuning_set(3, kdt.ROUND_ROBIN, bits, rb, items, 0, pdims)
                    got = _run_batched(pts, offsets, kdt.ROUND_ROBIN)
                    assert got[3] == kdt.OK
                    assert np.array_equal(got[1], ref[1]) and np.array_equal(got[2], ref[2])
                    assert got[0].tobytes() == ref[0].tobytes()
        kdt.tuning_clear()
        t = torch.from_numpy(pts).to(DEV)
        rb, items, pdims, ms = kdt.tune_batched(t, offsets, kdt.ROUND_ROBIN, reps=2)
        torch.cuda.synchronize()
        _say(f"tuner picked radix {rb} items {items} presort dims {pdims} at {ms:.3f} ms")
        assert rb in (8, 9, 10) and items in (4, 8) and pdims in (1, 4) and ms > 0
        assert kdt.tuning_get(3, kdt.ROUND_ROBIN, bits) == (rb, items, 0, pdims)
        got = _run_batched(pts, offsets, kdt.ROUND_ROBIN)
        assert np.array_equal(got[1], ref[1])
        for c in range(len(sizes)):
            _assert_cloud(pts, offsets, c, *got[:3], kdt.ROUND_ROBIN, "tuned")
    finally:
        kdt.tuning_clear()
