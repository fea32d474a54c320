"""Pins for the CPU oracle: it is checked here against what the paper and the
mathematics fix, not against itself.

* Sec. 5 walkthrough: the printed final tree (and, through the independent
  tag/sort model, every printed intermediate state).
* Fig. 1 caption's 6-point set: tree derived by hand (tests/golden).
* Closed forms of Sec. 4 (used by the model and by the GPU path) against
  direct counting.
* Special cases with textbook answers: k = 1 is the breadth-first
  ("Eytzinger") layout of the sorted list; identical points keep original
  index order in an in-order traversal; N = 0, 1, 2, 3.
* Exhaustive uniqueness on tiny inputs: exactly one ordering satisfies the
  k-d and balance conditions, and it is the oracle's.
* Brute force k-d / split-rule check on every node for N <= 4096.
* The oracle's checker accepts the oracle's tree and rejects planted errors.
"""
import itertools
import os

import numpy as np
import pytest

import oracle
from paper_model import F, level, num_levels, paper_build, sb, ss
from paper_2211_00120_amd import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_walkthrough():
    states = {}
    cur = None
    with open(os.path.join(GOLDEN, "walkthrough_10pt.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if len(parts) == 1:
                cur = parts[0]
                states[cur] = {}
            else:
                states[cur][parts[0]] = [int(v) for v in parts[1:]]
    return states


def _read_six():
    vals = {}
    with open(os.path.join(GOLDEN, "six_point.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            vals[parts[0]] = [int(v) for v in parts[1:]]
    return vals


# ------------------------------------------------------------ brute force
@np.errstate(over="ignore")
def brute_ok(P, perm, dim, widest):
    """Check every (ancestor, descendant) pair and every node's dim by brute
    force: descendants are enumerated per depth from index ranges, domains
    are propagated top-down."""
    P = np.asarray(P, np.float32)
    n, k = P.shape
    perm = np.asarray(perm, np.int64)
    if sorted(perm.tolist()) != list(range(n)):
        return False
    if n == 0:
        return True
    lo = np.empty((n, k), np.float32)
    hi = np.empty((n, k), np.float32)
    lo[0] = P.min(axis=0)
    hi[0] = P.max(axis=0)
    for a in range(n):
        d = int(dim[a])
        if widest:
            ext = (hi[a] - lo[a]).astype(np.float32)
            want = int(np.flatnonzero(ext == ext.max())[0])
        else:
            want = level(a) % k
        if d != want:
            return False
        pv, pi = P[perm[a], d], perm[a]
        for child, is_left in ((2 * a + 1, True), (2 * a + 2, False)):
            if child < n:
                lo[child], hi[child] = lo[a], hi[a]
                if is_left:
                    hi[child, d] = pv
                else:
                    lo[child, d] = pv
            first, last = child, child + 1
            while first < n:
                idx = perm[first:min(last, n)]
                v = P[idx, d]
                if is_left:
                    good = (v < pv) | ((v == pv) & (idx < pi))
                else:
                    good = (v > pv) | ((v == pv) & (idx > pi))
                if not good.all():
                    return False
                first, last = 2 * first + 1, 2 * last + 1
    return True


# ---------------------------------------------------------------- tests
def test_walkthrough_final_tree():
    st = _read_walkthrough()
    P = np.stack([st["input"]["x"], st["input"]["y"]], axis=1).astype(np.float32)
    perm, dim = oracle.build(P, oracle.RR)
    got = P[perm]
    np.testing.assert_array_equal(got[:, 0], st["final"]["x"])
    np.testing.assert_array_equal(got[:, 1], st["final"]["y"])
    assert dim.tolist() == [level(s) % 2 for s in range(10)]


def test_walkthrough_model_replays_every_printed_state():
    st = _read_walkthrough()
    P = np.stack([st["input"]["x"], st["input"]["y"]], axis=1).astype(np.float32)
    seen = {}

    def trace(label, tags, order):
        seen[label] = (tags, order)

    paper_build(P, widest=False, trace=trace)
    for label in ["sort0", "update0", "sort1", "update1", "sort2", "update2", "final"]:
        tags, order = seen[label]
        assert tags == st[label]["tags"], label
        assert P[order, 0].astype(int).tolist() == st[label]["x"], label
        assert P[order, 1].astype(int).tolist() == st[label]["y"], label
    assert set(seen) == {"sort0", "update0", "sort1", "update1", "sort2", "update2", "final"}


def test_walkthrough_pivot_of_root_is_six():
    # Sec. 5: the root's pivot position in step 0 is ss(lChild(0)) = 6.
    assert ss(1, 10) == 6 == oracle.subtree_size(1, 10)


def test_six_point_set():
    v = _read_six()
    P = np.asarray(v["points"], np.float32).reshape(6, 2)
    perm, dim = oracle.build(P, oracle.RR)
    assert perm.tolist() == v["perm"]
    assert dim.tolist() == v["dim_rr"]
    perm, dim = oracle.build(P, oracle.WIDEST)
    assert perm.tolist() == v["perm"]
    assert dim.tolist() == v["dim_widest"]


def _bfs_size(s, n):
    count, stack = 0, [s]
    while stack:
        c = stack.pop()
        if c < n:
            count += 1
            stack += [2 * c + 1, 2 * c + 2]
    return count


@pytest.mark.parametrize("n", list(range(0, 70)) + [127, 128, 129, 255, 256, 1000, 4095, 4096])
def test_subtree_size_and_closed_forms(n):
    L = num_levels(n)
    assert L == (0 if n == 0 else int(np.floor(np.log2(n))) + 1)
    for s in range(0, min(n, 4096)):
        want = _bfs_size(s, n)
        assert oracle.subtree_size(s, n) == want
        assert ss(s, n) == want
    # sb(s,l) = F(l) + sum of sizes of the left siblings (Sec. 4.2)
    for l in range(max(L - 1, 0)):
        acc = F(l)
        for s in range(F(l), F(l + 1)):
            assert sb(s, l, n) == acc, (n, l, s)
            acc += _bfs_size(s, n)
        assert acc == n                                # segments tile [F(l), N)


def test_literal_c_precedence_reading_is_rejected():
    # Sec. 4.1 counts a subtree as its inner nodes plus its nodes on the
    # lowest level.  Read with C operator precedence, the printed inner-node
    # term is 2^(L-l-2) instead of 2^(L-l-1) - 1.  For the walkthrough (N =
    # 10, L = 4) node 1 (level 1) has 2^2 - 1 = 3 inner nodes and 3 of the 3
    # lowest-level nodes, 6 in all -- the C reading would give 2 + 3 = 5, but
    # the printed step-0 update puts 6 points into subtree 1.
    n, s = 10, 1
    L, l = num_levels(n), level(s)
    lowest = [x for x in range(F(L - 1), n) if _is_below(x, s)]
    assert len(lowest) == 3
    assert (2 ** (L - l - 1) - 1) + len(lowest) == ss(1, n) == 6
    assert 2 ** (L - l - 2) + len(lowest) == 5


def _is_below(x, s):
    while x > s:
        x = (x - 1) // 2
    return x == s


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_tiny_n(n):
    P = np.arange(n * 2, dtype=np.float32).reshape(n, 2)[::-1].copy()
    perm, dim = oracle.build(P, oracle.RR)
    if n == 0:
        assert perm.size == 0
    elif n == 1:
        assert perm.tolist() == [0]
    elif n == 2:
        # root is the larger point, its left child the smaller
        assert perm.tolist() == [0, 1]          # P[0] = (2,3) > P[1] = (0,1)
    else:
        # sorted by x: indices 2,1,0 -> root = middle, children = ends
        assert perm.tolist() == [1, 2, 0]


def _inorder(n):
    out = []

    def rec(s):
        if s < n:
            rec(2 * s + 1)
            out.append(s)
            rec(2 * s + 2)

    rec(0)
    return out


@pytest.mark.parametrize("n", [1, 2, 5, 16, 17, 100, 1023, 1024, 3000])
def test_k1_is_breadth_first_layout_of_sorted_list(n):
    P = workloads.grid(n, 1, seed=n, levels=max(2, n // 7))
    perm, dim = oracle.build(P, oracle.RR)
    srt = sorted(range(n), key=lambda i: (P[i, 0], i))      # stable sort by (x, index)
    want = np.empty(n, np.int64)
    for rank, node in enumerate(_inorder(n)):
        want[node] = srt[rank]
    assert perm.tolist() == want.tolist()
    assert not dim.any()


@pytest.mark.parametrize("mode", [oracle.RR, oracle.WIDEST])
@pytest.mark.parametrize("n,k", [(1, 3), (9, 2), (64, 3), (500, 4)])
def test_identical_points(n, k, mode):
    P = np.full((n, k), 0.5, np.float32)
    perm, dim = oracle.build(P, mode)
    assert [int(perm[s]) for s in _inorder(n)] == list(range(n))
    if mode == oracle.WIDEST:
        assert not dim.any()                      # all extents 0: lowest dim
    else:
        assert dim.tolist() == [level(s) % k for s in range(n)]


@np.errstate(over="ignore")
def _all_valid(P, widest):
    n = len(P)
    sols = []
    for perm in itertools.permutations(range(n)):
        perm = np.asarray(perm)
        # dims implied by the candidate: RR by level, WIDEST by its own domains
        dim = np.zeros(n, np.int64)
        lo = [None] * n
        hi = [None] * n
        if n:
            lo[0], hi[0] = P.min(axis=0), P.max(axis=0)
        for a in range(n):
            if widest:
                ext = (hi[a] - lo[a]).astype(np.float32)
                dim[a] = int(np.flatnonzero(ext == ext.max())[0])
            else:
                dim[a] = level(a) % P.shape[1]
            for c, left in ((2 * a + 1, True), (2 * a + 2, False)):
                if c < n:
                    lo[c], hi[c] = lo[a].copy(), hi[a].copy()
                    if left:
                        hi[c][dim[a]] = P[perm[a], dim[a]]
                    else:
                        lo[c][dim[a]] = P[perm[a], dim[a]]
        if brute_ok(P, perm, dim, widest):
            sols.append((perm.tolist(), dim.tolist()))
    return sols


@pytest.mark.parametrize("widest", [False, True])
@pytest.mark.parametrize("seed", range(6))
def test_exhaustive_uniqueness(seed, widest):
    n = 4 + seed % 4                                   # 4..7 points
    P = workloads.grid(n, 2, seed=100 + seed, levels=3)  # many ties
    sols = _all_valid(P, widest)
    assert len(sols) == 1
    perm, dim = oracle.build(P, oracle.WIDEST if widest else oracle.RR)
    assert sols[0] == (perm.tolist(), dim.tolist())


@pytest.mark.parametrize("widest", [False, True])
@pytest.mark.parametrize("n,k,seed", [(37, 2, 1), (300, 3, 2), (1000, 4, 3), (4096, 3, 4), (4095, 2, 5)])
def test_bruteforce_invariants(n, k, seed, widest):
    P = workloads.grid(n, k, seed=seed, levels=5) if seed % 2 else workloads.uniform(n, k, seed)
    mode = oracle.WIDEST if widest else oracle.RR
    perm, dim = oracle.build(P, mode)
    assert brute_ok(P, perm, dim, widest)
    assert oracle.check(P, perm, dim, mode) == (0, 0)


@pytest.mark.parametrize("widest", [False, True])
def test_signed_values_and_zero_signs(widest):
    P = workloads.signed_mix(700, 3, seed=11)
    mode = oracle.WIDEST if widest else oracle.RR
    perm, dim = oracle.build(P, mode)
    assert brute_ok(P, perm, dim, widest)


@pytest.mark.parametrize("widest", [False, True])
@pytest.mark.parametrize("seed", range(12))
def test_oracle_equals_paper_loop(seed, widest):
    r = np.random.default_rng(seed)
    n = int(r.integers(1, 260))
    k = int(r.integers(1, 5))
    P = workloads.grid(n, k, seed=seed, levels=int(r.integers(2, 9)))
    perm_m, dim_m = paper_build(P, widest=widest)
    perm_o, dim_o = oracle.build(P, oracle.WIDEST if widest else oracle.RR)
    assert perm_m.tolist() == perm_o.tolist()
    assert dim_m.tolist() == dim_o.tolist()


@pytest.mark.parametrize("widest", [False, True])
def test_checker_rejects_planted_errors(widest):
    mode = oracle.WIDEST if widest else oracle.RR
    P = workloads.uniform(513, 3, seed=7)
    perm, dim = oracle.build(P, mode)
    assert oracle.check(P, perm, dim, mode)[0] == 0
    r = np.random.default_rng(0)
    for _ in range(20):
        a, b = r.choice(513, 2, replace=False)
        p2 = perm.copy()
        p2[a], p2[b] = p2[b], p2[a]
        # a swap breaks the order; in split-widest mode it may first show
        # up as a changed domain, hence a dim mismatch
        assert oracle.check(P, p2, dim, mode)[0] in ((2, 3) if widest else (2,))
        assert not brute_ok(P, p2, dim, widest)
    p3 = perm.copy()
    p3[5] = p3[6]
    assert oracle.check(P, p3, dim, mode)[0] == 1
    d2 = dim.copy()
    d2[300] = (d2[300] + 1) % 3
    assert oracle.check(P, perm, d2, mode)[0] in (2, 3)
    assert not brute_ok(P, perm, d2, widest)


# ---------------------------------------------------------------- int32 points
# Table 1's int1 rows build over 32-bit integers (Sec. 7.2 templates the
# builder over the point type).  Integers compare exactly; the split-widest
# extent of an integer domain is the exact difference hi - lo.

I32_MIN, I32_MAX = -(2 ** 31), 2 ** 31 - 1


def _i32_points(n, k, seed, levels=None):
    r = np.random.default_rng(seed)
    if levels:
        P = r.integers(-levels // 2, levels - levels // 2, size=(n, k))
    else:
        P = r.integers(I32_MIN, I32_MAX, size=(n, k), endpoint=True)
        # now and then the extremes and values near 0
        m = r.random((n, k)) < 0.2
        P[m] = r.choice([I32_MIN, I32_MAX, 0, -1, 1], size=int(m.sum()))
    return P.astype(np.int32)


def brute_ok_i32(P, perm, dim, widest):
    """brute_ok for int32 points: every (ancestor, descendant) pair under the
    (value, index) order, and every node's dim from its domain with exact
    (int64) extents."""
    P = np.asarray(P, np.int64)
    n, k = P.shape
    perm = np.asarray(perm, np.int64)
    if sorted(perm.tolist()) != list(range(n)):
        return False
    if n == 0:
        return True
    lo = np.empty((n, k), np.int64)
    hi = np.empty((n, k), np.int64)
    lo[0], hi[0] = P.min(axis=0), P.max(axis=0)
    for a in range(n):
        d = int(dim[a])
        ext = hi[a] - lo[a]
        want = int(np.flatnonzero(ext == ext.max())[0]) if widest else level(a) % k
        if d != want:
            return False
        pv, pi = P[perm[a], d], perm[a]
        for child, is_left in ((2 * a + 1, True), (2 * a + 2, False)):
            if child < n:
                lo[child], hi[child] = lo[a], hi[a]
                if is_left:
                    hi[child, d] = pv
                else:
                    lo[child, d] = pv
            first, last = child, child + 1
            while first < n:
                idx = perm[first:min(last, n)]
                v = P[idx, d]
                good = ((v < pv) | ((v == pv) & (idx < pi))) if is_left else ((v > pv) | ((v == pv) & (idx > pi)))
                if not good.all():
                    return False
                first, last = 2 * first + 1, 2 * last + 1
    return True


@pytest.mark.parametrize("n", [1, 2, 5, 16, 17, 100, 1023, 1024, 3000])
def test_i32_k1_is_breadth_first_layout_of_sorted_list(n):
    P = _i32_points(n, 1, seed=n, levels=max(2, n // 7) if n % 2 else None)
    perm, dim = oracle.build(P, oracle.RR)
    srt = sorted(range(n), key=lambda i: (int(P[i, 0]), i))   # stable sort by (x, index)
    want = np.empty(n, np.int64)
    for rank, node in enumerate(_inorder(n)):
        want[node] = srt[rank]
    assert perm.tolist() == want.tolist()
    assert not dim.any()


@pytest.mark.parametrize("mode", [oracle.RR, oracle.WIDEST])
@pytest.mark.parametrize("value", [I32_MIN, -1, 0, 7, I32_MAX])
def test_i32_identical_points(mode, value):
    n, k = 300, 3
    P = np.full((n, k), value, np.int32)
    perm, dim = oracle.build(P, mode)
    assert [int(perm[s]) for s in _inorder(n)] == list(range(n))
    if mode == oracle.WIDEST:
        assert not dim.any()
    else:
        assert dim.tolist() == [level(s) % k for s in range(n)]


@pytest.mark.parametrize("mode", [oracle.RR, oracle.WIDEST])
@pytest.mark.parametrize("seed", range(4))
def test_i32_equals_float_on_exactly_representable_values(mode, seed):
    """Integers of magnitude below 2^23 are exact float32 values whose
    differences are exact too: the int32 and float32 builds coincide."""
    r = np.random.default_rng(seed)
    P = r.integers(-(2 ** 23), 2 ** 23, size=(2000 + seed, 1 + seed % 4)).astype(np.int32)
    if seed % 2:
        P //= 1 << 18                                   # ties
    pi, di = oracle.build(P, mode)
    pf, df = oracle.build(P.astype(np.float32), mode)
    assert np.array_equal(pi, pf) and np.array_equal(di, df)


@pytest.mark.parametrize("widest", [False, True])
@pytest.mark.parametrize("n,k,seed", [(37, 2, 1), (300, 3, 2), (1000, 4, 3), (2047, 3, 4)])
def test_i32_bruteforce_invariants(n, k, seed, widest):
    P = _i32_points(n, k, seed, levels=9 if seed % 2 else None)
    mode = oracle.WIDEST if widest else oracle.RR
    perm, dim = oracle.build(P, mode)
    assert brute_ok_i32(P, perm, dim, widest)
    assert oracle.check(P, perm, dim, mode) == (0, 0)


def test_i32_widest_extent_is_exact():
    """Extents that float32 rounding or int32 overflow would get wrong.
    Root domain: x spans 2^24, y spans 2^24 + 1 (both 2^24 in float32, a tie
    the lowest dimension would win): the exact extent picks y.  Second set:
    x spans the whole int32 range (an int32 subtraction would wrap to -1),
    y a small range: x."""
    P = np.array([[0, 0], [2 ** 24, 2 ** 24 + 1], [5, 6]], np.int32)
    _, dim = oracle.build(P, oracle.WIDEST)
    assert dim[0] == 1
    _, dimf = oracle.build(P.astype(np.float32), oracle.WIDEST)
    assert dimf[0] == 0                                   # float32 reading: a tie
    P = np.array([[I32_MIN, 0], [I32_MAX, 10], [3, 4]], np.int32)
    _, dim = oracle.build(P, oracle.WIDEST)
    assert dim[0] == 0


def test_i32_checker_rejects_planted_errors():
    P = _i32_points(500, 3, 77)
    for mode in (oracle.RR, oracle.WIDEST):
        perm, dim = oracle.build(P, mode)
        bad = perm.copy()
        bad[[3, 9]] = bad[[9, 3]]
        assert oracle.check(P, bad, dim, mode)[0] == 2
        d2 = dim.copy()
        d2[10] = (d2[10] + 1) % 3
        assert oracle.check(P, perm, d2, mode)[0] in (2, 3)
