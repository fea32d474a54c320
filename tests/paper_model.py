"""A direct model of the paper's tag/sort loop, for tests only.

This is a second, independent way of computing the tree, used to pin the
oracle (they must agree) and to replay the printed states of the Sec. 5
walkthrough.  It follows the algorithm as the paper states it, not the
oracle's recursion:

* every point carries a tag, initially 0 (Sec. 3);
* for l = 0 .. L-2: sort all (tag, point) pairs by tag, then by the point's
  coordinate in the split dimension (Sec. 3.1), then by original index (the
  tie-break reading adopted for this build); then update every array entry
  i >= F(l) from its tag s and the pivot position sb(s,l) + ss(2s+1) (Sec. 3.2);
* a final sort by tag puts every point at its node (Sec. 5);
* sb and ss are the O(1) closed forms of Sec. 4 with the published errata
  (L = 32 - clz(N)), read as mathematics: the inner-node term is
  2^(L-l-1) - 1, not the C-precedence reading 1 << (L-l-2);
* split-widest (Sec. 6): each subtree's dimension is the widest float32 extent
  of its domain, obtained by starting from the scene box, clipping by the new
  parent's plane and then by every already-fixed ancestor's plane while
  walking up to the root.

Pure Python, O(N log^2 N) with large constants: use for N up to a few
thousand.
"""
from __future__ import annotations

import numpy as np


def num_levels(n: int) -> int:
    """L = 32 - clz(N) (Sec. 4.2 after the revision-3 erratum); 0 for N = 0."""
    return int(n).bit_length()


def level(s: int) -> int:
    """level(s) = 31 - clz(s+1) (Sec. 2)."""
    return (s + 1).bit_length() - 1


def F(l: int) -> int:
    """Number of nodes in the top l full levels, 2^l - 1 (Sec. 2)."""
    return (1 << l) - 1


def ss(s: int, n: int) -> int:
    """Subtree size in O(1) (Sec. 4.1)."""
    L = num_levels(n)
    l = level(s)
    sh = L - l - 1
    fllc = ~((~s) << sh)                     # first lowest-level child
    return ((1 << sh) - 1) + min(max(0, n - fllc), 1 << sh)


def sb(s: int, l: int, n: int) -> int:
    """Segment begin of subtree s in iteration l (Sec. 4.2)."""
    L = num_levels(n)
    nls = s - F(l)
    sh = L - l - 1
    return F(l) + nls * ((1 << sh) - 1) + min(nls * (1 << sh), n - F(L - 1))


@np.errstate(over="ignore")
def _widest(lo, hi) -> int:
    # float32 extents; an extent may overflow to +inf, which compares as
    # larger than every finite extent
    ext = (np.asarray(hi, np.float32) - np.asarray(lo, np.float32)).astype(np.float32)
    best = 0
    for d in range(1, len(ext)):
        if ext[d] > ext[best]:
            best = d
    return best


def paper_build(points, widest: bool = False, trace=None):
    """Run the tag/sort loop.  Returns (perm, dim) like the oracle.

    trace, if given, is called as trace(label, tags, order) after every sort
    and every update (labels 'sort<l>', 'update<l>', 'final'); order[i] is the
    original index of the point at array position i."""
    P = np.asarray(points, dtype=np.float32)
    n, k = P.shape
    if n == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint8)
    L = num_levels(n)
    tags = [0] * n
    order = list(range(n))
    dims = {}
    if widest:
        dims[0] = _widest(P.min(axis=0), P.max(axis=0))

    def dim_of(tag, l):
        return dims[tag] if widest else l % k

    for l in range(L - 1):
        pairs = sorted(zip(tags, order),
                       key=lambda ti: (ti[0], P[ti[1], dim_of(ti[0], l)], ti[1]))
        tags = [t for t, _ in pairs]
        order = [i for _, i in pairs]
        if trace:
            trace(f"sort{l}", list(tags), list(order))
        new = list(tags)
        for i in range(F(l), n):
            s = tags[i]
            piv = sb(s, l, n) + ss(2 * s + 1, n)
            if i == piv:
                continue
            child = 2 * s + 1 if i < piv else 2 * s + 2
            new[i] = child
            if widest:
                # domain of the new subtree: scene box clipped by s's plane
                # (its pivot sits at array position piv), then by every fixed
                # ancestor of s (ancestor a sits at array position a).
                lo = P.min(axis=0).copy()
                hi = P.max(axis=0).copy()
                ds = dims[s]
                plane = P[order[piv], ds]
                if child == 2 * s + 1:
                    hi[ds] = min(hi[ds], plane)
                else:
                    lo[ds] = max(lo[ds], plane)
                c = s
                while c > 0:
                    a = (c - 1) // 2
                    da = dims[a]
                    plane = P[order[a], da]
                    if c == 2 * a + 1:
                        hi[da] = min(hi[da], plane)
                    else:
                        lo[da] = max(lo[da], plane)
                    c = a
                dims[child] = _widest(lo, hi)
        tags = new
        if trace:
            trace(f"update{l}", list(tags), list(order))
    pairs = sorted(zip(tags, order))
    tags = [t for t, _ in pairs]
    order = [i for _, i in pairs]
    if trace:
        trace("final", list(tags), list(order))
    assert tags == list(range(n))
    perm = np.asarray(order, dtype=np.uint32)
    if widest:
        dim = np.asarray([dims[s] for s in range(n)], dtype=np.uint8)
    else:
        dim = np.asarray([level(s) % k for s in range(n)], dtype=np.uint8)
    return perm, dim
