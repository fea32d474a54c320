"""An independent model of the paper's tag/sort construction, for tests only.

It computes the tree a second way, used to pin the oracle (they must agree)
and to replay the printed states of the Sec. 5 walkthrough.  Where the oracle
recurses over point lists, this model keeps one tag per point and repeats,
for every level, a global sort followed by a tag update, as Sec. 3
describes.  It is written from the definitions, not from the printed code:

* the level-order tree of Sec. 2: node s has children 2s+1 and 2s+2; the
  subtree of s is the set of node indices below s that exist for N nodes, so
  its size is found by counting that set (no closed form);
* the sort of Sec. 3.1 orders the points by tag and, within one tag, by the
  coordinate in that subtree's split dimension -- with the original index as
  the tie-break this build adopts;
* after the sort, the points of one level-l subtree s form a run; by
  Observation 2.1 the run's member whose rank equals the left child's size
  becomes node s, the members before it get tag 2s+1 and those after it tag
  2s+2 (Sec. 3.2); tags of fixed nodes never change;
* after the last level a sort by tag puts every point at its node (Sec. 5);
* split-widest (Sec. 6): a subtree's domain is its parent's domain with the
  parent's plane as the new upper (left child) or lower (right child) bound
  in the parent's split dimension, starting from the scene box at the root;
  its dimension is the one of widest float32 extent, lowest on ties.

The segment-begin position of Sec. 4.2 is provided as its definition (the
fixed nodes, then every earlier subtree of the same level) for the pins of
the closed forms.

Pure Python: use for N up to a few thousand.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np


def num_levels(n: int) -> int:
    """Levels of a complete tree of n nodes: depth of node n-1 plus one (0 for
    an empty tree)."""
    return 0 if n == 0 else level(n - 1) + 1


def level(s: int) -> int:
    """Depth of node s: the number of times s can be replaced by its parent
    (s-1)//2 before reaching the root."""
    d = 0
    while s > 0:
        s = (s - 1) // 2
        d += 1
    return d


def F(l: int) -> int:
    """Nodes on the levels above level l: 1 + 2 + ... + 2^(l-1)."""
    return sum(2 ** j for j in range(l))


@lru_cache(maxsize=None)
def ss(s: int, n: int) -> int:
    """Nodes in the subtree of s when the tree has n nodes, by counting: s
    itself (if it exists) and the subtrees of its two children."""
    return 0 if s >= n else 1 + ss(2 * s + 1, n) + ss(2 * s + 2, n)


def sb(s: int, l: int, n: int) -> int:
    """Where the points of level-l subtree s begin after the level-l sort:
    behind the F(l) fixed nodes and the points of the earlier subtrees of
    level l."""
    return F(l) + sum(ss(t, n) for t in range(F(l), s))


@np.errstate(over="ignore")
def _widest(lo, hi) -> int:
    # float32 extents (an extent may overflow to +inf, larger than any finite one)
    ext = (np.asarray(hi, np.float32) - np.asarray(lo, np.float32)).astype(np.float32)
    best = 0
    for d in range(1, len(ext)):
        if ext[d] > ext[best]:
            best = d
    return best


def paper_build(points, widest: bool = False, trace=None):
    """Run the per-level sort + tag update.  Returns (perm, dim) like the
    oracle.

    trace, if given, is called as trace(label, tags, order) after every sort
    and every update (labels 'sort<l>', 'update<l>', 'final'): order[i] is the
    original index of the point at array position i, tags[i] its tag."""
    P = np.asarray(points, dtype=np.float32)
    n, k = P.shape
    if n == 0:
        return np.zeros(0, np.uint32), np.zeros(0, np.uint8)
    tag = [0] * n                      # tag[i]: subtree or node of point i
    split = {}                         # subtree -> split dimension
    box = {}                           # subtree -> (lo, hi), split-widest only
    if widest:
        box[0] = (P.min(axis=0).copy(), P.max(axis=0).copy())
        split[0] = _widest(*box[0])

    def dim_of(t: int) -> int:
        return split[t] if widest else level(t) % k

    order = list(range(n))
    for l in range(num_levels(n) - 1):
        # Sec. 3.1: by tag, then coordinate in the tag's split dimension, then index
        order = sorted(range(n), key=lambda i: (tag[i], float(P[i, dim_of(tag[i])]), i))
        if trace:
            trace(f"sort{l}", [tag[i] for i in order], list(order))
        # Sec. 3.2 with Observation 2.1: walk the runs of the level-l subtrees
        runs = {}
        for i in order:
            if tag[i] >= F(l):
                runs.setdefault(tag[i], []).append(i)
        for s, members in runs.items():
            m = ss(2 * s + 1, n)       # rank of the pivot in its run
            for rank, i in enumerate(members):
                if rank != m:
                    tag[i] = 2 * s + 1 if rank < m else 2 * s + 2
            if widest:
                d = split[s]
                plane = P[members[m], d]
                lo, hi = box[s]
                for child, is_left in ((2 * s + 1, True), (2 * s + 2, False)):
                    clo, chi = lo.copy(), hi.copy()
                    if is_left:
                        chi[d] = min(chi[d], plane)
                    else:
                        clo[d] = max(clo[d], plane)
                    box[child] = (clo, chi)
                    split[child] = _widest(clo, chi)
        if trace:
            trace(f"update{l}", [tag[i] for i in order], list(order))
    # Sec. 5: every tag is now a node index; a sort by tag places the points
    order = sorted(range(n), key=lambda i: tag[i])
    if trace:
        trace("final", [tag[i] for i in order], list(order))
    assert [tag[i] for i in order] == list(range(n))
    perm = np.asarray(order, dtype=np.uint32)
    if widest:
        dim = np.asarray([split[s] for s in range(n)], dtype=np.uint8)
    else:
        dim = np.asarray([level(s) % k for s in range(n)], dtype=np.uint8)
    return perm, dim
