"""Geometric clustering and block subdivision (oracle; test infrastructure only).

Algorithm 1 (Sec. 4.1) splits the centroid cloud recursively by a hyperplane
until a cluster holds at most ``n_min`` indices; the facets are then permuted
so that every cluster is a contiguous index range.  Algorithm 2 (Sec. 4.2)
subdivides ``I x I`` recursively until a block is admissible in the sense of
the condition ``min(diam A_s, diam A_t) <= c * dist(A_s, A_t)`` on the
centroid clouds.

Readings fixed here:

* split: along the longest axis of the cluster's centroid bounding box (ties
  x < y < z) at the median; indices are ordered by (coordinate, original
  index) and the left child takes the first floor(#tau / 2);
* leaf iff ``#tau <= n_min``;
* diam / dist of a centroid cloud are taken on its axis-aligned bounding
  box: ``diam = |hi - lo|_2`` and ``dist = |max(0, lo_t - hi_s, lo_s - hi_t)|_2``
  (component-wise).  A box pair that passes also passes for the exact point
  clouds, so the test is conservative;
* ``dist = 0`` is never admissible;
* Algorithm 2 as printed has no branch for a leaf cluster; an inadmissible
  block whose row or column cluster is a leaf becomes a dense leaf block
  (the minimal block size stop of Sec. 4 (b)).

Sums of squares are evaluated as ``(x*x + y*y) + z*z``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Cluster:
    begin: int               # first position in the permuted order
    end: int                 # one past the last position
    lo: np.ndarray           # bounding box of the centroids
    hi: np.ndarray
    children: list = field(default_factory=list)
    level: int = 0

    @property
    def size(self) -> int:
        return self.end - self.begin

    @property
    def is_leaf(self) -> bool:
        return not self.children


def _norm3(v) -> float:
    return math.sqrt((v[0] * v[0] + v[1] * v[1]) + v[2] * v[2])


def build_index_tree(centroids: np.ndarray, n_min: int):
    """Algorithm 1 applied to the full index set.  Returns (root, perm) with
    ``perm[k]`` = original index of the facet at permuted position ``k``."""
    if n_min < 1:
        raise ValueError("n_min must be >= 1")
    centroids = np.asarray(centroids, dtype=np.float64)
    perm = []

    def rec(idx: np.ndarray, level: int) -> Cluster:
        pts = centroids[idx]
        lo = pts.min(axis=0)
        hi = pts.max(axis=0)
        begin = len(perm)
        if idx.size <= n_min:
            perm.extend(int(i) for i in idx)
            return Cluster(begin, begin + idx.size, lo, hi, [], level)
        ext = hi - lo
        axis = int(np.argmax(ext))  # first maximum: x before y before z
        order = np.lexsort((idx, pts[:, axis]))
        s = idx[order]
        h = idx.size // 2
        left = rec(s[:h], level + 1)
        right = rec(s[h:], level + 1)
        return Cluster(begin, right.end, lo, hi, [left, right], level)

    root = rec(np.arange(centroids.shape[0], dtype=np.int64), 0)
    return root, np.array(perm, dtype=np.int64)


def diam(cl: Cluster) -> float:
    return _norm3(cl.hi - cl.lo)


def dist(a: Cluster, b: Cluster) -> float:
    gap = np.maximum(0.0, np.maximum(b.lo - a.hi, a.lo - b.hi))
    return _norm3(gap)


def admissible(s: Cluster, t: Cluster, eta: float) -> bool:
    d = dist(s, t)
    if not d > 0.0:
        return False
    return min(diam(s), diam(t)) <= eta * d


def build_block_tree(root: Cluster, eta: float):
    """Algorithm 2 from (root, root).  Returns two lists of leaf blocks as
    tuples ``(row_begin, row_end, col_begin, col_end)``: (dense, low_rank),
    each sorted by (row_begin, col_begin)."""
    dense, lowrank = [], []

    def rec(s: Cluster, t: Cluster):
        if admissible(s, t, eta):
            lowrank.append((s.begin, s.end, t.begin, t.end))
        elif s.is_leaf or t.is_leaf:
            dense.append((s.begin, s.end, t.begin, t.end))
        else:
            for sc in s.children:
                for tc in t.children:
                    rec(sc, tc)

    rec(root, root)
    dense.sort(key=lambda b: (b[0], b[2]))
    lowrank.sort(key=lambda b: (b[0], b[2]))
    return dense, lowrank


def leaves(root: Cluster):
    out = []

    def rec(c):
        if c.is_leaf:
            out.append(c)
        else:
            for ch in c.children:
                rec(ch)

    rec(root)
    return out


def count_nodes(root: Cluster) -> int:
    return 1 + sum(count_nodes(c) for c in root.children)
