"""Cluster tree by recursive geometric bisection (oracle).

Paper: Section 3.1 partitions the index set into M leaf blocks and then
groups p blocks at a time into the blocks of the next coarser level ("typical
choices of p are 2 or 2^d").  The multigrid hierarchy needs every leaf on one
level (U_1 spans all M blocks), so the tree has uniform depth.

Readings (the paper gives no construction; MCBH is used there):
* binary tree (p = 2) of uniform depth L = smallest integer with
  leaf * 2^L >= N (L = 0 when N <= leaf);
* each cluster is split along the longest side of the tight bounding box of
  its points (ties go to the lowest axis);
* the split is at the median: the cluster's points are stably sorted by that
  coordinate (ties keep their current order) and the first ceil(n/2) go to
  the left child.

Tree order: position k of the permuted index set holds user index perm[k].
Cluster j at depth d owns positions offsets[d][j] .. offsets[d][j+1]-1, and
its children are clusters 2j and 2j+1 at depth d+1.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Tree:
    perm: np.ndarray          # (N,) tree position -> user index
    L: int                    # leaf depth
    offsets: list             # offsets[d]: (2^d + 1,) int64
    lo: list                  # lo[d]: (2^d, dim) tight box lower corners
    hi: list                  # hi[d]: (2^d, dim) tight box upper corners

    @property
    def n(self) -> int:
        return int(self.perm.shape[0])

    def size(self, d: int, j: int) -> int:
        return int(self.offsets[d][j + 1] - self.offsets[d][j])

    def rows(self, d: int, j: int) -> slice:
        return slice(int(self.offsets[d][j]), int(self.offsets[d][j + 1]))


def leaf_depth(n: int, leaf: int) -> int:
    """Smallest L with leaf * 2^L >= n."""
    L = 0
    while leaf * (1 << L) < n:
        L += 1
    return L


def _box(P: np.ndarray, dim: int):
    if P.shape[0] == 0:
        return np.full(dim, np.inf), np.full(dim, -np.inf)
    return P.min(axis=0), P.max(axis=0)


def build_tree(points: np.ndarray, leaf: int) -> Tree:
    """Median bisection along the longest box side, uniform depth."""
    points = np.asarray(points, dtype=np.float64)
    n, dim = points.shape
    if n < 1 or leaf < 1:
        raise ValueError("need n >= 1 and leaf >= 1")
    L = leaf_depth(n, leaf)
    perm = np.arange(n, dtype=np.int64)
    offsets = [np.array([0, n], dtype=np.int64)]
    for d in range(L):
        off = offsets[d]
        new = [0]
        for j in range(1 << d):
            s, e = int(off[j]), int(off[j + 1])
            idx = perm[s:e]
            P = points[idx]
            lo, hi = _box(P, dim)
            ext = hi - lo if e > s else np.zeros(dim)
            axis = int(np.argmax(ext))          # first maximum: lowest axis
            order = np.argsort(P[:, axis], kind="stable")
            perm[s:e] = idx[order]
            nl = (e - s + 1) // 2
            new += [s + nl, e]
        offsets.append(np.array(new, dtype=np.int64))
    lo_all, hi_all = [], []
    Pt = points[perm]
    for d in range(L + 1):
        off = offsets[d]
        lo = np.empty((1 << d, dim))
        hi = np.empty((1 << d, dim))
        for j in range(1 << d):
            lo[j], hi[j] = _box(Pt[off[j]:off[j + 1]], dim)
        lo_all.append(lo)
        hi_all.append(hi)
    return Tree(perm, L, offsets, lo_all, hi_all)
