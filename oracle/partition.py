"""Close/far block partition by dual tree traversal (oracle).

Paper: Section 3.1 splits A into close (full-rank) blocks D_ij and far
(low-rank) blocks F_ij = U_i S_ij V_j (eq. f), and the same split is applied
again to the coupling matrix of each coarser level (eq. s1).  The method is
said to use strong admissibility; the criterion itself is not given.

Readings:
* admissible(s, t)  <=>  dist(B_s, B_t) > 0  and
                         max(diam B_s, diam B_t) <= eta * dist(B_s, B_t),
  with B the tight axis-aligned box of a cluster's points, diam its
  Euclidean diagonal and dist the Euclidean box-to-box gap.  The comparison
  is done on squares: max(diam_s^2, diam_t^2) <= eta^2 * dist^2, with the
  squared sums accumulated over axes in increasing axis order.
* traversal from (root, root): an admissible pair is far at its depth;
  otherwise a leaf pair is close (near); otherwise all four child pairs are
  visited.  So F_d is the set of far pairs at depth d whose parents are
  close (the interaction lists, the blocks of D_k in eq. s1) and N_d the set
  of visited non-admissible pairs at depth d.
* d_top, the coarsest level of the hierarchy, is the shallowest depth with a
  non-empty far list.

Pair lists are (k, 2) int64 arrays sorted by (row cluster, column cluster).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Partition:
    near: list    # near[d]: N_d pairs, d = 0..L (near[L] = close leaf pairs)
    far: list     # far[d]: F_d pairs, d = 0..L
    eta: float

    @property
    def L(self) -> int:
        return len(self.far) - 1

    @property
    def d_top(self):
        """Shallowest depth with a far pair, or None when there is none."""
        for d, f in enumerate(self.far):
            if f.shape[0]:
                return d
        return None


def _sq_sum(v: np.ndarray) -> np.ndarray:
    s = v[:, 0] * v[:, 0]
    for a in range(1, v.shape[1]):
        s = s + v[:, a] * v[:, a]
    return s


def admissible(lo_s, hi_s, lo_t, hi_t, eta: float) -> np.ndarray:
    """Vectorised strong admissibility test for pairs of boxes."""
    ds = _sq_sum(hi_s - lo_s)
    dt = _sq_sum(hi_t - lo_t)
    gap = np.maximum(np.maximum(lo_t - hi_s, lo_s - hi_t), 0.0)
    dist2 = _sq_sum(gap)
    eta2 = float(eta) * float(eta)
    return (dist2 > 0.0) & (np.maximum(ds, dt) <= eta2 * dist2)


def _sorted(pairs: np.ndarray) -> np.ndarray:
    if pairs.shape[0] == 0:
        return pairs.reshape(0, 2).astype(np.int64)
    order = np.lexsort((pairs[:, 1], pairs[:, 0]))
    return pairs[order].astype(np.int64)


def build_partition(tree, eta: float) -> Partition:
    near, far = [], []
    cur = np.zeros((1, 2), dtype=np.int64)
    for d in range(tree.L + 1):
        s, t = cur[:, 0], cur[:, 1]
        adm = admissible(tree.lo[d][s], tree.hi[d][s],
                         tree.lo[d][t], tree.hi[d][t], eta)
        far.append(_sorted(cur[adm]))
        nr = _sorted(cur[~adm])
        near.append(nr)
        if d < tree.L:
            kids = []
            for a in (0, 1):
                for b in (0, 1):
                    kids.append(np.stack([2 * nr[:, 0] + a,
                                          2 * nr[:, 1] + b], axis=1))
            cur = np.concatenate(kids, axis=0) if kids else cur[:0]
    return Partition(near, far, float(eta))
