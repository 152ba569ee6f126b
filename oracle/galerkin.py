"""Restricted (coarse) operators of the H2-MG hierarchy (oracle).

Paper: Section 3.3.  Multiplying A e = r by U_1^T on the left and inserting
V_1^T V_1 = I gives the restricted operator A_2 = U_1^T A V_1^T, which with
orthonormal bases equals U_1^T D V_1^T + D_2 + U_2 (...) V_2 (eq. a2_str);
the same step repeats level by level.  With V = U^T (symmetric case) and the
orthonormal coarse spaces W_d of ortho.py this is the Galerkin product

    A^{(d)} = W_d^T A_H2 W_d,   d = L, L-1, ..., d_top,

and the operator of MG level k >= 2 is A^{(d)} with d = L - k + 2.  The last
level (depth d_top, where every pair of clusters is close or in the
interaction list) is small and dense.

The level transfer from level k+1 to level k (the prolongation V_k^T = U_k)
is P_1 = W_L for the fine level and P_k = W_d^T W_{d-1} for k >= 2.
"""
from __future__ import annotations

import numpy as np

from .ortho import coarse_basis


def galerkin(A: np.ndarray, W: np.ndarray, offsets, r: int) -> np.ndarray:
    """W^T A W for a block-diagonal W whose block j covers rows
    offsets[j]:offsets[j+1] and columns j*r:(j+1)*r."""
    nb = len(offsets) - 1
    C = np.empty((nb * r, A.shape[1]))
    for j in range(nb):
        s, e = offsets[j], offsets[j + 1]
        C[j * r:(j + 1) * r] = W[s:e, j * r:(j + 1) * r].T @ A[s:e]
    out = np.empty((nb * r, nb * r))
    for j in range(nb):
        s, e = offsets[j], offsets[j + 1]
        out[:, j * r:(j + 1) * r] = C[:, s:e] @ W[s:e, j * r:(j + 1) * r]
    return out


class Hierarchy:
    """Dense operators A_1 .. A_l, prolongations P_1 .. P_{l-1} (tree order).

    A_1 = A_H2.  Without any far block (d_top is None) there is one level and
    it is solved directly.
    """

    def __init__(self, h2, A_tree=None):
        self.h2 = h2
        A1 = h2.dense_tree() if A_tree is None else A_tree
        self.ops = [A1]
        self.prolong = []
        self.depths = [None]               # depth of each level (None: fine)
        d_top = h2.d_top
        if d_top is not None:
            W_prev = None
            for d in range(h2.L, d_top - 1, -1):
                W = coarse_basis(h2, d)
                self.ops.append(galerkin(A1, W, h2.tree.offsets[d], h2.r))
                if W_prev is None:
                    self.prolong.append(W)
                else:
                    self.prolong.append(W_prev.T @ W)
                self.depths.append(d)
                W_prev = W

    @property
    def levels(self) -> int:
        return len(self.ops)
