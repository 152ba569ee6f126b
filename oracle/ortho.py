"""Orthonormal cluster bases (oracle).

Paper: Section 3.3 derives the restricted operator assuming orthogonal
bases (U_1^T U_1 = I, V_1 V_1^T = I) and Section 4.1 states that U_1 has
orthonormal columns.  Chebyshev bases are not orthonormal, so they are
orthonormalised.

Reading: for every cluster s, Q_s comes from the Householder QR of its direct
basis U_s = Q_s R_s (numpy/LAPACK), with signs fixed so that diag(R_s) > 0;
this makes Q_s unique when U_s has full column rank.  The coarse space at
depth d is W_d = blockdiag(Q_s, s at depth d) (tree order).  Since the
direct basis of a parent restricted to a child is U_c E_c, range(W_{d-1}) is
contained in range(W_d) and the level transfer is W_d^T W_{d-1}.
"""
from __future__ import annotations

import numpy as np


def qr_pos(U: np.ndarray):
    """Reduced QR with a positive diagonal in R."""
    Q, R = np.linalg.qr(U)
    sg = np.sign(np.diag(R))
    sg[sg == 0] = 1.0
    return Q * sg[None, :], R * sg[:, None]


def cluster_q(h2, d: int, j: int) -> np.ndarray:
    return qr_pos(h2.basis(d, j))[0]


def cluster_r(h2, d: int, j: int) -> np.ndarray:
    return qr_pos(h2.basis(d, j))[1]


def coarse_basis(h2, d: int) -> np.ndarray:
    """W_d (N x 2^d r), block diagonal in tree order."""
    r = h2.r
    W = np.zeros((h2.n, (1 << d) * r))
    for j in range(1 << d):
        W[h2.rows(d, j), j * r:(j + 1) * r] = cluster_q(h2, d, j)
    return W
