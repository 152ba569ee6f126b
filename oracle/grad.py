"""Gradient of the quadratic loss L = b^T A^{-1} b (oracle; test
infrastructure only).

The paper solves A x = b for a kernel matrix A = K(p; l) + s I; the loss and
its gradient in the kernel length scale l, the shift s and the point
coordinates p follow from the definition alone (A symmetric, so the adjoint
solve is the forward solve x = A^{-1} b):
    dL/dl      = -x^T (dA/dl) x,     dA/dl = [dk/dl (r_ij)] (no shift)
    dL/ds      = -x^T x
    dL/dp_{ia} = -2 x_i sum_j x_j g(r_ij) (p_{ia} - p_{ja})
               = -2 x_i [ p_{ia} (G x)_i - (G (x * p_{.a}))_i ],
with g(r) = k'(r) / r and G = [g(r_ij)] (its diagonal cancels; set to 0).

`dense_*` use the exact kernel matrices; `h2_*` use the H2 approximations of
k, dk/dl and g on the same tree (the oracle's H2 construction with the
derivative kinds of kernels.py), which is what the library computes.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .h2 import H2
from .kernels import kernel_matrix, make_kernel


def dense_loss(P, kind, ell, shift, b):
    """L = b^T K^{-1} b and x = K^{-1} b (dense Cholesky)."""
    K = kernel_matrix(make_kernel(kind, ell), P, shift)
    x = scipy.linalg.cho_solve(scipy.linalg.cho_factor(K, lower=True), b)
    return float(b @ x), x


def _point_gradient(P, x, Gx, G_apply):
    gp = np.empty_like(P)
    for a in range(P.shape[1]):
        gp[:, a] = -2.0 * x * (P[:, a] * Gx - G_apply(x * P[:, a]))
    return gp


def dense_gradient(P, kind, ell, shift, b):
    """(L, dL/dl, dL/ds, dL/dp) with the exact kernel matrices."""
    P = np.asarray(P, dtype=np.float64)
    L, x = dense_loss(P, kind, ell, shift, b)
    Kl = kernel_matrix(make_kernel(kind + "/dl", ell), P, 0.0)
    G = kernel_matrix(make_kernel(kind + "/g", ell), P, 0.0)
    dl = -float(x @ (Kl @ x))
    ds = -float(x @ x)
    gp = _point_gradient(P, x, G @ x, G.__matmul__)
    return L, dl, ds, gp


def h2_loss(P, kind, ell, shift, b, leaf, eta, m):
    """L = b^T A_H2^{-1} b with the dense form of the oracle's A_H2."""
    A = H2(P, kind, shift, leaf, eta, m, ell).dense()
    x = scipy.linalg.cho_solve(scipy.linalg.cho_factor(A, lower=True), b)
    return float(b @ x), x


def h2_gradient(P, kind, ell, shift, b, leaf, eta, m, x=None):
    """(L, dL/dl, dL/ds, dL/dp) with A, dA/dl and G replaced by their H2
    approximations on the tree of P (x: the solution of A_H2 x = b, solved
    densely when not given)."""
    P = np.asarray(P, dtype=np.float64)
    if x is None:
        L, x = h2_loss(P, kind, ell, shift, b, leaf, eta, m)
    else:
        L = float(b @ x)
    Hl = H2(P, kind + "/dl", 0.0, leaf, eta, m, ell)
    Hg = H2(P, kind + "/g", 0.0, leaf, eta, m, ell)
    dl = -float(x @ Hl.matvec(x))
    ds = -float(x @ x)
    gp = _point_gradient(P, x, Hg.matvec(x), Hg.matvec)
    return L, dl, ds, gp
