"""Kernel functions and dense kernel matrices (oracle).

Paper: Section 4.1 (eq. a_gau) and Section 4.2 (eq. a_exp) define the kernel
matrices a_ij = k(|p_i - p_j|) off the diagonal and a_ii = 1 + c on it, with
k(0) = 1 for both kernels.  The diagonal is therefore k(0) + shift.

Readings:
* Gaussian in length-scale form: k(r) = exp(-r^2 / (2 l^2)), so the paper's
  dispersion sigma equals 2 l^2.
* Matern-3/2: k(r) = (1 + sqrt(3) r / l) exp(-sqrt(3) r / l).
* Exponential: k(r) = exp(-r / l) (the paper's sigma is l).

A kernel is represented here by a callable taking two point arrays
X (n, dim) and Y (m, dim) and returning the (n, m) matrix of k(x_i, y_j)
*without* the diagonal shift.  The shift is added by `kernel_matrix` only on
the diagonal of a square block of a point set with itself.
"""
from __future__ import annotations

import numpy as np

KINDS = ("exp", "gauss", "matern32")


def distances(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Euclidean distance matrix |x_i - y_j| (plain broadcast, FP64)."""
    diff = X[:, None, :] - Y[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=-1))


def radial(kind: str, length_scale: float):
    """The radial profile k(r) of a named kernel."""
    ell = float(length_scale)
    if kind == "exp":
        return lambda r: np.exp(-r / ell)
    if kind == "gauss":
        return lambda r: np.exp(-(r * r) / (2.0 * ell * ell))
    if kind == "matern32":
        a = np.sqrt(3.0) / ell
        return lambda r: (1.0 + a * r) * np.exp(-a * r)
    raise ValueError(f"unknown kernel kind {kind!r}")


def make_kernel(kind: str, length_scale: float):
    """Kernel callable k(X, Y) -> (n, m) matrix for a radial kernel."""
    prof = radial(kind, length_scale)
    return lambda X, Y: prof(distances(X, Y))


def polynomial_kernel(degree: int):
    """k(x, y) = prod_a (1 + x_a y_a)^degree.

    A polynomial of degree `degree` in each coordinate of x (and of y), so
    tensor interpolation with degree+1 nodes per axis reproduces it exactly.
    Used only to pin the H2 construction.
    """
    def k(X, Y):
        out = np.ones((X.shape[0], Y.shape[0]))
        for a in range(X.shape[1]):
            out *= (1.0 + np.outer(X[:, a], Y[:, a])) ** degree
        return out
    return k


def kernel_matrix(kern, X: np.ndarray, shift: float, Y=None) -> np.ndarray:
    """Dense kernel matrix.  With Y omitted: the square matrix of X with
    itself, with `shift` added to the diagonal (a_ii = k(0) + c)."""
    if Y is None:
        K = kern(X, X)
        K[np.diag_indices_from(K)] += shift
        return K
    return kern(X, Y)
