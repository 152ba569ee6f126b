"""Kernel functions and dense kernel matrices (oracle).

Paper: Section 4.1 (eq. a_gau) and Section 4.2 (eq. a_exp) define the kernel
matrices a_ij = k(|p_i - p_j|) off the diagonal and a_ii = 1 + c on it, with
k(0) = 1 for both kernels.  The diagonal is therefore k(0) + shift.

Readings:
* Gaussian in length-scale form: k(r) = exp(-r^2 / (2 l^2)), so the paper's
  dispersion sigma equals 2 l^2.
* Matern-3/2: k(r) = (1 + sqrt(3) r / l) exp(-sqrt(3) r / l).
* Exponential: k(r) = exp(-r / l) (the paper's sigma is l).
* Laplace single layer (Section 4.3): k(r) = 1 / (4 pi r) off the diagonal;
  its value at r = 0 is set to 0 here, because the boundary-element matrix
  replaces the singular self term by its own regularised diagonal.

Derivative kernels (for the gradient of b^T A^{-1} b; no shift): a kind
"<base>/dl" is the radial profile dk/dl (derivative in the length scale at
fixed r) and "<base>/g" is g(r) = k'(r) / r, through which the gradient of
k(|p_i - p_j|) in p_i is g(r_ij) (p_i - p_j).  g is set to 0 at r = 0 (its
self term cancels in the gradient; for the exponential kernel g is singular
there).  Closed forms, with z = sqrt(3) r / l for Matern-3/2:
  exp:      dk/dl = (r / l^2) exp(-r/l),        g = -exp(-r/l) / (l r)
  gauss:    dk/dl = (r^2 / l^3) exp(-r^2/2l^2), g = -exp(-r^2/2l^2) / l^2
  matern32: dk/dl = (z^2 / l) exp(-z),          g = -(3 / l^2) exp(-z)

A kernel is represented here by a callable taking two point arrays
X (n, dim) and Y (m, dim) and returning the (n, m) matrix of k(x_i, y_j)
*without* the diagonal shift.  The shift is added by `kernel_matrix` only on
the diagonal of a square block of a point set with itself.
"""
from __future__ import annotations

import numpy as np

KINDS = ("exp", "gauss", "matern32")            # smooth kernels with k(0) = 1; also "laplace"


def distances(X: np.ndarray, Y: np.ndarray) -> np.ndarray:
    """Euclidean distance matrix |x_i - y_j| (plain broadcast, FP64)."""
    diff = X[:, None, :] - Y[None, :, :]
    return np.sqrt(np.sum(diff * diff, axis=-1))


def radial(kind: str, length_scale: float):
    """The radial profile k(r) of a named kernel ("exp", "gauss",
    "matern32", or one of those followed by "/dl" or "/g")."""
    ell = float(length_scale)
    if "/" in kind:
        return _derivative(kind, ell)
    if kind == "exp":
        return lambda r: np.exp(-r / ell)
    if kind == "gauss":
        return lambda r: np.exp(-(r * r) / (2.0 * ell * ell))
    if kind == "matern32":
        a = np.sqrt(3.0) / ell
        return lambda r: (1.0 + a * r) * np.exp(-a * r)
    if kind == "laplace":
        def g(r):
            r = np.asarray(r, dtype=np.float64)
            safe = np.where(r > 0.0, r, 1.0)
            return np.where(r > 0.0, 1.0 / (4.0 * np.pi * safe), 0.0)
        return g
    raise ValueError(f"unknown kernel kind {kind!r}")


def _derivative(kind: str, ell: float):
    base, which = kind.split("/")
    if which == "dl":
        if base == "exp":
            return lambda r: (r / ell ** 2) * np.exp(-r / ell)
        if base == "gauss":
            return lambda r: (r * r / ell ** 3) * np.exp(-(r * r) / (2.0 * ell * ell))
        if base == "matern32":
            a = np.sqrt(3.0) / ell
            return lambda r: ((a * r) ** 2 / ell) * np.exp(-a * r)
    if which == "g":
        if base == "exp":
            def g(r):
                r = np.asarray(r, dtype=np.float64)
                safe = np.where(r > 0.0, r, 1.0)
                return np.where(r > 0.0, -np.exp(-safe / ell) / (ell * safe), 0.0)
            return g
        if base == "gauss":
            return lambda r: np.where(np.asarray(r) > 0.0,
                                      -np.exp(-(r * r) / (2.0 * ell * ell)) / ell ** 2, 0.0)
        if base == "matern32":
            a = np.sqrt(3.0) / ell
            return lambda r: np.where(np.asarray(r) > 0.0, -(3.0 / ell ** 2) * np.exp(-a * r), 0.0)
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
