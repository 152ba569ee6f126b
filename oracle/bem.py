"""The boundary-element matrix of the Laplace single layer (oracle; test
infrastructure only).

Paper: Section 4.3.  Triangles with centroids y_j, quadrature weights w_j
(the triangle areas) and collocation points x_i = y_i give
    A_ij = w_j / (4 pi ||x_i - y_j||)  (i != j),   A_ii = w_i / (4 pi R_i),
with R_i the mean distance from the centroid of triangle i to its three
vertices, and the right-hand side of a point source x_0 off the surface,
f_j = 1 / (4 pi ||y_j - x_0||).

Finding and reading for the diagonal: with A_ii = w_i / (4 pi R_i) the
matrix is indefinite on the bumpy torus (about half of its eigenvalues are
negative at 576 to 8000 panels): the regularised self term is about 3 times
smaller than the potential of the panel's own uniform density at its
centroid.  The self term used instead is that potential itself,
A_ii = I_i / (4 pi), with I_i the integral of 1 / |y_i - y| over the flat
triangle, in closed form: the sum over the three edges of
d_e ln((s_2 + r_2) / (s_1 + r_1)), where d_e is the distance from the
centroid to the edge line, s_1, s_2 the signed positions of the edge's end
points along it and r_1, r_2 their distances to the centroid.  With it the
matrix is positive definite.

A has column weights, so it is not symmetric.  Reading: the library solves
the symmetric form S y = W^(1/2) f with S = W^(1/2) A W^(-1/2)
= W^(1/2) G W^(1/2), G_ij = 1 / (4 pi r_ij), G_ii = 1 / (4 pi R_i), and
recovers sigma = W^(-1/2) y; S is the kernel matrix 1/(4 pi r) in the scaled
form of h2.py with s = sqrt(w) and d = A_ii.
"""
from __future__ import annotations

import numpy as np

from .kernels import distances


def panels(V: np.ndarray, T: np.ndarray):
    """Centroids (nt, 3), areas (nt,) and R_i (nt,) of a triangle mesh."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    y = (a + b + c) / 3.0
    w = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    R = (np.linalg.norm(y - a, axis=1) + np.linalg.norm(y - b, axis=1)
         + np.linalg.norm(y - c, axis=1)) / 3.0
    return y, w, R


def self_integral(V: np.ndarray, T: np.ndarray) -> np.ndarray:
    """Integral of 1 / |y_i - y| over triangle i, y_i its centroid (closed
    form, edge by edge)."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    y = (a + b + c) / 3.0
    total = np.zeros(len(T))
    for p1, p2 in ((a, b), (b, c), (c, a)):
        e = p2 - p1
        t = e / np.linalg.norm(e, axis=1)[:, None]
        s1 = np.sum((p1 - y) * t, axis=1)
        s2 = np.sum((p2 - y) * t, axis=1)
        d = np.linalg.norm(y - (p1 - s1[:, None] * t), axis=1)
        r1 = np.linalg.norm(p1 - y, axis=1)
        r2 = np.linalg.norm(p2 - y, axis=1)
        total += d * np.log((s2 + r2) / (s1 + r1))
    return total


def diagonal(V: np.ndarray, T: np.ndarray, self_term: str = "analytic") -> np.ndarray:
    """A_ii: I_i / (4 pi) ("analytic", used by the library) or the paper's
    w_i / (4 pi R_i) ("paper")."""
    y, w, R = panels(V, T)
    if self_term == "paper":
        return w / (4.0 * np.pi * R)
    return self_integral(V, T) / (4.0 * np.pi)


def collocation_matrix(V: np.ndarray, T: np.ndarray, self_term: str = "analytic") -> np.ndarray:
    """The (nonsymmetric) collocation matrix A, dense (small meshes only)."""
    y, w, R = panels(V, T)
    D = distances(y, y)
    np.fill_diagonal(D, 1.0)
    A = w[None, :] / (4.0 * np.pi * D)
    A[np.diag_indices_from(A)] = diagonal(V, T, self_term)
    return A


def symmetric_scaling(V: np.ndarray, T: np.ndarray, self_term: str = "analytic"):
    """(points, s, d) of the symmetric form: centroids, sqrt(w), A_ii."""
    y, w, R = panels(V, T)
    return y, np.sqrt(w), diagonal(V, T, self_term)


def harmonic_basis(points: np.ndarray) -> np.ndarray:
    """The harmonic polynomials of degree <= 2 in 3D, one column each:
    1, x, y, z, xy, yz, zx, x^2 - y^2, x^2 + y^2 - 2 z^2."""
    x, y, z = points[:, 0], points[:, 1], points[:, 2]
    return np.stack([np.ones_like(x), x, y, z, x * y, y * z, z * x, x * x - y * y,
                     x * x + y * y - 2.0 * z * z], axis=1)


def harmonic_rhs(points: np.ndarray, coeffs) -> np.ndarray:
    """Values of the harmonic polynomial sum_k c_k h_k at the points (the
    right-hand side of a Dirichlet problem whose solution is harmonic)."""
    return harmonic_basis(points) @ np.asarray(coeffs, dtype=np.float64)


def radon7():
    """Radon's seven-point rule on a triangle (exact for polynomials of degree
    <= 5): barycentric coordinates (7, 3) and weights (7,) summing to 1.  The
    centroid with weight 9/40, and the two orbits (a, a, 1 - 2a) with
    a = (6 -+ sqrt 15) / 21 and weights (155 -+ sqrt 15) / 1200."""
    r15 = np.sqrt(15.0)
    a1, a2 = (6.0 - r15) / 21.0, (6.0 + r15) / 21.0
    w1, w2 = (155.0 - r15) / 1200.0, (155.0 + r15) / 1200.0
    bary = [[1 / 3, 1 / 3, 1 / 3]]
    wts = [9.0 / 40.0]
    for a, w in ((a1, w1), (a2, w2)):
        for k in range(3):
            b = [a, a, a]
            b[k] = 1.0 - 2.0 * a
            bary.append(b)
            wts.append(w)
    return np.array(bary), np.array(wts)


def quadrature7(V: np.ndarray, T: np.ndarray):
    """Radon's seven-point rule on every triangle: points (nt, 7, 3) and
    weights (nt, 7), the rule's weights times the triangle's area."""
    bary, wts = radon7()
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    pts = (bary[None, :, 0, None] * a[:, None, :] + bary[None, :, 1, None] * b[:, None, :]
           + bary[None, :, 2, None] * c[:, None, :])
    area = 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=1)
    return pts, area[:, None] * wts[None, :]


def near_quadrature7(V: np.ndarray, T: np.ndarray):
    """Per-panel quadrature of the symmetric form's close entries (config 5's
    near field, in the reading that keeps the operator symmetric): the entry
    between distinct panels i and j is the seven-point rule applied on both
    triangles to the double integral of 1 / (4 pi |x - y|), divided by
    s_i s_j = sqrt(w_i w_j):
        S_ij = sum_p sum_q u_ip u_jq / (4 pi |y_ip - y_jq|),  u_ip = omega_ip / s_i.
    Returns (points (nt, 7, 3), u (nt, 7)); with the centroid as the only
    point and u_i = s_i this is the one-point entry s_i s_j / (4 pi r_ij)."""
    pts, om = quadrature7(V, T)
    s = np.sqrt(om.sum(axis=1))
    return pts, om / s[:, None]


def point_source_rhs(points: np.ndarray, x0) -> np.ndarray:
    """f_j = 1 / (4 pi ||y_j - x_0||): the potential of a unit point charge at
    x_0 off the surface (Section 4.3's right-hand side)."""
    return 1.0 / (4.0 * np.pi * np.linalg.norm(points - np.asarray(x0, dtype=np.float64), axis=1))
