"""Pins of the oracle's derivative kernels and of the gradient of the
quadratic loss L = b^T A^{-1} b (oracle/grad.py).

Independent references: central finite differences of the kernel profiles
and of the dense loss itself (every gradient component, so a dropped factor
2, a sign or a transposed difference p_i - p_j fails), and the exactness of
the length-scale and shift derivatives of the H2 loss (tensor interpolation
is linear in the kernel and the tree does not depend on l or s).
"""
import numpy as np
import pytest

import synth
from oracle.grad import dense_gradient, dense_loss, h2_gradient, h2_loss
from oracle.h2 import H2
from oracle.kernels import radial

KINDS = ["exp", "gauss", "matern32"]


@pytest.mark.parametrize("kind", KINDS)
def test_derivative_profiles_match_finite_differences(kind):
    r = np.array([0.03, 0.1, 0.27, 0.6, 1.1])
    ell, h = 0.2, 1e-6
    fd_l = (radial(kind, ell + h)(r) - radial(kind, ell - h)(r)) / (2 * h)
    np.testing.assert_allclose(radial(kind + "/dl", ell)(r), fd_l, rtol=1e-7)
    k = radial(kind, ell)
    fd_r = (k(r + h) - k(r - h)) / (2 * h)
    np.testing.assert_allclose(radial(kind + "/g", ell)(r) * r, fd_r, rtol=1e-7)
    assert radial(kind + "/g", ell)(np.array([0.0]))[0] == 0.0
    assert radial(kind + "/dl", ell)(np.array([0.0]))[0] == 0.0


@pytest.mark.parametrize("kind", KINDS)
def test_dense_gradient_matches_finite_differences_of_the_loss(kind):
    P = synth.uniform_points(120, 3, 4)
    b = synth.normal_vector(120, 5)
    ell, s, h = 0.3, 0.1, 1e-6
    L, dl, ds, gp = dense_gradient(P, kind, ell, s, b)
    assert L == pytest.approx(dense_loss(P, kind, ell, s, b)[0], rel=1e-14)
    fd_l = (dense_loss(P, kind, ell + h, s, b)[0] - dense_loss(P, kind, ell - h, s, b)[0]) / (2 * h)
    fd_s = (dense_loss(P, kind, ell, s + h, b)[0] - dense_loss(P, kind, ell, s - h, b)[0]) / (2 * h)
    assert dl == pytest.approx(fd_l, rel=1e-6)
    assert ds == pytest.approx(fd_s, rel=1e-6)
    for i, a in [(0, 0), (7, 1), (55, 2), (119, 0)]:
        Pp, Pm = P.copy(), P.copy()
        Pp[i, a] += h
        Pm[i, a] -= h
        fd = (dense_loss(Pp, kind, ell, s, b)[0] - dense_loss(Pm, kind, ell, s, b)[0]) / (2 * h)
        assert gp[i, a] == pytest.approx(fd, rel=1e-5, abs=1e-7 * np.abs(gp).max())


def test_h2_length_scale_and_shift_derivatives_are_exact():
    """dA_H2/dl is the H2 interpolant of dk/dl on the same tree and nodes, so
    the H2 gradient in l and s equals finite differences of the H2 loss."""
    P = synth.uniform_points(600, 2, 6)
    b = synth.normal_vector(600, 7)
    ell, s, h = 0.15, 1e-2, 1e-6
    assert sum(len(f) for f in H2(P, "exp", s, 32, 0.7, 4, ell).part.far) > 0
    args = (P, "exp")
    L, dl, ds, gp = h2_gradient(P, "exp", ell, s, b, 32, 0.7, 4)
    fd_l = (h2_loss(*args, ell + h, s, b, 32, 0.7, 4)[0] - h2_loss(*args, ell - h, s, b, 32, 0.7, 4)[0]) / (2 * h)
    fd_s = (h2_loss(*args, ell, s + h, b, 32, 0.7, 4)[0] - h2_loss(*args, ell, s - h, b, 32, 0.7, 4)[0]) / (2 * h)
    assert dl == pytest.approx(fd_l, rel=1e-6)
    assert ds == pytest.approx(fd_s, rel=1e-6)


def test_h2_gradient_approaches_the_dense_gradient_with_the_order():
    P = synth.uniform_points(800, 2, 8)
    b = synth.normal_vector(800, 9)
    _, dl0, ds0, gp0 = dense_gradient(P, "matern32", 0.2, 1e-2, b)
    errs = []
    for m in (3, 5, 7):
        _, dl, ds, gp = h2_gradient(P, "matern32", 0.2, 1e-2, b, 32, 0.7, m)
        errs.append(max(abs(dl - dl0) / abs(dl0), abs(ds - ds0) / abs(ds0),
                        np.linalg.norm(gp - gp0) / np.linalg.norm(gp0)))
    assert errs[0] > errs[1] > errs[2]
    assert errs[2] < 1e-4
