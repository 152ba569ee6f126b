"""Pins of the oracle's boundary-element matrix (oracle/bem.py) and of the
scaled form of its H2 construction.

Independent references: closed forms for an equilateral triangle, the exact
area of a flat square, the single-layer potential of a uniform density on a
sphere (u = radius on the surface), the symmetric form as a similarity
transform of the paper's matrix, and exactness of the H2 construction for a
polynomial kernel in the scaled form.
"""
import numpy as np
import pytest

import synth
from oracle.bem import (collocation_matrix, panels, point_source_rhs, self_integral,
                        symmetric_scaling)
from oracle.h2 import H2
from oracle.kernels import kernel_matrix, make_kernel, polynomial_kernel


def _sphere(n_theta=40, n_phi=80, radius=1.0):
    """Latitude-longitude triangulation of a sphere (poles as single vertices)."""
    th = np.pi * np.arange(1, n_theta) / n_theta
    ph = 2 * np.pi * np.arange(n_phi) / n_phi
    T, F = np.meshgrid(th, ph, indexing="ij")
    V = radius * np.stack([np.sin(T) * np.cos(F), np.sin(T) * np.sin(F), np.cos(T)], -1).reshape(-1, 3)
    V = np.vstack([V, [[0, 0, radius]], [[0, 0, -radius]]])
    top, bot = len(V) - 2, len(V) - 1
    tris = []
    for i in range(n_theta - 2):
        for j in range(n_phi):
            a, b = i * n_phi + j, i * n_phi + (j + 1) % n_phi
            c, d = (i + 1) * n_phi + (j + 1) % n_phi, (i + 1) * n_phi + j
            tris += [[a, b, c], [a, c, d]]
    for j in range(n_phi):
        tris.append([top, (j + 1) % n_phi, j])
        k = (n_theta - 2) * n_phi
        tris.append([bot, k + j, k + (j + 1) % n_phi])
    return V, np.array(tris)


def test_panels_equilateral_and_flat_square():
    a = 0.3
    V = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * np.sqrt(3) / 2, 0]])
    y, w, R = panels(V, np.array([[0, 1, 2]]))
    assert w[0] == pytest.approx(np.sqrt(3) / 4 * a * a, rel=1e-14)
    assert R[0] == pytest.approx(a / np.sqrt(3), rel=1e-14)
    np.testing.assert_allclose(y[0], [a / 2, a * np.sqrt(3) / 6, 0], atol=1e-15)
    g = np.linspace(0, 2, 11)
    X, Y = np.meshgrid(g, g, indexing="ij")
    Vs = np.stack([X.ravel(), Y.ravel(), np.zeros(X.size)], -1)
    idx = np.arange(121).reshape(11, 11)
    Ts = np.concatenate([np.stack([idx[:-1, :-1], idx[1:, :-1], idx[1:, 1:]], -1).reshape(-1, 3),
                         np.stack([idx[:-1, :-1], idx[1:, 1:], idx[:-1, 1:]], -1).reshape(-1, 3)])
    assert panels(Vs, Ts)[1].sum() == pytest.approx(4.0, rel=1e-13)


def _polar_self_integral(V, T, nth=20000):
    """Integral of 1/r over a flat triangle around its centroid in polar
    coordinates: the integral over the angle of the distance to the boundary
    along that ray (midpoint rule in the angle)."""
    out = []
    for tri in T:
        a, b, c = V[tri]
        y = (a + b + c) / 3
        e1 = (b - a) / np.linalg.norm(b - a)
        nrm = np.cross(b - a, c - a)
        e2 = np.cross(nrm / np.linalg.norm(nrm), e1)
        pts = [np.array([(p - y) @ e1, (p - y) @ e2]) for p in (a, b, c)]
        th = 2 * np.pi * (np.arange(nth) + 0.5) / nth
        d = np.stack([np.cos(th), np.sin(th)], 1)
        rho = np.full(nth, np.inf)
        for p, q in ((pts[0], pts[1]), (pts[1], pts[2]), (pts[2], pts[0])):
            e = q - p
            den = d[:, 0] * (-e[1]) + d[:, 1] * e[0]
            with np.errstate(divide="ignore", invalid="ignore"):
                t = (p[0] * (-e[1]) + p[1] * e[0]) / den
                u = (d[:, 0] * p[1] - d[:, 1] * p[0]) / den
            ok = (t > 0) & (u >= -1e-12) & (u <= 1 + 1e-12)
            rho = np.where(ok, np.minimum(rho, t), rho)
        out.append(rho.sum() * 2 * np.pi / nth)
    return np.array(out)


def test_self_integral_closed_form_matches_polar_integration():
    V, T = synth.bumpy_torus_mesh(12, 6, bumps=4, seed=1)
    Tsub = T[::7]
    np.testing.assert_allclose(self_integral(V, Tsub), _polar_self_integral(V, Tsub), rtol=1e-6)
    a = 0.3
    Ve = np.array([[0, 0, 0], [a, 0, 0], [a / 2, a * np.sqrt(3) / 2, 0]])
    # equilateral: 3 edges at distance a/(2 sqrt 3), ends at +-a/2
    h = a / (2 * np.sqrt(3))
    r = np.hypot(a / 2, h)
    assert self_integral(Ve, np.array([[0, 1, 2]]))[0] == pytest.approx(
        3 * h * np.log((a / 2 + r) / (-a / 2 + r)), rel=1e-13)


def test_the_regularised_diagonal_is_indefinite_the_analytic_one_is_not():
    V, T = synth.bumpy_torus_mesh(24, 12, seed=0)
    for term, positive in (("paper", False), ("analytic", True)):
        y, s, d = symmetric_scaling(V, T, term)
        A = collocation_matrix(V, T, term)
        S = (s[:, None] * A) / s[None, :]
        lam = np.linalg.eigvalsh(0.5 * (S + S.T))[0]
        assert (lam > 0) == positive, (term, lam)


def test_uniform_density_on_a_sphere_gives_the_radius():
    """For a sphere of radius rho, integral of 1/(4 pi |x - y|) over the
    surface is rho at every surface point: A 1 must approach rho."""
    rho = 0.7
    V, T = _sphere(radius=rho)
    u = collocation_matrix(V, T) @ np.ones(len(T))
    assert np.abs(u / rho - 1).max() < 0.03
    assert abs(np.median(u) / rho - 1) < 0.01


def test_harmonic_basis_is_harmonic_and_independent():
    from oracle.bem import harmonic_basis
    rng = np.random.default_rng(4)
    P = rng.random((50, 3))
    h = 1e-3
    lap = -6.0 * harmonic_basis(P)
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        lap += harmonic_basis(P + e) + harmonic_basis(P - e)
    lap /= h * h
    assert np.abs(lap).max() < 1e-5            # degree <= 2: central differences are exact
    assert np.linalg.matrix_rank(harmonic_basis(P)) == 9


@pytest.mark.parametrize("k,degree", [(0, 0), (3, 1), (4, 2), (8, 2)])
def test_sphere_density_of_a_harmonic_polynomial(k, degree):
    """On a sphere of radius rho the single layer maps the surface harmonic of
    degree l to rho / (2 l + 1) times itself, so Dirichlet data given by a
    homogeneous harmonic polynomial f of degree l has the density
    sigma = (2 l + 1) f / rho.  The discretised system reproduces it away
    from the poles of the latitude-longitude mesh (|z| < 0.8 rho, where its
    triangles degenerate) to first order: the error halves when the mesh is
    refined twice in each direction."""
    from oracle.bem import harmonic_rhs, panels
    rho = 0.7
    errs = []
    for nt, nphi in ((20, 40), (40, 80)):
        V, T = _sphere(nt, nphi, radius=rho)
        y = panels(V, T)[0]
        c = np.zeros(9)
        c[k] = 1.0
        f = harmonic_rhs(y, c)
        sigma = np.linalg.solve(collocation_matrix(V, T), f)
        exact = (2 * degree + 1) * f / rho
        band = np.abs(y[:, 2]) < 0.8 * rho
        errs.append(np.linalg.norm((sigma - exact)[band]) / np.linalg.norm(exact[band]))
        big = band & (np.abs(exact) > 0.3 * np.abs(exact).max())
        assert abs(np.median(sigma[big] / exact[big]) - 1.0) < 0.02
    assert errs[1] < 0.04 and errs[1] < 0.65 * errs[0], errs


def test_symmetric_form_is_a_similarity_of_the_collocation_matrix():
    V, T = synth.bumpy_torus_mesh(24, 12, bumps=5, seed=3)
    A = collocation_matrix(V, T)
    y, s, d = symmetric_scaling(V, T)
    S = s[:, None] * kernel_matrix(make_kernel("laplace", 1.0), y, 0.0) * s[None, :]
    S[np.diag_indices_from(S)] += d
    np.testing.assert_allclose(S, (s[:, None] * A) / s[None, :], rtol=1e-13)
    np.testing.assert_allclose(S, S.T, rtol=1e-14)
    assert np.linalg.eigvalsh(S)[0] > 0
    f = point_source_rhs(y, [0.0, 0.0, 2.0])
    sigma = np.linalg.solve(A, f)
    ys = np.linalg.solve(S, s * f)
    np.testing.assert_allclose(ys / s, sigma, rtol=1e-10)


def test_scaled_h2_is_exact_for_a_polynomial_kernel_and_matches_dense():
    """The scaled form diag(s) K diag(s) + diag(d): with a polynomial kernel
    of degree m-1 the H2 approximation is exact; with the Laplace kernel and
    no far blocks the blockwise product equals the dense scaled matrix."""
    P = synth.uniform_points(500, 3, 4)
    s = 0.5 + synth.uniform_points(500, 1, 5)[:, 0]
    d = 1.0 + synth.uniform_points(500, 1, 6)[:, 0]
    h = H2(P, polynomial_kernel(3), 0.0, 20, 0.7, 4, scale=s, diag=d)
    assert sum(len(f) for f in h.part.far) > 0
    x = synth.normal_vector(500, 7)
    K = s[:, None] * kernel_matrix(polynomial_kernel(3), P, 0.0) * s[None, :] + np.diag(d)
    np.testing.assert_allclose(h.matvec(x), K @ x, rtol=1e-9, atol=1e-9 * np.abs(K @ x).max())
    V, T = synth.bumpy_torus_mesh(16, 8, bumps=3, seed=2)
    y, s2, d2 = symmetric_scaling(V, T)
    hb = H2(y, "laplace", 0.0, 16, 1e-9, 3, 1.0, scale=s2, diag=d2)
    assert sum(len(f) for f in hb.part.far) == 0
    A = collocation_matrix(V, T)
    S = (s2[:, None] * A) / s2[None, :]
    z = synth.normal_vector(len(T), 8)
    np.testing.assert_allclose(hb.matvec(z), S @ z, rtol=1e-12, atol=1e-14)


def _sphere_mean(fun, centre, radius, nt=48, nphi=96):
    """Mean of fun over the sphere |y - centre| = radius: Gauss-Legendre in
    cos(theta), the trapezoidal rule in phi (exponentially accurate for
    functions analytic on the sphere)."""
    t, wt = np.polynomial.legendre.leggauss(nt)
    phi = 2 * np.pi * np.arange(nphi) / nphi
    st = np.sqrt(1 - t * t)
    pts = np.stack([np.outer(st, np.cos(phi)), np.outer(st, np.sin(phi)),
                    np.outer(t, np.ones(nphi))], axis=-1).reshape(-1, 3)
    w = np.repeat(wt, nphi) / (2.0 * nphi)           # weights sum to 1
    return float(w @ fun(np.asarray(centre) + radius * pts))


def test_point_source_rhs_mean_value_property():
    """The point-source potential is harmonic away from x_0: its mean over a
    sphere that does not enclose x_0 is its value at the centre,
    1 / (4 pi |c - x_0|); over a sphere that encloses x_0 it is
    1 / (4 pi R) (Newton's shell theorem).  A dropped 4 pi, a squared
    distance or a sign error fails one of the two."""
    x0 = np.array([0.3, -0.2, 1.5])
    c = np.array([0.1, 0.4, -0.3])
    f = lambda y: point_source_rhs(y, x0)               # noqa: E731
    d = float(np.linalg.norm(c - x0))
    for R in (0.3 * d, 0.6 * d):
        assert abs(_sphere_mean(f, c, R) - 1.0 / (4 * np.pi * d)) <= 1e-12 / d
    for R in (1.7 * d, 3.0 * d):
        assert abs(_sphere_mean(f, c, R) - 1.0 / (4 * np.pi * R)) <= 1e-12 / R
    # positive and decreasing with the distance
    y = x0 + np.array([[1.0, 0, 0], [2.0, 0, 0], [0, 0, 4.0]])
    v = point_source_rhs(y, x0)
    assert np.all(v > 0) and np.allclose(v, 1 / (4 * np.pi * np.array([1.0, 2.0, 4.0])), rtol=1e-15)


def test_radon7_is_exact_to_degree_five():
    """Radon's rule integrates x^a y^b over the unit right triangle exactly
    (a! b! / (a + b + 2)!) for a + b <= 5, and is not exact at degree 6."""
    from math import factorial

    from oracle.bem import quadrature7, radon7
    bary, w = radon7()
    assert w.sum() == pytest.approx(1.0, abs=1e-15) and np.all(w > 0) and np.all(bary > 0)
    V = np.array([[0.0, 0, 0], [1.0, 0, 0], [0.0, 1, 0]])
    pts, om = quadrature7(V, np.array([[0, 1, 2]]))
    x, y = pts[0, :, 0], pts[0, :, 1]
    for deg in range(6):
        for a in range(deg + 1):
            b = deg - a
            exact = factorial(a) * factorial(b) / factorial(a + b + 2)
            assert om[0] @ (x ** a * y ** b) == pytest.approx(exact, rel=1e-14, abs=1e-16)
    worst = max(abs(om[0] @ (x ** a * y ** (6 - a)) - factorial(a) * factorial(6 - a) / factorial(8))
                for a in range(7))
    assert worst > 1e-6


def test_quadrature7_weights_and_points():
    """Weights sum to the triangle's area; points lie inside the triangle."""
    from oracle.bem import quadrature7
    V, T = synth.bumpy_torus_mesh(16, 8)
    y, w, _ = panels(V, T)
    pts, om = quadrature7(V, T)
    np.testing.assert_allclose(om.sum(axis=1), w, rtol=1e-14)
    np.testing.assert_allclose(pts.mean(axis=1), y, atol=1e-15)     # the rule is symmetric
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, c - a)
    for k in range(7):
        p = pts[:, k, :]
        for u, v in ((a, b), (b, c), (c, a)):
            assert np.all(np.einsum("ij,ij->i", np.cross(v - u, p - u), n) > 0)


def _refined(V3, level):
    """A triangle split into 4^level similar sub-triangles."""
    tris = [V3]
    for _ in range(level):
        nxt = []
        for a, b, c in tris:
            ab, bc, ca = (a + b) / 2, (b + c) / 2, (c + a) / 2
            nxt += [np.array([a, ab, ca]), np.array([ab, b, bc]), np.array([ca, bc, c]), np.array([ab, bc, ca])]
        tris = nxt
    return np.array(tris)


def test_near_quadrature7_double_integral_of_separated_panels():
    """For two panels a few diameters apart the seven-point rule on both
    triangles gives the double integral of 1/(4 pi |x - y|) to its
    degree-5 accuracy: compared with the same rule on 4^3 sub-triangles of
    each (converged to about 1e-12 here), within 1e-6 relative; and the
    one-point entry differs by about 1e-3, so the rule is doing work."""
    from oracle.bem import near_quadrature7, quadrature7
    A = np.array([[0.0, 0, 0], [0.1, 0, 0], [0.02, 0.09, 0.01]])
    B = A + np.array([0.25, 0.05, 0.03])
    V = np.vstack([A, B])
    T = np.array([[0, 1, 2], [3, 4, 5]])
    qy, qu = near_quadrature7(V, T)
    s = np.sqrt(panels(V, T)[1])
    r = np.linalg.norm(qy[0][:, None, :] - qy[1][None, :, :], axis=-1)
    S01 = float(qu[0] @ (1 / (4 * np.pi * r)) @ qu[1])
    ref = 0.0
    sa, sb = _refined(A, 3), _refined(B, 3)
    Vs = np.vstack([sa.reshape(-1, 3), sb.reshape(-1, 3)])
    Ts = np.arange(len(Vs)).reshape(-1, 3)
    pts, om = quadrature7(Vs, Ts)
    na = len(sa)
    pa, wa = pts[:na].reshape(-1, 3), om[:na].reshape(-1)
    pb, wb = pts[na:].reshape(-1, 3), om[na:].reshape(-1)
    for i0 in range(0, len(pa), 512):
        d = np.linalg.norm(pa[i0:i0 + 512, None, :] - pb[None, :, :], axis=-1)
        ref += float(wa[i0:i0 + 512] @ (1 / (4 * np.pi * d)) @ wb)
    ref /= s[0] * s[1]
    one = s[0] * s[1] / (4 * np.pi * np.linalg.norm(panels(V, T)[0][0] - panels(V, T)[0][1]))
    assert abs(S01 - ref) <= 5e-6 * ref
    assert abs(one - ref) >= 1e-3 * ref


def test_near_quadrature_reduces_to_the_scaled_form_and_is_spd():
    """With one quadrature point per panel (its centroid, u = s) the
    quadrature near field is exactly the scaled one-point form; with
    Radon's rule on a small bumpy torus the matrix (far blocks compressed)
    is symmetric and positive definite."""
    from oracle.bem import near_quadrature7
    V, T = synth.bumpy_torus_mesh(24, 12)
    y, s, d = symmetric_scaling(V, T)
    lap = make_kernel("laplace", 1.0)
    base = H2(y, lap, 0.0, 32, 0.7, 3, scale=s, diag=d)
    one = H2(y, lap, 0.0, 32, 0.7, 3, scale=s, diag=d, near_quad=(y[:, None, :], s[:, None]))
    np.testing.assert_allclose(one.dense(), base.dense(), rtol=1e-14, atol=1e-15)
    q7 = H2(y, lap, 0.0, 32, 0.7, 3, scale=s, diag=d, near_quad=near_quadrature7(V, T))
    A7 = q7.dense()
    assert np.abs(A7 - A7.T).max() <= 1e-15 * np.abs(A7).max()
    lam = np.linalg.eigvalsh(A7)
    assert lam[0] > 0
    # the close entries move, the far ones do not
    D = A7 - base.dense()
    assert np.abs(D).max() > 1e-4 * np.abs(A7).max()
