"""Pins of the oracle's Chebyshev bases and H2 matrix.

Independent references: numpy's Chebyshev polynomials, scipy's barycentric
interpolator, the exactness of interpolation on polynomial kernels (which
makes A_H2 equal the kernel matrix for any partition), the densified matrix,
and the plain kernel matrix.
"""
import numpy as np
import pytest
import scipy.interpolate
from numpy.polynomial import chebyshev

import synth
from oracle import cheb, kernels
from oracle.h2 import H2
from oracle.ortho import coarse_basis, qr_pos


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6])
def test_nodes_are_roots_of_T_m(m):
    t = cheb.cheb_nodes(m)
    coef = np.zeros(m + 1)
    coef[m] = 1.0
    np.testing.assert_allclose(chebyshev.chebval(t, coef), 0.0, atol=1e-14)
    assert len(np.unique(t)) == m and np.all(np.abs(t) < 1)


@pytest.mark.parametrize("m", [2, 3, 4, 5])
def test_lagrange_matches_barycentric_interpolation(m):
    nodes = cheb.cheb_nodes(m)
    np.testing.assert_allclose(cheb.lagrange(nodes, nodes), np.eye(m), atol=1e-15)
    f = np.cos(3.0 * nodes) + nodes ** 2
    t = np.linspace(-1, 1, 41)
    ref = scipy.interpolate.BarycentricInterpolator(nodes, f)(t)
    np.testing.assert_allclose(cheb.lagrange(t, nodes) @ f, ref, rtol=1e-13, atol=1e-13)


@pytest.mark.parametrize("dim,m", [(1, 4), (2, 3), (3, 4)])
def test_tensor_basis_unity_reproduction_and_node_order(dim, m):
    rng = np.random.default_rng(0)
    c = rng.random(dim)
    h = 0.1 + rng.random(dim)
    X = c + h * (2 * rng.random((50, dim)) - 1)
    U = cheb.tensor_eval(X, c, h, m)
    np.testing.assert_allclose(U.sum(axis=1), 1.0, atol=1e-13)     # partition of unity
    xi = cheb.cluster_nodes(c, h, m)
    np.testing.assert_allclose(cheb.tensor_eval(xi, c, h, m), np.eye(m ** dim), atol=1e-13)
    # node order: axis 0 varies fastest
    if dim >= 2:
        assert xi[0, 1] == xi[1, 1] and xi[0, 0] != xi[1, 0]
    # any polynomial of degree m-1 per axis is reproduced exactly
    coef = rng.standard_normal([m] * dim)

    def q(Y):
        out = np.zeros(len(Y))
        for idx in np.ndindex(*coef.shape):
            out += coef[idx] * np.prod([Y[:, a] ** idx[a] for a in range(dim)], axis=0)
        return out
    np.testing.assert_allclose(U @ q(xi), q(X), rtol=1e-11, atol=1e-11)


def _small(kern="exp", n=1200, dim=2, leaf=32, m=3, eta=0.7, seed=5, shift=1e-2, ell=0.1):
    return H2(synth.uniform_points(n, dim, seed), kern, shift, leaf, eta, m, ell)


def test_nested_bases_reproduce_direct_bases():
    h = _small()
    for d in range(h.d_top, h.L):
        for j in range(0, 2 ** d, 5):
            U = h.basis(d, j)
            for c in (2 * j, 2 * j + 1):
                s = h.tree.offsets[d + 1][c] - h.tree.offsets[d][j]
                e = s + h.tree.size(d + 1, c)
                np.testing.assert_allclose(h.basis(d + 1, c) @ h.transfer(d + 1, c),
                                           U[s:e], rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dim,m,n,leaf", [(2, 3, 1200, 32), (3, 2, 1500, 32), (1, 4, 2000, 16)])
def test_polynomial_kernel_makes_h2_exact(dim, m, n, leaf):
    """Interpolation of degree m-1 per axis is exact on a kernel of that
    degree, so A_H2 must equal K whatever the partition."""
    P = synth.uniform_points(n, dim, 2)
    h = H2(P, kernels.polynomial_kernel(m - 1), 0.5, leaf, 0.7, m)
    assert sum(f.shape[0] for f in h.part.far) > 0
    K = h.kernel_dense()
    A = h.dense()
    assert np.linalg.norm(A - K) <= 1e-12 * np.linalg.norm(K)


def test_blockwise_matvec_equals_densified_and_is_symmetric():
    h = _small(n=777, leaf=24)
    A = h.dense()
    x = synth.normal_vector(h.n, 3)
    y = h.matvec(x)
    assert np.linalg.norm(A @ x - y) <= 1e-13 * np.linalg.norm(y)
    assert np.abs(A - A.T).max() <= 1e-15 * np.abs(A).max()
    z = synth.normal_vector(h.n, 4)
    assert abs(z @ h.matvec(x) - x @ h.matvec(z)) <= 1e-12 * np.linalg.norm(y) * np.linalg.norm(z)
    np.testing.assert_allclose(h.matvec(2.0 * x - z), 2.0 * y - h.matvec(z), rtol=1e-12, atol=1e-12)


def test_sampled_rows_equal_full_matvec():
    h = _small(n=1200, leaf=32, m=3)
    x = synth.normal_vector(h.n, 5)
    yt = h.matvec_tree(x[h.tree.perm])
    for leaf in (0, 13, 2 ** h.L - 1):
        r = h.rows(h.L, leaf)
        np.testing.assert_allclose(h.matvec_rows(x, leaf), yt[r], rtol=1e-13, atol=1e-13)


def test_no_far_blocks_means_exact_kernel_matrix():
    h = _small(n=500, leaf=16, eta=1e-9)
    assert h.d_top is None
    np.testing.assert_array_equal(h.dense(), h.kernel_dense())


def test_compression_error_decays_with_order():
    errs = []
    for m in (2, 3, 4, 5):
        h = _small(n=1200, leaf=32, m=m)
        K = h.kernel_dense()
        errs.append(np.linalg.norm(h.dense() - K) / np.linalg.norm(K))
    assert all(a > b for a, b in zip(errs, errs[1:]))
    assert errs[-1] < 1e-5


def test_exp2d_4k_compression_error_and_structure():
    w = synth.workload("exp2d_4k")
    h = H2(w.make_points(), w.kernel, w.shift, w.leaf, w.eta, w.cheb_m, w.length_scale)
    assert (h.L, h.d_top) == (6, 4)
    assert h.part.near[h.L].shape[0] == 1440
    assert sum(f.shape[0] for f in h.part.far) == 1522
    K = h.kernel_dense()
    err = np.linalg.norm(h.dense() - K) / np.linalg.norm(K)
    assert 1e-6 < err < 1e-4


# ---------------------------------------------------------------- orthonormal bases
def test_qr_pos_and_coarse_basis():
    h = _small(n=777, leaf=24)
    for d in range(h.d_top, h.L + 1):
        W = coarse_basis(h, d)
        np.testing.assert_allclose(W.T @ W, np.eye(W.shape[1]), atol=1e-13)
        for j in range(0, 2 ** d, 7):
            U = h.basis(d, j)
            Q, R = qr_pos(U)
            assert np.all(np.diag(R) > 0) and np.allclose(np.triu(R), R)
            np.testing.assert_allclose(Q @ R, U, atol=1e-13)
        if d < h.L:                                    # nested coarse spaces
            Wf = coarse_basis(h, d + 1)
            np.testing.assert_allclose(Wf @ (Wf.T @ W), W, atol=1e-12)


def test_orthogonalised_coupling_gives_same_block():
    h = _small(n=777, leaf=24)
    d = h.L
    s, t = h.part.far[d][0]
    Qs, Rs = qr_pos(h.basis(d, s))
    Qt, Rt = qr_pos(h.basis(d, t))
    S = h.coupling(d, s, t)
    np.testing.assert_allclose(Qs @ (Rs @ S @ Rt.T) @ Qt.T,
                               h.basis(d, s) @ S @ h.basis(d, t).T, rtol=1e-12, atol=1e-14)
