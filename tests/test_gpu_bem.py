"""GPU parity of the scaled H2 form and of the boundary-element problem
(Laplace single layer on the bumpy torus) against the CPU oracle.

* panel quantities (centroids, sqrt(area), closed-form self term): 1e-13;
* scaled matvec diag(s) K diag(s) + diag(d), near field evaluated or stored:
  1e-12 relative (the matvec bar), for a Matern kernel with random s and d
  and for the Laplace kernel of the boundary-element matrix;
* restricted operators of the scaled form against the oracle's dense
  Galerkin products: 1e-10;
* solves: residual below 1e-8 recomputed by the oracle's matvec; the density
  sigma = W^(-1/2) y against the oracle's dense solve with A_H2 (kappa times
  the residual) and against the dense solution of the collocation system
  A sigma = f, within the compression error of this shape (1.2e-4 relative in
  the matrix, 1.9e-3 in the oracle's own density).
"""
import numpy as np
import pytest

import synth
from oracle.bem import collocation_matrix, harmonic_rhs, panels, point_source_rhs, symmetric_scaling
from oracle.galerkin import Hierarchy
from oracle.h2 import H2 as OracleH2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


_cache = {}


def bem_problem():
    if "bem" not in _cache:
        from paper_2501_17656_amd import H2Matrix, bem_panels
        V, T = synth.bumpy_torus_mesh(80, 40)
        y, s, d = bem_panels(_dev(V), _dev(T.astype(np.int64)))
        print(f"[gpu] bem torus 80x40: {len(T)} panels", flush=True)
        g = H2Matrix(y, "laplace", 1.0, 0.0, 64, 0.7, 3, scale=s, diag=d)
        yo, so, do = symmetric_scaling(V, T)
        o = OracleH2(yo, "laplace", 0.0, 64, 0.7, 3, 1.0, scale=so, diag=do)
        _cache["bem"] = (V, T, y, s, d, g, o)
    return _cache["bem"]


def test_bem_panels_match_oracle():
    V, T, y, s, d, g, o = bem_problem()
    yo, so, do = symmetric_scaling(V, T)
    np.testing.assert_allclose(_host(y), yo, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(_host(s), so, rtol=1e-14)
    np.testing.assert_allclose(_host(d), do, rtol=1e-13)
    assert np.all(_host(d) > panels(V, T)[1] / (4 * np.pi * panels(V, T)[2]))


@pytest.mark.parametrize("stored", [False, True])
def test_scaled_matern_matvec_matches_oracle(stored):
    from paper_2501_17656_amd import H2Matrix
    P = synth.uniform_points(3000, 3, 11)
    sc = 0.5 + synth.uniform_points(3000, 1, 12)[:, 0]
    dg = 1.0 + synth.uniform_points(3000, 1, 13)[:, 0]
    g = H2Matrix(_dev(P), "matern32", 0.2, 0.0, 32, 0.7, 2, scale=_dev(sc), diag=_dev(dg))
    if stored:
        g.store_near(True)
    o = OracleH2(P, "matern32", 0.0, 32, 0.7, 2, 0.2, scale=sc, diag=dg)
    x = synth.normal_vector(3000, 14)
    yv = _host(g.matvec(_dev(x)))
    yo = o.matvec(x)
    rel = np.linalg.norm(yv - yo) / np.linalg.norm(yo)
    print(f"[gpu] scaled matern matvec (stored near {stored}) rel err {rel:.2e}")
    assert rel <= 1e-12
    g.close()


@pytest.mark.parametrize("stored", [False, True])
def test_bem_matvec_matches_oracle(stored):
    V, T, y, s, d, g, o = bem_problem()
    if stored:
        g.store_near(True)
    x = synth.normal_vector(len(T), 15)
    yv = _host(g.matvec(_dev(x)))
    yo = o.matvec(x)
    rel = np.linalg.norm(yv - yo) / np.linalg.norm(yo)
    print(f"[gpu] bem matvec (stored near {stored}) rel err {rel:.2e}")
    if stored:
        g.store_near(False)
    assert rel <= 1e-12


def test_bem_restricted_operators_match_dense_galerkin():
    V, T, y, s, d, g, o = bem_problem()
    g.setup()
    H = Hierarchy(o)
    assert g.levels == H.levels
    for k in range(2, H.levels + 1):
        v = synth.normal_vector(g.level_size(k), 20 + k)
        yk = _host(g.level_apply(k, _dev(v)))
        yo = H.ops[k - 1] @ v
        rel = np.linalg.norm(yk - yo) / np.linalg.norm(yo)
        print(f"[gpu] bem level {k} rel err {rel:.2e}")
        assert rel <= 1e-10


@pytest.mark.parametrize("smoother,prec", [("cg", "fp64"), ("bj", "fp64"), ("bj", "fp32")])
def test_bem_solve_gives_the_density(smoother, prec):
    from paper_2501_17656_amd import bem_density, bem_point_source_rhs
    V, T, y, s, d, g, o = bem_problem()
    x0 = [0.0, 0.0, 1.5]
    f = bem_point_source_rhs(y, s, x0)
    yo, so, do = symmetric_scaling(V, T)
    fo = so * point_source_rhs(yo, x0)
    np.testing.assert_allclose(_host(f), fo, rtol=1e-13)
    sol, info = g.solve(f, rtol=1e-8, smoother=smoother, precision=prec)
    res = np.linalg.norm(fo - o.matvec(_host(sol))) / np.linalg.norm(fo)
    sigma = _host(bem_density(sol, s))
    sigma_h2 = np.linalg.solve(o.dense(), fo) / so
    sigma_dense = np.linalg.solve(collocation_matrix(V, T), point_source_rhs(yo, x0))
    err_h2 = np.linalg.norm(sigma - sigma_h2) / np.linalg.norm(sigma_h2)
    err = np.linalg.norm(sigma - sigma_dense) / np.linalg.norm(sigma_dense)
    print(f"[gpu] bem {smoother}/{prec}: {info['cycles']} cycles, oracle residual {res:.2e}, "
          f"density vs oracle A_H2 solve {err_h2:.2e}, vs dense collocation {err:.2e}")
    assert info["converged"] and res < 1.5e-8
    assert err_h2 < 1e-5          # kappa(S) ~ 230 times the 1e-8 residual
    assert err < 4e-3             # the oracle's own A_H2 solution is 1.9e-3 away


def test_bem_harmonic_rhs_solve_gives_the_density():
    """Dirichlet data of a random harmonic polynomial (the benchmark's
    right-hand side): the scaled values match the oracle's, and the FP32
    block-smoother solve reaches the dense collocation density within the
    compression error."""
    from paper_2501_17656_amd import bem_density, bem_harmonic_rhs
    V, T, y, s, d, g, o = bem_problem()
    c = synth.harmonic_coefficients(7)
    f = bem_harmonic_rhs(y, s, c)
    yo, so, do = symmetric_scaling(V, T)
    fo = so * harmonic_rhs(yo, c)
    np.testing.assert_allclose(_host(f), fo, rtol=1e-13, atol=1e-15 * np.abs(fo).max())
    sol, info = g.solve(f, rtol=1e-8, smoother="bj", precision="fp32")
    sigma = _host(bem_density(sol, s))
    sigma_dense = np.linalg.solve(collocation_matrix(V, T), harmonic_rhs(yo, c))
    err = np.linalg.norm(sigma - sigma_dense) / np.linalg.norm(sigma_dense)
    print(f"[gpu] bem harmonic rhs: {info['cycles']} cycles, density vs dense collocation {err:.2e}")
    assert info["converged"] and err < 4e-3


# ---------------------------------------------------------------- seven-point near field
def bem7_problem():
    """The bumpy torus of the tests above with the close entries given by
    Radon's seven-point rule on both triangles (the benchmark's near field),
    on the GPU and in the oracle."""
    if "bem7" not in _cache:
        from paper_2501_17656_amd import H2Matrix, bem_panels, bem_quadrature7
        from oracle.bem import near_quadrature7
        V, T = synth.bumpy_torus_mesh(80, 40)
        Vd, Td = _dev(V), _dev(T.astype(np.int64))
        y, s, d = bem_panels(Vd, Td)
        qy, qu = bem_quadrature7(Vd, Td)
        g = H2Matrix(y, "laplace", 1.0, 0.0, 64, 0.7, 3, scale=s, diag=d)
        g.set_near_quadrature(qy, qu)
        yo, so, do = symmetric_scaling(V, T)
        o = OracleH2(yo, "laplace", 0.0, 64, 0.7, 3, 1.0, scale=so, diag=do, near_quad=near_quadrature7(V, T))
        _cache["bem7"] = (V, T, y, s, d, qy, qu, g, o)
    return _cache["bem7"]


def test_bem_quadrature7_matches_oracle():
    from oracle.bem import near_quadrature7
    V, T, y, s, d, qy, qu, g, o = bem7_problem()
    qyo, quo = near_quadrature7(V, T)
    np.testing.assert_allclose(_host(qy), qyo, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(_host(qu), quo, rtol=1e-13)


def test_bem7_matvec_and_low_precision_products_match_oracle():
    """FP64 matvec (stored seven-point tiles) to the matvec bar, 1e-12; the
    FP32 and BF16 fine-level products (FP32 copy of the tiles) to their
    rounding bounds against the same oracle product."""
    V, T, y, s, d, qy, qu, g, o = bem7_problem()
    x = synth.normal_vector(len(T), 17)
    yo = o.matvec(x)
    yv = _host(g.matvec(_dev(x)))
    rel = np.linalg.norm(yv - yo) / np.linalg.norm(yo)
    print(f"[gpu] bem7 matvec rel err {rel:.2e}")
    assert rel <= 1e-12
    # the seven-point entries differ from the one-point ones: not the old matrix
    po, so, do = symmetric_scaling(V, T)
    base = OracleH2(po, "laplace", 0.0, 64, 0.7, 3, 1.0, scale=so, diag=do)
    assert np.linalg.norm(base.matvec(x) - yo) > 1e-5 * np.linalg.norm(yo)
    g.setup(("fp64", "fp32", "bf16"))
    for prec, tol in (("fp32", 1e-5), ("bf16", 2e-2)):
        yl = _host(g.level_apply(1, _dev(x), precision=prec))
        relp = np.linalg.norm(yl - yo) / np.linalg.norm(yo)
        print(f"[gpu] bem7 level-1 product {prec}: rel err {relp:.2e}")
        assert relp <= tol


def test_bem7_restricted_operators_match_oracle():
    V, T, y, s, d, qy, qu, g, o = bem7_problem()
    H = Hierarchy(o)
    g.setup(("fp64",))
    assert g.levels == H.levels
    for k in range(2, H.levels + 1):
        Ak = H.ops[k - 1]
        xk = synth.normal_vector(Ak.shape[0], 30 + k)
        yk = _host(g.level_apply(k, _dev(xk)))
        rel = np.linalg.norm(yk - Ak @ xk) / np.linalg.norm(Ak @ xk)
        print(f"[gpu] bem7 level {k} operator rel err {rel:.2e}")
        assert rel <= 1e-10


@pytest.mark.parametrize("precision,smoother", [("fp64", "cg"), ("fp32", "bj"), ("fp64", "bj")])
def test_bem7_solve_matches_oracle(precision, smoother):
    """Solves of the seven-point system to 1e-8: residual recomputed by the
    oracle's matvec; the density against the oracle's dense solve of the same
    A_H2 (kappa times the residual)."""
    V, T, y, s, d, qy, qu, g, o = bem7_problem()
    from paper_2501_17656_amd import bem_density, bem_harmonic_rhs
    coeffs = synth.harmonic_coefficients(7)
    f = bem_harmonic_rhs(y, s, coeffs)
    g.setup(("fp64", "fp32"))
    yv, info = g.solve(f, rtol=1e-8, precision=precision, smoother=smoother)
    fh = _host(f)
    res = np.linalg.norm(fh - o.matvec(_host(yv))) / np.linalg.norm(fh)
    A = o.dense()
    ys = np.linalg.solve(A, fh)
    kappa = np.linalg.cond(A)
    err = np.linalg.norm(_host(yv) - ys) / np.linalg.norm(ys)
    sigma = _host(bem_density(yv, s))
    print(f"[gpu] bem7 {precision} {smoother}: {info['cycles']} cycles, oracle residual {res:.2e}, "
          f"error vs dense {err:.2e} (kappa {kappa:.1e}), density norm {np.linalg.norm(sigma):.4e}")
    assert info["converged"] and res < 1e-8
    assert err <= kappa * 1e-8 * 1.5


def test_bem7_block_solve_equals_single_solves():
    """16 right-hand sides on the seven-point system (stored tiles in the
    matrix-core products): each column as the single solve, to 1e-8."""
    V, T, y, s, d, qy, qu, g, o = bem7_problem()
    n = len(T)
    B = synth.normal_vector(n, 44, nrhs=16)
    g.setup(("fp64", "fp32"))
    X, info = g.solve_multi(_dev(B), rtol=1e-8, precision="fp32", smoother="bj")
    assert info["converged"]
    Xh = _host(X)
    for k in (0, 15):
        res = np.linalg.norm(B[:, k] - o.matvec(Xh[:, k])) / np.linalg.norm(B[:, k])
        print(f"[gpu] bem7 16-column col {k}: oracle residual {res:.2e}")
        assert res < 1e-8


def test_bem7_quadrature_errors():
    from paper_2501_17656_amd import H2MGError
    V, T, y, s, d, qy, qu, g, o = bem7_problem()
    with pytest.raises(H2MGError, match="STATE"):
        g.set_near_quadrature(qy, qu)                   # twice
    with pytest.raises(H2MGError, match="STATE"):
        g.store_near(False)                             # the tiles are the only form of these entries
