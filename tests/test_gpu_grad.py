"""GPU parity of the derivative-kernel H2 matrices and of the gradient of
L = b^T A^{-1} b (h2mg_build_derivative, h2mg_quadratic_gradient and the
autograd function), against the CPU oracle.

Shape: the differentiation workload at N = 4096 (uniform points in [0,1)^3,
exponential kernel l = 0.15, shift 1e-2), leaf 32 and 3^3 Chebyshev nodes
(rank 27), so that far blocks exist at this size.  Tolerances:
  * derivative-kernel matvecs: 1e-12 relative (the same bar as the matvec);
  * gradient against the oracle's H2 gradient: the solve stops at 1e-12
    relative residual, so x and everything quadratic in it agree to ~1e-10;
  * against the dense FP64 gradient: within the H2 compression error of this
    shape (the oracle's own H2 gradient is 1.1e-4 (l), 4e-5 (s) and 1.7e-3
    (points) away from it);
  * against central differences of the library's loss in l and s (h = 1e-6,
    solves to 1e-12): 1e-5 relative.
"""
import numpy as np
import pytest

import synth
from oracle.grad import dense_gradient, h2_gradient
from oracle.h2 import H2 as OracleH2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

N, DIM, KIND, ELL, SHIFT, LEAF, ETA, M = 4096, 3, "exp", 0.15, 1e-2, 32, 0.7, 3


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


_state = {}


def setup_problem():
    if not _state:
        from paper_2501_17656_amd import H2Matrix
        P = synth.uniform_points(N, DIM, 0)
        b = synth.normal_vector(N, 1)
        print(f"[gpu] build {KIND} n={N} leaf={LEAF} m={M}", flush=True)
        g = H2Matrix(_dev(P), KIND, ELL, SHIFT, LEAF, ETA, M)
        x, info = g.solve(_dev(b), rtol=1e-12, smoother="bj")
        assert info["converged"]
        _state.update(P=P, b=b, g=g, x=x)
    return _state


@pytest.mark.parametrize("kind", ["exp", "gauss", "matern32"])
@pytest.mark.parametrize("which", ["dl", "g"])
def test_derivative_matvec_matches_oracle(kind, which):
    from paper_2501_17656_amd import H2Matrix
    P = synth.uniform_points(4096, 3, 2)
    g = H2Matrix(_dev(P), kind, 0.2, 1e-2, 32, 0.7, 3)
    d = g.derivative(which)
    x = synth.normal_vector(4096, 3)
    y = _host(d.matvec(_dev(x)))
    o = OracleH2(P, f"{kind}/{which}", 0.0, 32, 0.7, 3, 0.2)
    yo = o.matvec(x)
    rel = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    print(f"[gpu] {kind}/{which} matvec rel err {rel:.2e}")
    assert rel <= 1e-12
    d.close()
    g.close()


def test_gradient_matches_oracle_h2_gradient():
    st = setup_problem()
    g, x, P, b = st["g"], st["x"], st["P"], st["b"]
    hl, hg = g.derivative("dl"), g.derivative("g")
    L, dl, ds, gp, gb = g.quadratic_gradient(hl, hg, _dev(b), x, b_grad=True)
    Lo, dlo, dso, gpo = h2_gradient(P, KIND, ELL, SHIFT, b, LEAF, ETA, M)
    gp = _host(gp)
    rel_p = np.linalg.norm(gp - gpo) / np.linalg.norm(gpo)
    print(f"[gpu] L {L:.12e} / {Lo:.12e}; dl {dl:.10e} / {dlo:.10e}; ds {ds:.10e} / {dso:.10e}; "
          f"points rel {rel_p:.2e}")
    assert L == pytest.approx(Lo, rel=1e-10)
    assert dl == pytest.approx(dlo, rel=1e-9)
    assert ds == pytest.approx(dso, rel=1e-9)
    assert rel_p <= 1e-9
    np.testing.assert_allclose(_host(gb), 2.0 * _host(x), rtol=0, atol=0)
    hl.close()
    hg.close()


def test_gradient_against_dense_fp64_gradient():
    st = setup_problem()
    g, x, P, b = st["g"], st["x"], st["P"], st["b"]
    hl, hg = g.derivative("dl"), g.derivative("g")
    L, dl, ds, gp, _ = g.quadratic_gradient(hl, hg, _dev(b), x)
    L0, dl0, ds0, gp0 = dense_gradient(P, KIND, ELL, SHIFT, b)
    rel_p = np.linalg.norm(_host(gp) - gp0) / np.linalg.norm(gp0)
    print(f"[gpu] vs dense: L {abs(L - L0) / abs(L0):.2e}, dl {abs(dl - dl0) / abs(dl0):.2e}, "
          f"ds {abs(ds - ds0) / abs(ds0):.2e}, points {rel_p:.2e}")
    assert abs(L - L0) <= 1e-3 * abs(L0)
    assert abs(dl - dl0) <= 1e-3 * abs(dl0)
    assert abs(ds - ds0) <= 1e-3 * abs(ds0)
    assert rel_p <= 5e-3
    hl.close()
    hg.close()


def test_autograd_backward_and_finite_differences():
    from paper_2501_17656_amd.autograd import quadratic_loss
    st = setup_problem()
    P, b = st["P"], st["b"]
    pts = _dev(P).requires_grad_(True)
    ell = torch.tensor(ELL, dtype=torch.float64, device="cuda", requires_grad=True)
    s = torch.tensor(SHIFT, dtype=torch.float64, device="cuda", requires_grad=True)
    bd = _dev(b).requires_grad_(True)
    kw = dict(kernel=KIND, leaf=LEAF, eta=ETA, m=M, rtol=1e-12)
    loss = quadratic_loss(pts, ell, s, bd, **kw)
    (3.0 * loss).backward()
    g, x = st["g"], st["x"]
    hl, hg = g.derivative("dl"), g.derivative("g")
    L, dl, ds, gp, gb = g.quadratic_gradient(hl, hg, _dev(b), x, scale=3.0, b_grad=True)
    hl.close()
    hg.close()
    assert float(loss.detach()) == pytest.approx(L, rel=1e-10)
    assert float(ell.grad) == pytest.approx(dl, rel=1e-9)
    assert float(s.grad) == pytest.approx(ds, rel=1e-9)
    assert torch.allclose(pts.grad, gp, rtol=1e-8, atol=1e-8 * float(gp.abs().max()))
    assert torch.allclose(bd.grad, gb, rtol=1e-9, atol=0.0)
    h = 1e-6
    with torch.no_grad():
        fd_l = (float(quadratic_loss(pts, ELL + h, SHIFT, bd, **kw)) -
                float(quadratic_loss(pts, ELL - h, SHIFT, bd, **kw))) / (2 * h)
        fd_s = (float(quadratic_loss(pts, ELL, SHIFT + h, bd, **kw)) -
                float(quadratic_loss(pts, ELL, SHIFT - h, bd, **kw))) / (2 * h)
    print(f"[gpu] autograd dl {float(ell.grad) / 3:.8e} fd {fd_l:.8e}; ds {float(s.grad) / 3:.8e} fd {fd_s:.8e}")
    assert float(ell.grad) / 3.0 == pytest.approx(fd_l, rel=1e-5)
    assert float(s.grad) / 3.0 == pytest.approx(fd_s, rel=1e-5)


def test_autograd_with_mixed_precision_solve():
    """FP32 cycles inside FP64 refinement reach the same x (both solves stop
    at 1e-12), so the loss and every gradient agree with the FP64 solve's."""
    from paper_2501_17656_amd.autograd import quadratic_loss
    st = setup_problem()
    P, b = st["P"], st["b"]
    out = []
    for prec in ("fp64", "fp32"):
        pts = _dev(P).requires_grad_(True)
        ell = torch.tensor(ELL, dtype=torch.float64, device="cuda", requires_grad=True)
        s = torch.tensor(SHIFT, dtype=torch.float64, device="cuda", requires_grad=True)
        loss = quadratic_loss(pts, ell, s, _dev(b), kernel=KIND, leaf=LEAF, eta=ETA, m=M, rtol=1e-12,
                              precision=prec)
        loss.backward()
        out.append((float(loss.detach()), float(ell.grad), float(s.grad), pts.grad.clone()))
    (L0, l0, s0, p0), (L1, l1, s1, p1) = out
    assert L1 == pytest.approx(L0, rel=1e-9)
    assert l1 == pytest.approx(l0, rel=1e-8) and s1 == pytest.approx(s0, rel=1e-8)
    assert torch.allclose(p1, p0, rtol=1e-7, atol=1e-7 * float(p0.abs().max()))


def test_gradient_argument_errors():
    from paper_2501_17656_amd import H2Matrix, H2MGError
    st = setup_problem()
    g, x, b = st["g"], st["x"], st["b"]
    with pytest.raises(H2MGError):
        g.derivative("value")
    other = H2Matrix(_dev(synth.uniform_points(N, DIM, 7)), KIND, ELL, SHIFT, LEAF, ETA, M)
    og = other.derivative("g")
    with pytest.raises(H2MGError):
        g.quadratic_gradient(None, og, _dev(b), x)       # built on other points
    with pytest.raises(H2MGError):
        g.quadratic_gradient(og, None, _dev(b), x)       # not the length-scale derivative
    og.close()
    other.close()
