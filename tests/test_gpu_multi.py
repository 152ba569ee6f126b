"""GPU parity of the product with a block of vectors (h2mg_matvec_multi,
matrix-core tile products) against the single-vector product and the oracle.

Each column of the block product must equal the single product of that
column up to rounding order (1e-13 relative) and the oracle to 1e-12 (the
matvec bar), with the near-field tiles stored or evaluated inside the
product.  Shapes: rank 64 in 3D with leaves of 64 and 128 points (chunk
order equal to the tree order) and with ragged leaves of 78-79 points (two
chunks per leaf, the second partial); rank 27 (32 x 32 padded tiles) and
rank 16 / rank 9 in 2D (16 x 16 tiles, the latter padded); 1, 5 and 16
columns; no far blocks.
"""
import numpy as np
import pytest

import synth
from oracle.h2 import H2 as OracleH2

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SHAPES = {
    # name: (n, dim, kernel, length, shift, leaf, eta, m)
    "matern3d_leaf64": (16384, 3, "matern32", 0.2, 1e-2, 64, 0.7, 4),
    "exp3d_leaf128_ragged": (10000, 3, "exp", 0.15, 1e-2, 128, 0.7, 4),
    "matern3d_no_far": (2048, 3, "matern32", 0.2, 1e-2, 64, 1e-9, 4),
    "gauss3d_r27": (6000, 3, "gauss", 0.1, 1e-2, 64, 0.7, 3),
    "exp2d_r16": (4096, 2, "exp", 0.1, 1e-2, 64, 0.7, 4),
    "exp2d_r9_ragged": (1200, 2, "exp", 0.1, 1e-2, 32, 0.7, 3),
}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("name", list(SHAPES))
def test_block_product_matches_single_products_and_oracle(name):
    from paper_2501_17656_amd import H2Matrix
    n, dim, ker, ell, shift, leaf, eta, m = SHAPES[name]
    P = synth.uniform_points(n, dim, 21)
    print(f"[gpu] build {name} n={n} leaf={leaf} rank {m ** dim}", flush=True)
    g = H2Matrix(_dev(P), ker, ell, shift, leaf, eta, m)
    g.store_near(True)
    o = OracleH2(P, ker, shift, leaf, eta, m, ell)
    X = synth.normal_vector(n, 22, nrhs=16)
    for nrhs in (1, 5, 16):
        Xk = np.ascontiguousarray(X[:, :nrhs])
        Y = _host(g.matvec_multi(_dev(Xk)))
        for k in range(nrhs):
            ys = _host(g.matvec(_dev(Xk[:, k])))
            rel = np.linalg.norm(Y[:, k] - ys) / np.linalg.norm(ys)
            assert rel <= 1e-13, (nrhs, k, rel)
        for k in ((0, nrhs - 1) if nrhs == 16 else ()):
            yo = o.matvec(Xk[:, k])
            rel = np.linalg.norm(Y[:, k] - yo) / np.linalg.norm(yo)
            print(f"[gpu] {name} nrhs={nrhs} column {k}: rel err vs oracle {rel:.2e}")
            assert rel <= 1e-12
    Y1 = _host(g.matvec_multi(_dev(X)))
    np.testing.assert_array_equal(_host(g.matvec_multi(_dev(X))), Y1)      # fixed order
    g.close()


def test_block_product_argument_errors():
    from paper_2501_17656_amd import H2Matrix, H2MGError
    P = synth.uniform_points(4096, 2, 3)
    g = H2Matrix(_dev(P), "exp", 0.1, 1e-2, 64, 0.7, 2)            # rank 4: tiles too small
    g.store_near(True)
    with pytest.raises(H2MGError):
        g.matvec_multi(_dev(np.zeros((4096, 4))))
    g.close()
    P3 = synth.uniform_points(8192, 3, 4)
    g = H2Matrix(_dev(P3), "exp", 0.1, 1e-2, 64, 0.7, 4)
    with pytest.raises(H2MGError):
        g.matvec_multi(_dev(np.zeros((8192, 17))))
    g.close()


@pytest.mark.parametrize("name", ["exp3d_leaf128_ragged", "gauss3d_r27", "exp2d_r9_ragged"])
def test_block_product_with_evaluated_near_field(name):
    """Without stored tiles the near-field tiles are evaluated inside the
    product; the result matches the oracle to the matvec bar and the
    stored-tile product up to rounding order."""
    from paper_2501_17656_amd import H2Matrix
    n, dim, ker, ell, shift, leaf, eta, m = SHAPES[name]
    P = synth.uniform_points(n, dim, 21)
    g = H2Matrix(_dev(P), ker, ell, shift, leaf, eta, m)
    o = OracleH2(P, ker, shift, leaf, eta, m, ell)
    X = synth.normal_vector(n, 23, nrhs=16)
    Ye = _host(g.matvec_multi(_dev(X)))
    g.store_near(True)
    Ys = _host(g.matvec_multi(_dev(X)))
    for k in (0, 9):
        yo = o.matvec(X[:, k])
        rel = np.linalg.norm(Ye[:, k] - yo) / np.linalg.norm(yo)
        print(f"[gpu] {name} evaluated near field, column {k}: rel err vs oracle {rel:.2e}")
        assert rel <= 1e-12
    assert np.linalg.norm(Ye - Ys) <= 1e-13 * np.linalg.norm(Ys)
    g.close()


@pytest.mark.parametrize("stored", [False, True])
def test_block_product_of_the_scaled_form(stored):
    """The scaled form diag(s) K diag(s) + diag(d) (random s, d; rank 27):
    the 16-column product with the near field evaluated or stored matches
    the oracle per column."""
    from paper_2501_17656_amd import H2Matrix
    n = 4096                       # leaves of 32 points: at least the rank
    P = synth.uniform_points(n, 3, 11)
    sc = 0.5 + synth.uniform_points(n, 1, 12)[:, 0]
    dg = 1.0 + synth.uniform_points(n, 1, 13)[:, 0]
    g = H2Matrix(_dev(P), "matern32", 0.2, 0.0, 32, 0.7, 3, scale=_dev(sc), diag=_dev(dg))
    if stored:
        g.store_near(True)
    o = OracleH2(P, "matern32", 0.0, 32, 0.7, 3, 0.2, scale=sc, diag=dg)
    X = synth.normal_vector(n, 24, nrhs=16)
    Y = _host(g.matvec_multi(_dev(X)))
    for k in (0, 5, 15):
        yo = o.matvec(X[:, k])
        rel = np.linalg.norm(Y[:, k] - yo) / np.linalg.norm(yo)
        print(f"[gpu] scaled form, stored {stored}, column {k}: rel err {rel:.2e}")
        assert rel <= 1e-12
    g.close()


def test_block_calls_reject_mismatched_out_and_x0():
    """matvec_multi's out and solve_multi's X0 must have the shape of X / B:
    a smaller buffer is refused before any launch (the library would write
    n * nrhs elements into it)."""
    from paper_2501_17656_amd import H2Matrix
    n = 1200
    P = synth.uniform_points(n, 2, 21)
    g = H2Matrix(_dev(P), "exp", 0.1, 1e-2, 32, 0.7, 3)
    X = _dev(synth.normal_vector(n, 22, nrhs=16))
    for bad in (torch.empty((n, 1), dtype=torch.float64, device="cuda"),
                torch.empty((n, 8), dtype=torch.float64, device="cuda"),
                torch.empty((n * 16,), dtype=torch.float64, device="cuda")):
        with pytest.raises(ValueError):
            g.matvec_multi(X, out=bad)
        with pytest.raises(ValueError):
            g.solve_multi(X, X0=bad, max_cycles=1)
    with pytest.raises(TypeError):
        g.matvec_multi(X, out=torch.empty((n, 16), dtype=torch.float32, device="cuda"))
    g.close()
