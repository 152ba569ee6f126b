"""Pins of the oracle's restricted operators, CG smoother, V-cycle and
iterative refinement.

Independent references: plain dense Galerkin products, Cauchy interlacing,
the blockwise form of eq. a2_str, scipy's CG, dense Cholesky solves, Galerkin
orthogonality of an exact two-grid correction, monotone A-norm error, and
torch's float32 -> bfloat16 conversion.
"""
import numpy as np
import pytest
import scipy.sparse.linalg
import torch

import synth
from oracle.cg import NotSPD, block_jacobi, cg, cg_solve, pcg
from oracle.galerkin import Hierarchy, galerkin
from oracle.h2 import H2
from oracle.ir import ir_solve, lowered, near_mask, round_bf16, round_fp32, vcycle_fp32
from oracle.ortho import coarse_basis, qr_pos
from oracle.vcycle import coarsest_factor, mg_cycle, solve, vcycle


@pytest.fixture(scope="module")
def small():
    P = synth.uniform_points(777, 2, 5)
    h = H2(P, "exp", 1e-2, 24, 0.7, 3, 0.1)
    return h, Hierarchy(h)


# ---------------------------------------------------------------- Galerkin
def test_blockwise_galerkin_equals_dense_product(small):
    h, H = small
    A = H.ops[0]
    for d in (h.L, h.d_top):
        W = coarse_basis(h, d)
        np.testing.assert_allclose(galerkin(A, W, h.tree.offsets[d], h.r), W.T @ A @ W,
                                   rtol=1e-12, atol=1e-12 * np.abs(A).max())


def test_coarse_operators_interlace_and_nest(small):
    h, H = small
    ev = np.linalg.eigvalsh(H.ops[0])
    for k in range(1, H.levels):
        Ak = H.ops[k]
        assert np.abs(Ak - Ak.T).max() <= 1e-12 * np.abs(Ak).max()
        evk = np.linalg.eigvalsh(0.5 * (Ak + Ak.T))
        assert evk[0] >= ev[0] * (1 - 1e-10) and evk[-1] <= ev[-1] * (1 + 1e-10)
        if k + 1 < H.levels:
            Pk = H.prolong[k]
            np.testing.assert_allclose(Pk.T @ Ak @ Pk, H.ops[k + 1],
                                       atol=1e-11 * np.abs(Ak).max())


def test_first_restricted_operator_blocks_follow_eq_a2_str(small):
    """A_2 = U_1^T D U_1 + D_2 + ...: its close-pair blocks are Q_s^T K_st Q_t
    and its depth-L interaction-list blocks are R_s S_st R_t^T."""
    h, H = small
    A2 = H.ops[1]
    r, L = h.r, h.L
    for s, t in h.part.near[L][::37].tolist():
        Qs = qr_pos(h.basis(L, s))[0]
        Qt = qr_pos(h.basis(L, t))[0]
        np.testing.assert_allclose(A2[s * r:(s + 1) * r, t * r:(t + 1) * r],
                                   Qs.T @ h.near_block(s, t) @ Qt, atol=1e-12)
    for s, t in h.part.far[L][::29].tolist():
        Rs = qr_pos(h.basis(L, s))[1]
        Rt = qr_pos(h.basis(L, t))[1]
        np.testing.assert_allclose(A2[s * r:(s + 1) * r, t * r:(t + 1) * r],
                                   Rs @ h.coupling(L, s, t) @ Rt.T, atol=1e-12)


# ---------------------------------------------------------------- CG
def _spd(n, seed, cond=1e3):
    rng = np.random.default_rng(seed)
    Q = np.linalg.qr(rng.standard_normal((n, n)))[0]
    return (Q * np.geomspace(1, cond, n)) @ Q.T


def test_cg_exact_in_n_steps_and_first_step():
    A = _spd(8, 0, cond=10.0)
    r = synth.normal_vector(8, 1)
    e = cg(A.__matmul__, r, None, 8)
    np.testing.assert_allclose(e, np.linalg.solve(A, r), rtol=1e-9)
    e1 = cg(A.__matmul__, r, None, 1)
    np.testing.assert_allclose(e1, (r @ r) / (r @ A @ r) * r, rtol=1e-14)


def test_cg_matches_scipy_and_is_monotone_in_a_norm():
    A = _spd(60, 2, 1e4)
    b = synth.normal_vector(60, 3)
    e0 = synth.normal_vector(60, 4)
    xs = np.linalg.solve(A, b)
    prev = np.inf
    for n in (1, 3, 8, 20):
        e = cg(A.__matmul__, b, e0, n)
        ref, _ = scipy.sparse.linalg.cg(A, b, x0=e0, rtol=0.0, atol=0.0, maxiter=n)
        np.testing.assert_allclose(e, ref, rtol=1e-9, atol=1e-12)
        err = np.sqrt((e - xs) @ A @ (e - xs))
        assert err <= prev
        prev = err


def test_cg_zero_rhs_and_breakdown():
    A = _spd(5, 0)
    np.testing.assert_array_equal(cg(A.__matmul__, np.zeros(5), None, 3), 0.0)
    with pytest.raises(NotSPD):
        cg(np.diag([1.0, -1.0, 2.0]).__matmul__, np.array([0.0, 1.0, 0.0]), None, 2)


def test_pcg_identity_preconditioner_is_cg_and_matches_scipy():
    A = _spd(60, 2, 1e4)
    b = synth.normal_vector(60, 3)
    e0 = synth.normal_vector(60, 4)
    for n in (1, 4, 9):
        np.testing.assert_allclose(pcg(A.__matmul__, lambda v: v.copy(), b, e0, n),
                                   cg(A.__matmul__, b, e0, n), rtol=1e-12, atol=1e-14)
    offs = [0, 20, 45, 60]
    Minv = block_jacobi(A, offs)
    Mdense = np.zeros_like(A)
    for s, e in zip(offs[:-1], offs[1:]):
        Mdense[s:e, s:e] = np.linalg.inv(A[s:e, s:e])
    np.testing.assert_allclose(Minv(b), Mdense @ b, rtol=1e-10)
    for n in (1, 3, 8):
        ref, _ = scipy.sparse.linalg.cg(A, b, x0=e0, rtol=0.0, atol=0.0, maxiter=n,
                                        M=scipy.sparse.linalg.LinearOperator(A.shape, matvec=Minv))
        np.testing.assert_allclose(pcg(A.__matmul__, Minv, b, e0, n), ref, rtol=1e-8, atol=1e-12)


def test_pcg_with_one_exact_block_solves_in_one_step():
    A = _spd(30, 5, 1e3)
    b = synth.normal_vector(30, 6)
    e = pcg(A.__matmul__, block_jacobi(A, [0, 30]), b, None, 1)
    np.testing.assert_allclose(e, np.linalg.solve(A, b), rtol=1e-9)


# ---------------------------------------------------------------- V-cycle
def test_single_level_is_a_direct_solve():
    P = synth.uniform_points(400, 2, 1)
    h = H2(P, "exp", 1e-2, 16, 1e-9, 3, 0.1)
    H = Hierarchy(h)
    assert H.levels == 1
    b = synth.normal_vector(400, 2)
    res = solve(H, b)
    assert res.cycles == 1 and res.history[-1] < 1e-13


def test_two_grid_correction_is_galerkin_orthogonal(small):
    """Exact coarse solve, no smoothing: U_1^T (b - A x*) = 0."""
    h, H = small
    H2lvl = Hierarchy.__new__(Hierarchy)
    H2lvl.h2, H2lvl.ops, H2lvl.prolong = h, H.ops[:2], H.prolong[:1]
    b = synth.normal_vector(h.n, 6)
    x = vcycle(H2lvl, np.zeros(h.n), b, n_f=0, n_c=0)
    res = H.prolong[0].T @ (b - H.ops[0] @ x)
    assert np.linalg.norm(res) <= 1e-12 * np.linalg.norm(b) * np.linalg.cond(H.ops[1])


def test_vcycle_error_monotone_and_converges_to_cholesky(small):
    h, H = small
    A = H.ops[0]
    b = synth.normal_vector(h.n, 8)
    xs = np.linalg.solve(A, b)
    fac = coarsest_factor(H.ops[-1])
    x = np.zeros(h.n)
    prev = np.inf
    for _ in range(6):
        x = vcycle(H, x, b, 1, 40, fac)
        err = np.sqrt((x - xs) @ A @ (x - xs))
        assert err <= prev * (1 + 1e-12)
        prev = err
    res = solve(H, b, rtol=1e-8)
    assert res.converged and res.history[-1] < 1e-8
    kappa = np.linalg.cond(A)
    assert np.linalg.norm(res.x - xs) <= kappa * 1e-8 * np.linalg.norm(xs)


def test_block_smoother_vcycle_contracts_and_converges(small):
    h, H = small
    A = H.ops[0]
    b = synth.normal_vector(h.n, 8)
    xs = np.linalg.solve(A, b)
    x = np.zeros(h.n)
    prev = np.inf
    for _ in range(4):
        x = vcycle(H, x, b, 1, 40, smoother="bj")
        err = np.sqrt((x - xs) @ A @ (x - xs))
        assert err <= prev * (1 + 1e-12)
        prev = err
    res = solve(H, b, rtol=1e-8, smoother="bj")
    assert res.converged and res.history[-1] < 1e-8


def test_vcycle_is_affine_in_initial_guess(small):
    """x* = x0 + (V-cycle correction of the residual b - A x0)."""
    h, H = small
    b = synth.normal_vector(h.n, 9)
    x0 = synth.normal_vector(h.n, 10)
    a = vcycle(H, x0, b)
    c = x0 + vcycle(H, np.zeros(h.n), b - H.ops[0] @ x0)
    np.testing.assert_allclose(a, c, rtol=1e-9, atol=1e-9 * np.linalg.norm(a))


# ---------------------------------------------------------------- refinement
def test_bf16_and_fp32_rounding_match_torch():
    x = synth.normal_vector(4096, 12) * np.geomspace(1e-6, 1e6, 4096)
    x32 = x.astype(np.float32).astype(np.float64)                # exact in fp32
    ref = torch.from_numpy(x32).to(torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(round_bf16(x32), ref)
    np.testing.assert_array_equal(round_fp32(x), x.astype(np.float32))


def test_fp64_refinement_is_the_plain_iteration(small):
    h, H = small
    b = synth.normal_vector(h.n, 13)
    a = solve(H, b, rtol=1e-10)
    c = ir_solve(H, b, "fp64", rtol=1e-10)
    assert a.cycles == c.cycles
    np.testing.assert_allclose(a.history, c.history, rtol=1e-6)


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_refinement_fixed_point_is_the_fp64_solution(small, prec):
    h, H = small
    b = synth.normal_vector(h.n, 14)
    res = ir_solve(H, b, prec, rtol=1e-8)
    A = H.ops[0]
    assert res.converged
    assert np.linalg.norm(b - A @ res.x) < 1e-8 * np.linalg.norm(b)


def test_near_mask_is_the_close_leaf_blocks(small):
    """The mask covers exactly the close leaf pairs: its blocks are the
    oracle's near blocks (their entries come from the kernel, not from the
    bases), it is symmetric and holds every diagonal block; outside it,
    A_H2 is the sum of the far blocks U S U^T."""
    h, H = small
    M = near_mask(H)
    assert np.array_equal(M, M.T)
    L = h.L
    for j in range(2 ** L):
        rj = h.rows(L, j)
        assert M[rj, rj].all()
    near_entries = sum((h.rows(L, s).stop - h.rows(L, s).start) * (h.rows(L, t).stop - h.rows(L, t).start)
                       for s, t in h.part.near[L])
    assert int(M.sum()) == near_entries
    far = np.zeros_like(H.ops[0])
    for d in range(L + 1):
        for s, t in h.part.far[d]:
            far[h.rows(d, s), h.rows(d, t)] = h.basis(d, s) @ h.coupling(d, s, t) @ h.basis(d, t).T
    np.testing.assert_array_equal(np.where(M, 0.0, H.ops[0]), np.where(M, 0.0, far))


def test_lowered_policy_and_fp32_arithmetic_cycle(small):
    """lowered(H, "bf16") rounds the fine operator's close blocks to FP32 and
    everything else to BF16; the FP32-arithmetic cycle returns FP32 values
    and stays within FP32 rounding (amplified by the cycle) of the FP64
    arithmetic cycle on the same operators."""
    h, H = small
    M = near_mask(H)
    Hl = lowered(H, "bf16")
    A = H.ops[0]
    np.testing.assert_array_equal(Hl.ops[0][M], round_fp32(A[M]))
    np.testing.assert_array_equal(Hl.ops[0][~M], round_bf16(A[~M]))
    for k in range(1, H.levels - 1):
        np.testing.assert_array_equal(Hl.ops[k], round_bf16(H.ops[k]))
    np.testing.assert_array_equal(Hl.ops[-1], H.ops[-1])
    b = synth.normal_vector(h.n, 15)
    d32 = vcycle_fp32(H, b, "fp32", 1, 2)
    np.testing.assert_array_equal(d32, round_fp32(d32))
    d = vcycle(lowered(H, "fp32"), np.zeros_like(b), b, 1, 2)
    rel = np.linalg.norm(d32 - d) / np.linalg.norm(d)
    assert 0 < rel < 1e-4


# ---------------------------------------------------------------- W/F-cycles, plain CG
def _truncated(H, nlev):
    """The first nlev levels of H with the last one solved directly."""
    T = Hierarchy.__new__(Hierarchy)
    T.h2, T.ops, T.prolong = H.h2, H.ops[:nlev], H.prolong[:nlev - 1]
    return T


def test_w_and_f_cycles_equal_v_on_two_levels(small):
    """With one coarse level the coarse correction is an exact solve, so the
    second coarse call is skipped and all three cycles coincide."""
    h, H = small
    T = _truncated(H, 2)
    b = synth.normal_vector(h.n, 21)
    v = vcycle(T, np.zeros(h.n), b, 1, 3)
    for kind in ("V", "W", "F"):
        np.testing.assert_array_equal(mg_cycle(T, np.zeros(h.n), b, kind, 1, 3), v)


def test_coarsest_solves_per_cycle_follow_the_recursion(small, monkeypatch):
    """Per cycle on l levels the coarsest level is solved once (V), 2^(l-2)
    times (W) and l-1 times (F); on three levels F and W coincide."""
    import oracle.vcycle as vc
    h, H = small
    l = len(H.ops)
    calls = []
    real = vc.scipy.linalg.cho_solve
    monkeypatch.setattr(vc.scipy.linalg, "cho_solve", lambda f, r: calls.append(1) or real(f, r))
    b = synth.normal_vector(h.n, 22)
    for kind, expect in (("V", 1), ("W", 2 ** (l - 2)), ("F", l - 1)):
        calls.clear()
        mg_cycle(H, np.zeros(h.n), b, kind, 1, 3)
        assert len(calls) == expect, kind
    T = _truncated(H, 3)
    np.testing.assert_array_equal(mg_cycle(T, np.zeros(h.n), b, "F", 1, 3),
                                  mg_cycle(T, np.zeros(h.n), b, "W", 1, 3))
    np.testing.assert_array_equal(mg_cycle(H, np.zeros(h.n), b, "V", 1, 3),
                                  vcycle(H, np.zeros(h.n), b, 1, 3))


@pytest.mark.parametrize("kind", ["W", "F"])
def test_w_f_cycles_error_monotone_and_converge(small, kind):
    h, H = small
    A = H.ops[0]
    b = synth.normal_vector(h.n, 23)
    xs = np.linalg.solve(A, b)
    x = np.zeros(h.n)
    prev = np.inf
    for _ in range(4):
        x = mg_cycle(H, x, b, kind, 1, 10)
        err = np.sqrt((x - xs) @ A @ (x - xs))
        assert err <= prev * (1 + 1e-12)
        prev = err
    v = mg_cycle(H, np.zeros(h.n), b, "V", 1, 10)
    assert not np.array_equal(v, mg_cycle(H, np.zeros(h.n), b, kind, 1, 10))
    res = solve(H, b, rtol=1e-8, n_c=10, kind=kind)
    assert res.converged and res.history[-1] < 1e-8
    assert np.linalg.norm(res.x - xs) <= np.linalg.cond(A) * 1e-8 * np.linalg.norm(xs)


def test_plain_cg_solve_distinct_eigenvalues_and_scipy():
    """CG on a matrix with k distinct eigenvalues terminates in k steps; on a
    general SPD matrix its iterates match scipy's CG."""
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((60, 60)))
    lam = np.repeat([1.0, 2.0, 5.0, 7.0, 11.0], 12)
    A = (Q * lam) @ Q.T
    b = rng.standard_normal(60)
    x, it, ok, hist = cg_solve(A.__matmul__, b, rtol=1e-10, max_iter=50)
    assert ok and it == 5
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-9)
    M = rng.standard_normal((40, 40))
    A = M @ M.T + 40 * np.eye(40)
    b = rng.standard_normal(40)
    x, it, ok, hist = cg_solve(A.__matmul__, b, rtol=1e-12, max_iter=3)
    xr, _ = scipy.sparse.linalg.cg(A, b, x0=np.zeros(40), rtol=1e-30, atol=0.0, maxiter=3)
    np.testing.assert_allclose(x, xr, rtol=1e-12)
    assert not ok and len(hist) == 4
    # block-Jacobi preconditioning with the whole matrix as one block: one step
    x, it, ok, _ = cg_solve(A.__matmul__, b, rtol=1e-12, max_iter=5,
                            precond=block_jacobi(A, [0, 40]))
    assert ok and it == 1


def test_smoothing_error_components_split_the_error(small):
    """The two parts are the orthogonal split of the error: with no smoothing
    step the error is -x_true, so U_1^T e = -U_1^T x_true and the parts'
    squares add up to ||x_true||^2; with smoothing the total drops."""
    from oracle.vcycle import smoothing_error_components
    h, H = small
    xt = synth.normal_vector(h.n, 31)
    (ue, qn), = smoothing_error_components(H, xt, n_f=0, n_c=3, cycles=1)
    np.testing.assert_allclose(ue, -H.prolong[0].T @ xt, rtol=1e-13, atol=1e-13)
    assert ue @ ue + qn ** 2 == pytest.approx(xt @ xt, rel=1e-12)
    comps = smoothing_error_components(H, xt, n_f=1, n_c=10, cycles=2)
    tot = [float(np.sqrt(u @ u + q * q)) for u, q in comps]
    assert tot[0] < np.linalg.norm(xt) and tot[1] < tot[0]
