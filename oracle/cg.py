"""The smoother Iter(A, r, e0): a fixed number of CG steps (oracle).

Paper: Section 3.3 uses several iterations of CG on A e = r as the smoother
Iter(A, r, e0) (operator, right-hand side, initial guess), n_f steps on the
finest level and n_c steps on the coarser ones (Remark on fine and coarse
iterations).

Reading (the paper gives no details): textbook Hestenes-Stiefel CG.
s = r - A e0 (no product when e0 is zero), p = s, gamma = s.s; each step
q = A p, delta = p.q, alpha = gamma / delta, e += alpha p, s -= alpha q,
gamma' = s.s, p = s + (gamma'/gamma) p.  The iteration stops early when
gamma is exactly zero, and delta <= 0 raises NotSPD (a non-SPD operator is
an error, not a silent stop).

A second smoother, preconditioned CG with a block-Jacobi preconditioner M
(the diagonal blocks of the level's operator, one per cluster), is a block
smoother on the leaf diagonal blocks and their coarse analogues; `pcg` is textbook
PCG: z = M^{-1} s, p = z, gamma = s.z, ..., p = z + (gamma'/gamma) p, and
`block_jacobi` applies M^{-1} block by block through Cholesky factors.

`cg_solve` is the comparison solver of the experiments: CG (or PCG) run on
A_H2 itself until the recurrence residual sqrt(s.s) / ||b|| falls below rtol.
"""
from __future__ import annotations

import numpy as np


class NotSPD(ArithmeticError):
    pass


def cg(apply, r: np.ndarray, e0=None, n: int = 1) -> np.ndarray:
    if e0 is None:
        e = np.zeros_like(r)
        s = r.copy()
    else:
        e = np.array(e0, copy=True)
        s = r - apply(e)
    p = s.copy()
    gamma = float(s @ s)
    for _ in range(n):
        if gamma == 0.0:
            break
        q = apply(p)
        delta = float(p @ q)
        if not delta > 0.0:
            raise NotSPD(f"p^T A p = {delta!r}")
        alpha = gamma / delta
        e += alpha * p
        s -= alpha * q
        gamma_new = float(s @ s)
        p = s + (gamma_new / gamma) * p
        gamma = gamma_new
    return e


def pcg(apply, precond, r: np.ndarray, e0=None, n: int = 1) -> np.ndarray:
    """n steps of preconditioned CG on A e = r; precond(s) returns M^{-1} s."""
    if e0 is None:
        e = np.zeros_like(r)
        s = r.copy()
    else:
        e = np.array(e0, copy=True)
        s = r - apply(e)
    z = precond(s)
    p = z.copy()
    gamma = float(s @ z)
    for _ in range(n):
        if gamma == 0.0:
            break
        q = apply(p)
        delta = float(p @ q)
        if not delta > 0.0:
            raise NotSPD(f"p^T A p = {delta!r}")
        alpha = gamma / delta
        e += alpha * p
        s -= alpha * q
        z = precond(s)
        gamma_new = float(s @ z)
        p = z + (gamma_new / gamma) * p
        gamma = gamma_new
    return e


def block_jacobi(A: np.ndarray, offsets):
    """M^{-1} for M = blockdiag(A[b, b]) over the row blocks
    offsets[j]:offsets[j+1]; each block by its Cholesky factorisation."""
    import scipy.linalg
    facs = []
    for j in range(len(offsets) - 1):
        s, e = int(offsets[j]), int(offsets[j + 1])
        try:
            facs.append((s, e, scipy.linalg.cho_factor(A[s:e, s:e], lower=True)))
        except np.linalg.LinAlgError as ex:
            raise NotSPD(f"diagonal block {j} is not positive definite") from ex

    def apply(v):
        out = np.empty_like(v)
        for s, e, f in facs:
            out[s:e] = scipy.linalg.cho_solve(f, v[s:e])
        return out
    return apply


def cg_solve(apply, b: np.ndarray, rtol: float = 1e-8, max_iter: int = 10000, precond=None):
    """CG (PCG when precond is given) on A x = b from x = 0.  Stops when the
    recurrence residual ||s|| / ||b|| < rtol.  Returns (x, iterations,
    converged, history of ||s|| / ||b|| before each iteration and at exit)."""
    nb = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, True, [0.0]
    s = b.copy()
    z = s if precond is None else precond(s)
    p = z.copy()
    gamma = float(s @ z)
    hist = []
    for it in range(max_iter + 1):
        rel = float(np.linalg.norm(s)) / nb
        hist.append(rel)
        if rel < rtol:
            return x, it, True, hist
        if it == max_iter:
            break
        q = apply(p)
        delta = float(p @ q)
        if not delta > 0.0:
            raise NotSPD(f"p^T A p = {delta!r}")
        alpha = gamma / delta
        x += alpha * p
        s -= alpha * q
        z = s if precond is None else precond(s)
        gamma_new = float(s @ z)
        p = z + (gamma_new / gamma) * p
        gamma = gamma_new
    return x, max_iter, False, hist
