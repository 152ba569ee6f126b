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
        e = np.array(e0, dtype=np.float64, copy=True)
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
