"""Tensor Chebyshev interpolation: cluster bases, transfers, couplings (oracle).

Paper: Section 3.1.  A far block is F_ij = U_i S_ij V_j with one basis per
block row and per block column (eq. f); the bases of a coarser level are
linked to the finer ones by transfer matrices (eq. s1, the U_k of
eq. h2).  The paper builds them with MCBH; here they come from tensor
Chebyshev interpolation, which gives nested bases by construction.

For a cluster s with tight box [lo, hi]:
* centre c = (lo + hi) / 2 and half-widths h = (hi - lo) / 2, with every
  h_a raised to at least 1e-9 * max_b H_b (H = the root's half-widths) so a
  flat box still maps to [-1, 1];
* 1-D nodes t_k = cos((2k + 1) pi / (2m)), k = 0..m-1 (roots of T_m), and
  cluster nodes xi_nu = c + h * (t_{nu_0}, t_{nu_1}, ...) over the tensor
  index nu with axis 0 varying fastest, so the rank is r = m^dim;
* Lagrange polynomials L_k(t) = prod_{j != k} (t - t_j) / (t_k - t_j) and the
  cluster basis U_s[i, nu] = prod_a L_{nu_a}((x_ia - c_a) / h_a) evaluated
  directly at the cluster's points (the "direct" basis, no nesting used);
* transfer from parent s to child c: E_c[nu', nu] = U_s evaluated at the
  child's node xi^c_nu' (so U_s restricted to c's rows = U_c E_c exactly in
  exact arithmetic: L^s_nu has degree m-1 per axis);
* coupling S_st[nu, mu] = k(xi^s_nu, xi^t_mu) (no diagonal shift).
"""
from __future__ import annotations

import numpy as np


def cheb_nodes(m: int) -> np.ndarray:
    k = np.arange(m, dtype=np.float64)
    return np.cos((2.0 * k + 1.0) * np.pi / (2.0 * m))


def lagrange(t: np.ndarray, nodes: np.ndarray) -> np.ndarray:
    """(n, m) matrix of L_k(t_i) for the 1-D node set."""
    t = np.asarray(t, dtype=np.float64)
    m = nodes.shape[0]
    out = np.ones((t.shape[0], m))
    for k in range(m):
        for j in range(m):
            if j != k:
                out[:, k] *= (t - nodes[j]) / (nodes[k] - nodes[j])
    return out


def box_frame(lo: np.ndarray, hi: np.ndarray, floor: float):
    """Centre and floored half-widths of a box."""
    c = 0.5 * (lo + hi)
    h = np.maximum(0.5 * (hi - lo), floor)
    return c, h


def width_floor(tree) -> float:
    H = 0.5 * (tree.hi[0][0] - tree.lo[0][0])
    return 1e-9 * float(np.max(H))


def tensor_eval(X: np.ndarray, c: np.ndarray, h: np.ndarray, m: int) -> np.ndarray:
    """U[i, nu] = prod_a L_{nu_a}((x_ia - c_a) / h_a), axis 0 fastest in nu."""
    n, dim = X.shape
    nodes = cheb_nodes(m)
    U = np.ones((n, 1))
    for a in range(dim):
        La = lagrange((X[:, a] - c[a]) / h[a], nodes)      # (n, m)
        # new index = nu_a * (m^a) + old index  (axis 0 fastest)
        U = (La[:, :, None] * U[:, None, :]).reshape(n, -1)
    return U


def cluster_nodes(c: np.ndarray, h: np.ndarray, m: int) -> np.ndarray:
    """(r, dim) interpolation nodes, axis 0 fastest."""
    dim = c.shape[0]
    t = cheb_nodes(m)
    grids = np.meshgrid(*([t] * dim), indexing="ij")      # grids[a][i0,i1,..]
    # flatten with axis 0 fastest: transpose the index order before reshape
    cols = [g.transpose(tuple(range(dim))[::-1]).reshape(-1) for g in grids]
    T = np.stack(cols, axis=1)
    return c[None, :] + h[None, :] * T


def transfer(child_c, child_h, parent_c, parent_h, m: int) -> np.ndarray:
    """E_c[nu', nu] = parent Lagrange basis nu at child node nu'."""
    return tensor_eval(cluster_nodes(child_c, child_h, m), parent_c, parent_h, m)


def coupling(kern, nodes_s: np.ndarray, nodes_t: np.ndarray) -> np.ndarray:
    return kern(nodes_s, nodes_t)
