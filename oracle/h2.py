"""The H2 matrix and its matvec, by their plain definitions (oracle).

Paper: Section 3.1.  A = D + F with D the close blocks and
F = U_1 S_1 V_1 (eq. h20), and the coupling matrix of each level split again
as S_{k-1} = D_k + U_k S_k V_k (eq. s1) down to the last level (eq. h2).  The
matvec recursion that follows eq. h2 (x_i = V_i x_{i-1} upward,
y_{i-1} = D_i x_{i-1} + U_i y_i downward, y = D x + U_1 y_1) computes, up to
rounding, exactly the product with the matrix

    A_H2 = sum over close leaf pairs (s, t) of   K[I_s, I_t]
         + sum over far pairs (s, t), any depth,  U_s S_st U_t^T

where U_s is the cluster basis of s evaluated directly at its points (the
nested bases reproduce it exactly, see cheb.py).  So the oracle multiplies by
that sum, block by block, with direct (non-nested, non-orthogonalised) bases.

Readings: the symmetric case V_i = U_i^T (one tree for rows and columns);
the garbled "S_i x_i" term of the recursion is read as the level's
interaction-list couplings D_{i+1} x_i (the recursion's own definition
y_{i-1} = D_i x_{i-1} + U_i y_i is taken as authoritative).
"""
from __future__ import annotations

import numpy as np

from . import cheb
from .kernels import kernel_matrix, make_kernel
from .partition import build_partition
from .tree import build_tree


class H2:
    """Direct-basis H2 approximation of a kernel matrix.

    `kern` is a callable k(X, Y) (see kernels.py) or a kind name.  Vectors
    passed to the public methods are in user order.

    Scaled form: with per-point `scale` s and `diag` d (user order), the
    matrix is diag(s) K diag(s) + diag(d) (d replaces the constant shift),
    so every block gets s on its rows and columns and the cluster bases are
    diag(s_rows) U.  This is the symmetric W^(1/2) G W^(1/2) form of the
    collocation matrix of the boundary-element experiment (Section 4.3):
    s = sqrt(panel area), d = area / (4 pi R_i), k = 1 / (4 pi r).
    """

    def __init__(self, points, kern, shift, leaf, eta, m, length_scale=None, scale=None,
                 diag=None, near_quad=None):
        if isinstance(kern, str):
            kern = make_kernel(kern, length_scale)
        self.kern = kern
        self.shift = float(shift)
        self.points = np.asarray(points, dtype=np.float64)
        self.n, self.dim = self.points.shape
        self.m = int(m)
        self.r = self.m ** self.dim
        self.tree = build_tree(self.points, leaf)
        self.part = build_partition(self.tree, eta)
        self.L = self.tree.L
        self.P = self.points[self.tree.perm]          # tree-ordered points
        perm = self.tree.perm
        self.sc = None if scale is None else np.asarray(scale, dtype=np.float64)[perm]
        self.dg = None if diag is None else np.asarray(diag, dtype=np.float64)[perm]
        # close entries by quadrature: point i carries sub-points Y[i, p] with
        # weights U[i, p], and the entry between distinct points i, j of a close
        # leaf pair is sum_p sum_q U[i, p] U[j, q] k(|Y[i, p] - Y[j, q]|)
        # (far blocks keep the point values; the diagonal keeps d or the shift)
        self.qy = self.qu = None
        if near_quad is not None:
            self.qy = np.asarray(near_quad[0], dtype=np.float64)[perm]
            self.qu = np.asarray(near_quad[1], dtype=np.float64)[perm]
        floor = cheb.width_floor(self.tree)
        self.c, self.h = [], []
        for d in range(self.L + 1):
            c, h = cheb.box_frame(self.tree.lo[d], self.tree.hi[d], floor)
            self.c.append(c)
            self.h.append(h)
        self._U = {}

    # ---- pieces -------------------------------------------------------
    @property
    def d_top(self):
        return self.part.d_top

    def rows(self, d, j):
        return self.tree.rows(d, j)

    def _basis_at(self, d, j, rows) -> np.ndarray:
        U = cheb.tensor_eval(self.P[rows], self.c[d][j], self.h[d][j], self.m)
        return U if self.sc is None else self.sc[rows, None] * U

    def basis(self, d, j) -> np.ndarray:
        """Direct cluster basis U_s (n_s x r) of cluster j at depth d (rows
        scaled by s in the scaled form)."""
        key = (d, j)
        if key not in self._U:
            self._U[key] = self._basis_at(d, j, self.rows(d, j))
        return self._U[key]

    def nodes(self, d, j) -> np.ndarray:
        return cheb.cluster_nodes(self.c[d][j], self.h[d][j], self.m)

    def coupling(self, d, s, t) -> np.ndarray:
        return cheb.coupling(self.kern, self.nodes(d, s), self.nodes(d, t))

    def transfer(self, d, j) -> np.ndarray:
        """E_c for child j at depth d (d >= 1) to its parent j // 2."""
        p = j // 2
        return cheb.transfer(self.c[d][j], self.h[d][j],
                             self.c[d - 1][p], self.h[d - 1][p], self.m)

    def near_block(self, s, t) -> np.ndarray:
        """Close leaf block K[I_s, I_t] (shift, or d, on the diagonal when
        s == t; rows and columns scaled by s in the scaled form)."""
        rs, rt = self.rows(self.L, s), self.rows(self.L, t)
        Xs = self.P[rs]
        if self.qy is not None:
            return self._quad_block(rs, rt, s == t)
        if s == t:
            K = kernel_matrix(self.kern, Xs, 0.0 if self.dg is not None else self.shift)
        else:
            K = kernel_matrix(self.kern, Xs, self.shift, self.P[rt])
        if self.sc is not None:
            K = self.sc[rs, None] * K * self.sc[None, rt]
        if s == t and self.dg is not None:
            K[np.diag_indices_from(K)] += self.dg[rs]
        return K

    def _quad_block(self, rs, rt, diagonal):
        """Close block by quadrature on both points (see __init__)."""
        ys, us = self.qy[rs], self.qu[rs]            # (ns, q, dim), (ns, q)
        yt, ut = self.qy[rt], self.qu[rt]
        ns, q, dim = ys.shape
        nt = yt.shape[0]
        K = np.zeros((ns, nt))
        for p in range(q):
            for r in range(q):
                Kpr = kernel_matrix(self.kern, ys[:, p, :], 0.0, yt[:, r, :])
                K += us[:, p, None] * Kpr * ut[None, :, r]
        if diagonal:
            K[np.diag_indices_from(K)] = self.dg[rs] if self.dg is not None else self.shift
        return K

    # ---- products -----------------------------------------------------
    def matvec_tree(self, xt: np.ndarray) -> np.ndarray:
        """y = A_H2 x with x, y in tree order (blockwise definition)."""
        xt = np.asarray(xt, dtype=np.float64)
        y = np.zeros_like(xt)
        L = self.L
        for s, t in self.part.near[L]:
            y[self.rows(L, s)] += self.near_block(s, t) @ xt[self.rows(L, t)]
        for d in range(L + 1):
            far = self.part.far[d]
            if far.shape[0] == 0:
                continue
            xhat = {}
            yhat = {}
            for s, t in far:
                if t not in xhat:
                    xhat[t] = self.basis(d, t).T @ xt[self.rows(d, t)]
                yhat[s] = yhat.get(s, 0.0) + self.coupling(d, s, t) @ xhat[t]
            for s, v in yhat.items():
                y[self.rows(d, s)] += self.basis(d, s) @ v
        return y

    def matvec(self, x: np.ndarray) -> np.ndarray:
        """y = A_H2 x in user order."""
        x = np.asarray(x, dtype=np.float64)
        perm = self.tree.perm
        yt = self.matvec_tree(x[perm])
        y = np.empty_like(yt)
        y[perm] = yt
        return y

    def matvec_rows(self, x: np.ndarray, leaf: int) -> np.ndarray:
        """Rows of one leaf (tree order) of y = A_H2 x, x in user order.

        The same blockwise sum as matvec_tree restricted to the block rows
        that contain the leaf: its close leaf pairs, and at every depth the
        far pairs of the leaf's ancestor (parent basis restricted to the
        leaf's rows).  Cost O(n_leaf * n) at most, so it can sample any size.
        """
        xt = np.asarray(x, dtype=np.float64)[self.tree.perm]
        L = self.L
        lr = self.rows(L, leaf)
        y = np.zeros(lr.stop - lr.start)
        near = self.part.near[L]
        lo, hi = np.searchsorted(near[:, 0], [leaf, leaf + 1])
        for s, t in near[lo:hi]:
            y += self.near_block(s, t) @ xt[self.rows(L, t)]
        for d in range(L + 1):
            far = self.part.far[d]
            anc = leaf >> (L - d)
            lo, hi = np.searchsorted(far[:, 0], [anc, anc + 1])
            if hi == lo:
                continue
            Ua = self._basis_at(d, anc, lr)
            acc = np.zeros(self.r)
            for s, t in far[lo:hi]:
                tr = self.rows(d, t)
                Ut = self._basis_at(d, t, tr)
                acc += self.coupling(d, s, t) @ (Ut.T @ xt[tr])
            y += Ua @ acc
        return y

    def dense_tree(self) -> np.ndarray:
        """A_H2 as a dense matrix in tree order (small N only)."""
        A = np.zeros((self.n, self.n))
        L = self.L
        for s, t in self.part.near[L]:
            A[self.rows(L, s), self.rows(L, t)] = self.near_block(s, t)
        for d in range(L + 1):
            for s, t in self.part.far[d]:
                A[self.rows(d, s), self.rows(d, t)] = (
                    self.basis(d, s) @ self.coupling(d, s, t) @ self.basis(d, t).T)
        return A

    def dense(self) -> np.ndarray:
        """A_H2 as a dense matrix in user order."""
        At = self.dense_tree()
        perm = self.tree.perm
        A = np.empty_like(At)
        A[np.ix_(perm, perm)] = At
        return A

    def kernel_dense(self) -> np.ndarray:
        """The exact kernel matrix K in user order (small N only), in the
        scaled form diag(s) K diag(s) + diag(d) when given."""
        if self.sc is None and self.dg is None:
            return kernel_matrix(self.kern, self.points, self.shift)
        perm = self.tree.perm
        s = np.ones(self.n) if self.sc is None else np.empty(self.n)
        if self.sc is not None:
            s[perm] = self.sc
        K = kernel_matrix(self.kern, self.points, 0.0 if self.dg is not None else self.shift)
        K = s[:, None] * K * s[None, :]
        if self.dg is not None:
            d = np.empty(self.n)
            d[perm] = self.dg
            K[np.diag_indices_from(K)] += d
        return K
