"""Pins of the oracle's kernels, cluster tree and block partition.

Each test checks the oracle against something other than itself: closed
forms, independent library routines (scipy's Bessel K, Python's stable sort)
or brute force over every matrix entry.
"""
import math

import numpy as np
import pytest
import scipy.special
import scipy.stats

import synth
from oracle import kernels
from oracle.partition import admissible, build_partition
from oracle.tree import build_tree, leaf_depth


# ---------------------------------------------------------------- kernels
@pytest.mark.parametrize("kind", kernels.KINDS)
def test_kernel_at_zero_is_one(kind):
    k = kernels.radial(kind, 0.3)
    assert k(np.array([0.0]))[0] == 1.0


def test_kernel_closed_forms():
    ell = 0.2
    r = np.array([ell])
    assert kernels.radial("exp", ell)(r)[0] == pytest.approx(math.exp(-1), rel=1e-15)
    assert kernels.radial("gauss", ell)(r)[0] == pytest.approx(math.exp(-0.5), rel=1e-15)
    r = np.array([ell / math.sqrt(3.0)])
    assert kernels.radial("matern32", ell)(r)[0] == pytest.approx(2 * math.exp(-1), rel=1e-15)


def _matern_general(nu, ell, r):
    z = math.sqrt(2 * nu) * r / ell
    return 2 ** (1 - nu) / scipy.special.gamma(nu) * z ** nu * scipy.special.kv(nu, z)


def test_kernels_match_matern_family_and_gaussian_pdf():
    """exp = Matern-1/2 and matern32 = Matern-3/2 (general Bessel-K form);
    gauss = scaled normal pdf."""
    ell = 0.15
    r = np.linspace(1e-3, 1.0, 57)
    np.testing.assert_allclose(kernels.radial("exp", ell)(r),
                               _matern_general(0.5, ell, r), rtol=1e-12)
    np.testing.assert_allclose(kernels.radial("matern32", ell)(r),
                               _matern_general(1.5, ell, r), rtol=1e-12)
    g = scipy.stats.norm.pdf(r, scale=ell) * math.sqrt(2 * math.pi) * ell
    np.testing.assert_allclose(kernels.radial("gauss", ell)(r), g, rtol=1e-12)


@pytest.mark.parametrize("kind", kernels.KINDS)
def test_kernel_matrix_symmetric_spd_with_shifted_diagonal(kind):
    X = synth.uniform_points(300, 3, 7)
    K = kernels.kernel_matrix(kernels.make_kernel(kind, 0.2), X, 1e-3)
    assert np.array_equal(K, K.T)
    np.testing.assert_array_equal(np.diag(K), 1.0 + 1e-3)
    np.linalg.cholesky(K)                       # raises if not SPD
    i, j = 3, 11
    rij = math.dist(X[i], X[j])
    assert K[i, j] == pytest.approx(kernels.radial(kind, 0.2)(np.array([rij]))[0], rel=1e-14)


# ---------------------------------------------------------------- tree
@pytest.mark.parametrize("n,dim,leaf", [(1200, 2, 32), (1000, 3, 37), (777, 1, 24),
                                        (64, 2, 64), (65, 2, 64), (1, 3, 8)])
def test_tree_invariants(n, dim, leaf):
    P = synth.uniform_points(n, dim, 3)
    t = build_tree(P, leaf)
    assert sorted(t.perm.tolist()) == list(range(n))          # bijection
    assert leaf * 2 ** t.L >= n and (t.L == 0 or leaf * 2 ** (t.L - 1) < n)
    Pt = P[t.perm]
    for d in range(t.L + 1):
        off = t.offsets[d]
        assert off[0] == 0 and off[-1] == n and np.all(np.diff(off) >= 0)
        for j in range(2 ** d):
            pts = Pt[off[j]:off[j + 1]]
            if len(pts):
                np.testing.assert_array_equal(t.lo[d][j], pts.min(0))   # tight box
                np.testing.assert_array_equal(t.hi[d][j], pts.max(0))
            if d < t.L:
                c = t.offsets[d + 1]
                assert c[2 * j] == off[j] and c[2 * j + 2] == off[j + 1]
                nl = c[2 * j + 1] - c[2 * j]
                assert nl == math.ceil((off[j + 1] - off[j]) / 2)
                if off[j + 1] - off[j] >= 2:
                    ext = pts.max(0) - pts.min(0)
                    ax = int(np.flatnonzero(ext == ext.max())[0])
                    left, right = pts[:nl, ax], pts[nl:, ax]
                    assert left.max() <= right.min()        # median split
    assert np.diff(t.offsets[t.L]).max() <= leaf


def test_tree_first_split_is_python_stable_sort_on_ties():
    """On a tensor grid (many equal coordinates) the first split equals
    Python's stable sort by the longest-axis coordinate."""
    P = synth.tensor_grid_points(400, 2)
    P = P * np.array([1.0, 0.5])                 # axis 0 is the longest
    t = build_tree(P, 200)                       # exactly one split
    assert t.L == 1
    expect = sorted(range(len(P)), key=lambda i: P[i, 0])
    assert t.perm.tolist() == expect


def test_tree_equal_sides_split_on_lowest_axis():
    P = synth.tensor_grid_points(256, 2)         # square: both sides equal
    t = build_tree(P, 128)
    expect = sorted(range(len(P)), key=lambda i: P[i, 0])
    assert t.perm.tolist() == expect


def test_leaf_depth():
    assert leaf_depth(1, 8) == 0 and leaf_depth(8, 8) == 0 and leaf_depth(9, 8) == 1
    assert leaf_depth(1 << 20, 128) == 13 and leaf_depth(4096, 64) == 6


# ---------------------------------------------------------------- partition
def _coverage(tree, part):
    n = tree.n
    cov = np.zeros((n, n), dtype=np.int16)
    for s, t in part.near[tree.L]:
        cov[tree.rows(tree.L, s), tree.rows(tree.L, t)] += 1
    for d in range(tree.L + 1):
        for s, t in part.far[d]:
            cov[tree.rows(d, s), tree.rows(d, t)] += 1
    return cov


@pytest.mark.parametrize("n,dim,leaf,eta", [(1200, 2, 32, 0.7), (1500, 3, 32, 0.7),
                                            (2000, 1, 16, 0.7), (900, 2, 20, 2.0)])
def test_partition_covers_every_entry_once(n, dim, leaf, eta):
    P = synth.uniform_points(n, dim, 11)
    t = build_tree(P, leaf)
    part = build_partition(t, eta)
    assert part.d_top is not None
    assert np.all(_coverage(t, part) == 1)


def test_partition_symmetry_diagonal_and_parents():
    P = synth.uniform_points(1200, 2, 4)
    t = build_tree(P, 32)
    part = build_partition(t, 0.7)
    for d in range(t.L + 1):
        for lst in (part.near[d], part.far[d]):
            fwd = set(map(tuple, lst.tolist()))
            assert fwd == {(b, a) for a, b in fwd}
        diag = {(j, j) for j in range(2 ** d)}
        assert diag <= set(map(tuple, part.near[d].tolist()))
        if d > 0:
            parents = set(map(tuple, part.near[d - 1].tolist()))
            for s, u in np.concatenate([part.near[d], part.far[d]]).tolist():
                assert (s // 2, u // 2) in parents


def test_partition_admissibility_brute_force():
    """Far pairs satisfy max diam <= eta * dist and visited near pairs do not,
    recomputed per pair with math.dist on the box corners."""
    P = synth.uniform_points(1200, 2, 4)
    t = build_tree(P, 32)
    eta = 0.7
    part = build_partition(t, eta)

    def crit(d, s, u):
        lo_s, hi_s, lo_u, hi_u = t.lo[d][s], t.hi[d][s], t.lo[d][u], t.hi[d][u]
        diam = max(math.dist(lo_s, hi_s), math.dist(lo_u, hi_u))
        gap = [max(0.0, lo_u[a] - hi_s[a], lo_s[a] - hi_u[a]) for a in range(2)]
        dist = math.hypot(*gap)
        return diam, dist

    for d in range(t.L + 1):
        for s, u in part.far[d].tolist():
            diam, dist = crit(d, s, u)
            assert dist > 0 and diam <= eta * dist * (1 + 1e-12)
        for s, u in part.near[d].tolist():
            diam, dist = crit(d, s, u)
            assert dist == 0 or diam >= eta * dist * (1 - 1e-12)


def test_partition_small_eta_has_no_far_blocks():
    P = synth.uniform_points(600, 2, 4)
    t = build_tree(P, 16)
    part = build_partition(t, 1e-8)
    assert part.d_top is None
    assert all(f.shape[0] == 0 for f in part.far)
    assert part.near[t.L].shape[0] == 4 ** t.L


def test_admissible_touching_boxes_are_never_far():
    lo = np.array([[0.0, 0.0]])
    hi = np.array([[1.0, 1.0]])
    assert not admissible(lo, hi, lo + 1.0, hi + 1.0, 1e9)[0]   # corner contact
    assert not admissible(lo, lo, lo, lo, 1.0)[0]                # point with itself
    assert admissible(lo, hi, lo + 3.0, hi + 3.0, 1.0)[0]
