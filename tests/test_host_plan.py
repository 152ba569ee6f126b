"""Host-side tests of the C ABI library (no GPU needed).

* the library loads and exports every function include/h2mg.h declares;
* the host cluster tree and block partition of the library equal the
  oracle's exactly (integer parity: permutation, offsets, pair lists);
* argument validation returns the documented status codes.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import synth
from oracle.partition import build_partition
from oracle.tree import build_tree
from paper_2501_17656_amd import H2MGError, Plan
from paper_2501_17656_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "h2mg.h")).read()
    return sorted(set(re.findall(r"^\s*(?:h2mg_status|void|const char\*)\s+(h2mg_\w+)\s*\(", text, re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared()
    assert len(names) >= 20
    lib = _lib.lib()
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), "binding and header disagree"


CASES = [
    ("uniform", 4096, 2, 64, 0.7, 4),       # the 4096-point exponential workload shape
    ("uniform", 1200, 2, 32, 0.7, 3),       # ragged leaves
    ("uniform", 3000, 3, 32, 0.7, 2),
    ("uniform", 2000, 1, 16, 0.7, 4),
    ("gmm", 5000, 3, 64, 0.7, 3),           # clustered points
    ("grid", 4096, 2, 64, 0.7, 4),          # many exact coordinate ties
    ("grid", 1000, 3, 20, 1.5, 2),
    ("uniform", 50, 2, 64, 0.7, 2),         # a single leaf
]


@pytest.mark.parametrize("kind,n,dim,leaf,eta,m", CASES)
def test_plan_matches_oracle_exactly(kind, n, dim, leaf, eta, m):
    if kind == "uniform":
        P = synth.uniform_points(n, dim, 3)
    elif kind == "gmm":
        P = synth.gaussian_mixture_points(n, dim, seed=3)
    else:
        P = synth.tensor_grid_points(n, dim)
    plan = Plan(P, leaf, eta, m)
    tree = build_tree(P, leaf)
    part = build_partition(tree, eta)
    assert plan.depth == tree.L
    np.testing.assert_array_equal(plan.perm(), tree.perm)
    for d in range(tree.L + 1):
        np.testing.assert_array_equal(plan.offsets(d), tree.offsets[d])
        np.testing.assert_array_equal(plan.pairs(d, far=False), part.near[d])
        np.testing.assert_array_equal(plan.pairs(d, far=True), part.far[d])
    assert plan.d_top == part.d_top
    sizes = np.diff(tree.offsets[tree.L])
    assert (plan.leaf_min, plan.leaf_max) == (sizes.min(), sizes.max())
    assert plan.rank == m ** dim


@pytest.mark.slow
def test_plan_matches_oracle_at_matern3d_1m_size():
    w = synth.workload("matern3d_1m")
    P = w.make_points()
    plan = Plan(P, w.leaf, w.eta, w.cheb_m)
    tree = build_tree(P, w.leaf)
    part = build_partition(tree, w.eta)
    np.testing.assert_array_equal(plan.perm(), tree.perm)
    for d in range(tree.L + 1):
        np.testing.assert_array_equal(plan.pairs(d, far=True), part.far[d])
        np.testing.assert_array_equal(plan.pairs(d, far=False), part.near[d])
    assert (plan.depth, plan.d_top) == (13, part.d_top)


@pytest.mark.parametrize("args,msg", [
    (dict(n=0), "n must be"),
    (dict(dim=4), "dim must be"),
    (dict(leaf=0), "leaf_size"),
    (dict(eta=0.0), "eta"),
    (dict(eta=float("nan")), "eta"),
    (dict(m=0), "cheb_m"),
    (dict(m=5, dim=3), "exceeds 64"),
    (dict(nan=True), "non-finite"),
    (dict(n=100, leaf=8, m=4, dim=2), "fewer than the rank"),
])
def test_plan_argument_errors(args, msg):
    n, dim = args.get("n", 100), args.get("dim", 2)
    P = synth.uniform_points(max(n, 1), min(dim, 3), 0)
    if dim == 4:
        P = synth.uniform_points(max(n, 1), 4, 0)
    if args.get("nan"):
        P[7, 0] = np.nan
    if n == 0:
        P = P[:0]
    with pytest.raises(H2MGError) as ei:
        Plan(P, args.get("leaf", 16), args.get("eta", 0.7), args.get("m", 2))
    assert ei.value.status_name == "INVALID_ARG"
    assert msg in str(ei.value)


def test_null_pointers_are_rejected_not_crashing():
    lib = _lib.lib()
    h = ctypes.c_void_p()
    st = lib.h2mg_plan_create(None, 10, 2, None, ctypes.byref(h))
    assert _lib.STATUS[st] == "INVALID_ARG"
    assert b"null" in lib.h2mg_last_error()
    assert _lib.STATUS[lib.h2mg_plan_query(None, None)] == "INVALID_ARG"
    assert _lib.STATUS[lib.h2mg_destroy(None)] == "OK"
