"""Pins of the oracle's Chebyshev H2 representation (R1) and its product.

Paper: Sec. 2.1 (A = S + U K V^T, nested over levels) and Sec. 3 opening
(Chebyshev interpolation). Pins: the Lagrange property, exact reproduction of
polynomials (a radial quadratic kernel is reproduced exactly by order >= 3),
convergence of the far-field error as the order grows, and the product
against the dense definition.
"""
import numpy as np
import pytest

import workloads as W
from oracle import chebyshev as cheb
from oracle import kernels
from oracle.h2 import H2
from oracle.tree import Tree


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_lagrange_property(n):
    t = cheb.nodes(n)
    assert np.allclose(cheb.lagrange_1d(n, t), np.eye(n), atol=1e-14)
    g = cheb.node_grid(n, 3)
    assert np.allclose(cheb.lagrange_nd(n, g), np.eye(n ** 3), atol=1e-13)


def test_nodes_are_first_kind_chebyshev():
    # roots of T_n: cos(n arccos t) = 0
    for n in (2, 3, 4, 7):
        t = cheb.nodes(n)
        assert np.allclose(np.cos(n * np.arccos(t)), 0.0, atol=1e-13)
        assert len(set(np.round(t, 12))) == n


def test_interpolation_reproduces_polynomials():
    rng = np.random.default_rng(0)
    X = rng.uniform(-1, 1, (50, 2))
    n = 4
    g = cheb.node_grid(n, 2)
    f = lambda P: 1 + 2 * P[:, 0] - P[:, 1] ** 3 + P[:, 0] ** 2 * P[:, 1] ** 3
    approx = cheb.lagrange_nd(n, X) @ f(g)
    assert np.allclose(approx, f(X), atol=1e-13)


@pytest.mark.parametrize("dim,depth", [(2, 3), (3, 3)])
def test_poly2_kernel_reproduced_exactly(dim, depth):
    pts = W.uniform_cube(300, dim, 21)
    tr = Tree(pts, depth)
    h = H2(tr, "poly2", 0.0, 1.0, 3)
    A = kernels.dense("poly2", 0.0, 1.0, pts)
    At = h.dense()
    assert np.linalg.norm(At - A) <= 1e-12 * np.linalg.norm(A)


def test_far_field_error_decreases_with_order():
    pts = W.uniform_cube(400, 2, 23)
    tr = Tree(pts, 3)
    A = kernels.dense("imq", 0.05, 1.0, pts)
    errs = []
    for n in (1, 2, 3, 4, 5, 6):
        At = H2(tr, "imq", 0.05, 1.0, n).dense()
        errs.append(np.linalg.norm(At - A) / np.linalg.norm(A))
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1))
    assert errs[-1] < 1e-4


def test_near_field_and_diagonal_exact():
    pts = W.uniform_cube(256, 2, 25)
    tr = Tree(pts, 3)
    h = H2(tr, "gauss", 0.1, 0.1, 3)
    At = h.dense()
    A = kernels.dense("gauss", 0.1, 0.1, pts)
    # pairs in adjacent leaves are represented exactly (P2P)
    L = tr.L
    lev = tr.levels[L]
    for i in range(0, lev.nb, 7):
        for j in lev.nbrs[i]:
            si = tr.perm[tr.leaf_points(i)]
            sj = tr.perm[tr.leaf_points(j)]
            assert np.allclose(At[np.ix_(si, sj)], A[np.ix_(si, sj)], rtol=0, atol=1e-15)


def test_matvec_many_rhs_consistent():
    wl = W.small_uniform(500, 3, 27, 3, 3, 1e-6)
    tr = Tree(wl.points, 3)
    h = H2(tr, wl.kernel, wl.kparam, wl.shift, 3)
    X = np.random.default_rng(1).standard_normal((500, 3))
    Y = h.matvec(X)
    for k in range(3):
        assert np.allclose(h.matvec(X[:, k]), Y[:, k], rtol=0, atol=1e-12)


def test_paper_kernel_definition():
    d = 1e-2
    r = np.array([0.0, 0.5e-2, 1e-2, 2e-2])
    assert np.allclose(kernels.kernel_of_r("paper", d, r), [1.0, 0.5, 1.0, 0.5])


@pytest.mark.parametrize("dim,depth,order,kind,param,shift", [
    (3, 3, 3, "imq", 0.005, 1.0),
    (2, 4, 4, "gauss", 0.3, 0.1),
    (3, 4, 3, "paper", 1e-2, 0.0),
])
def test_row_by_row_product_equals_nested_product(dim, depth, order, kind, param, shift):
    """Rows of A~ X taken one target at a time with direct moments and direct local evaluation at every
    level equal the nested product (child transfers up and down): nested Chebyshev interpolation is exact
    for the degree n-1 Lagrange polynomials, so the two differ by rounding only."""
    from oracle.h2 import h2_rows
    n = 1200 if dim == 3 else 900
    P = W.uniform_cube(n, dim, 31 + depth)
    X = W.normal_rhs(n, 2, 41 + depth)
    h = H2(Tree(P, depth), kind, param, shift, order)
    Y = h.matvec(X)
    rows = np.arange(0, n, 11)
    R = h2_rows(P, kind, param, shift, depth, order, X, rows)
    assert np.max(np.abs(R - Y[rows])) <= 1e-13 * np.max(np.abs(Y))


def test_row_by_row_product_reproduces_dense_for_quadratic_kernel():
    """Independent of the H2 code: with the radial quadratic kernel and order >= 3 every far-field block is
    interpolated exactly, so the row formula gives rows of the dense A X."""
    from oracle.h2 import h2_rows
    P = W.uniform_cube(800, 3, 51)
    X = W.normal_rhs(800, 3, 52)
    rows = [0, 1, 399, 798, 799]
    R = h2_rows(P, "poly2", 0.0, 0.5, 3, 3, X, rows)
    AX = kernels.dense("poly2", 0.0, 0.5, P) @ X
    assert np.max(np.abs(R - AX[rows])) <= 1e-12 * np.max(np.abs(AX))
