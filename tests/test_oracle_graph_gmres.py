"""Pins of the generic block elimination (worked examples of the paper) and of GMRES.

Sec. 2.1, graph example: eliminating x_1 from the 3x3 block system leaves
edges A_ab - A_a1 A_11^-1 A_1b and right-hand sides b_a - A_a1 A_11^-1 b_1.
App. C: on E = [[A00, ., U0, .], [., A11, ., U1], [V0^T, ., ., -I],
[., V1^T, -I, .]] eliminating A00 and A11 first leaves
[[-V0^T A00^-1 U0, -I], [-I, -V1^T A11^-1 U1]]; eliminating A00, then the
two auxiliary blocks, leaves A11 - U1 V0^T A00^-1 U0 V1^T (block LU order).
Sec. 3.2: right-preconditioned GMRES; with the exact inverse as
preconditioner it converges in one iteration.
"""
import numpy as np
import pytest

from oracle.graph import BlockGraph
from oracle.gmres import gmres_right


def rnd(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)


def test_three_by_three_graph_example():
    s = {1: 3, 2: 2, 3: 4}
    A = {(a, c): rnd((s[a], s[c]), 10 * a + c) for a in s for c in s}
    A[(1, 1)] += 5 * np.eye(3)
    g = BlockGraph(s)
    for k, B in A.items():
        g.set(*k, B)
    b = {k: rnd(v, 100 + k) for k, v in s.items()}
    g.b = {k: v.copy() for k, v in b.items()}
    g.eliminate(1)
    inv = np.linalg.inv(A[(1, 1)])
    for a in (2, 3):
        for c in (2, 3):
            assert np.allclose(g.E[(a, c)], A[(a, c)] - A[(a, 1)] @ inv @ A[(1, c)], atol=1e-13)
        assert np.allclose(g.b[a], b[a] - A[(a, 1)] @ inv @ b[1], atol=1e-13)


def _two_block():
    n0, n1, r = 5, 4, 2
    A00 = rnd((n0, n0), 1) + 6 * np.eye(n0)
    A11 = rnd((n1, n1), 2) + 6 * np.eye(n1)
    U0, U1 = rnd((n0, r), 3), rnd((n1, r), 4)
    V0, V1 = rnd((n0, r), 5), rnd((n1, r), 6)
    g = BlockGraph({"x0": n0, "x1": n1, "a": r, "b": r})
    g.set("x0", "x0", A00); g.set("x0", "a", U0)
    g.set("x1", "x1", A11); g.set("x1", "b", U1)
    # row of vertex a: V0^T x0 - b = 0; row of vertex b: V1^T x1 - a = 0 (App. C's E)
    g.set("a", "x0", V0.T); g.set("a", "b", -np.eye(r))
    g.set("b", "x1", V1.T); g.set("b", "a", -np.eye(r))
    return g, (A00, A11, U0, U1, V0, V1)


def test_appendix_c_level_by_level_form():
    g, (A00, A11, U0, U1, V0, V1) = _two_block()
    g.eliminate("x0")
    g.eliminate("x1")
    M = g.dense(["a", "b"])
    r = U0.shape[1]
    expect = np.block([[-V0.T @ np.linalg.solve(A00, U0), -np.eye(r)],
                       [-np.eye(r), -V1.T @ np.linalg.solve(A11, U1)]])
    assert np.allclose(M, expect, atol=1e-12)


def test_appendix_c_block_lu_form():
    g, (A00, A11, U0, U1, V0, V1) = _two_block()
    g.eliminate("x0")
    g.eliminate("a")
    g.eliminate("b")
    S = g.E[("x1", "x1")]
    assert np.allclose(S, A11 - U1 @ V0.T @ np.linalg.solve(A00, U0) @ V1.T, atol=1e-12)


def test_gmres_unpreconditioned_and_exact_preconditioner():
    n = 60
    A = rnd((n, n), 7) + 12 * np.eye(n)
    b = rnd(n, 8)
    x, it, res, _ = gmres_right(lambda v: A @ v, lambda v: v, b, tol=1e-12, maxit=n)
    assert res <= 1e-11
    assert np.allclose(x, np.linalg.solve(A, b), atol=1e-9)
    Ainv = np.linalg.inv(A)
    x1, it1, res1, _ = gmres_right(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-12, maxit=10)
    assert it1 == 1 and res1 <= 1e-12


def test_gmres_iterations_drop_with_better_preconditioner():
    n = 200
    rng = np.random.default_rng(9)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + np.diag(np.linspace(1, 50, n))
    b = rng.standard_normal(n)
    _, it0, r0, _ = gmres_right(lambda v: A @ v, lambda v: v, b, tol=1e-10, maxit=200)
    D = np.diag(A)
    _, it1, r1, _ = gmres_right(lambda v: A @ v, lambda v: v / D, b, tol=1e-10, maxit=200)
    assert r0 <= 1e-10 and r1 <= 1e-10 and it1 < it0


def _krylov_min(apply_op, r0, k, residual):
    """Brute force: the x in span{r0, Op r0, ..., Op^(k-1) r0} (orthonormalised) that minimises
    ||residual(x)||, by dense least squares."""
    K = np.zeros((r0.shape[0], k))
    v = r0.copy()
    for j in range(k):
        K[:, j] = v / np.linalg.norm(v)
        v = apply_op(K[:, j])
    Q, _ = np.linalg.qr(K)
    # residual is affine in x: residual(Q c) = residual(0) - R c with R[:, j] = residual(0) - residual(Q e_j)
    r_0 = residual(np.zeros(r0.shape[0]))
    R = np.stack([r_0 - residual(Q[:, j]) for j in range(k)], axis=1)
    c = np.linalg.lstsq(R, r_0, rcond=None)[0]
    return Q @ c


def _system(n=40, seed=21):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 3 * np.eye(n)
    d = np.linspace(1.0, 10.0, n)
    b = rng.standard_normal(n)
    return A, d, b


def test_gmres_iterates_minimise_over_the_krylov_space():
    """The k-th iterate of each variant is the minimiser GMRES is defined by (Sec. 3.2 and App. B):
    right: x = P^-1 y, y in K_k(A P^-1, b), minimising ||b - A x||; left: x in K_k(P^-1 A, P^-1 b),
    minimising ||P^-1 (b - A x)||. Checked against dense least squares on the Krylov basis."""
    from oracle.gmres import gmres_left
    A, d, b = _system()
    Pinv = lambda v: v / d
    for k in range(1, 6):
        xr, itr, _, _ = gmres_right(lambda v: A @ v, Pinv, b, tol=1e-300, maxit=k)
        y = _krylov_min(lambda v: A @ Pinv(v), b, k, lambda y: b - A @ Pinv(y))
        assert itr == k
        assert np.linalg.norm(xr - Pinv(y)) <= 1e-10 * np.linalg.norm(xr)
        xl, itl, _, _, _ = gmres_left(lambda v: A @ v, Pinv, b, tol=1e-300, maxit=k)
        xb = _krylov_min(lambda v: Pinv(A @ v), Pinv(b), k, lambda x: Pinv(b - A @ x))
        assert itl == k
        assert np.linalg.norm(xl - xb) <= 1e-10 * np.linalg.norm(xl)
    # the two variants minimise different norms over different spaces: after 3 steps they differ
    assert np.linalg.norm(xr - xl) > 1e-6 * np.linalg.norm(xr)


def test_left_gmres_special_preconditioners():
    """P = I: left and right GMRES are the same method; P^-1 = A^-1: one step solves the system."""
    from oracle.gmres import gmres_left
    A, d, b = _system(30, 22)
    xr, itr, rr, _ = gmres_right(lambda v: A @ v, lambda v: v, b, tol=1e-12, maxit=30)
    xl, itl, rp, rt, _ = gmres_left(lambda v: A @ v, lambda v: v, b, tol=1e-12, maxit=30)
    assert itl == itr and np.array_equal(xl, xr) and rp == rt == rr
    Ainv = np.linalg.inv(A)
    x1, it1, rp1, rt1, _ = gmres_left(lambda v: A @ v, lambda v: Ainv @ v, b, tol=1e-12, maxit=10)
    assert it1 == 1 and rp1 <= 1e-12 and rt1 <= 1e-11
    assert np.allclose(x1, np.linalg.solve(A, b), atol=1e-12)


def test_left_gmres_monitors_the_preconditioned_residual():
    """App. B: for left preconditioning the reported residual is ||P^-1 (b - A x)|| / ||P^-1 b||; with a
    badly scaled P the true residual can stay far above the tolerance."""
    from oracle.gmres import gmres_left
    rng = np.random.default_rng(23)
    n = 50
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 2 * np.eye(n)
    s = 10.0 ** rng.uniform(-4, 4, n)
    b = rng.standard_normal(n)
    Pinv = lambda v: s * v
    x, it, rp, rt, hist = gmres_left(lambda v: A @ v, Pinv, b, tol=1e-8, maxit=n)
    r = b - A @ x
    assert rp == pytest.approx(np.linalg.norm(s * r) / np.linalg.norm(s * b), rel=1e-12)
    assert rt == pytest.approx(np.linalg.norm(r) / np.linalg.norm(b), rel=1e-12)
    assert rp <= 1e-7 and hist[-1] <= 1e-8
    assert rt > 1e-4                  # the true residual is not what the left variant drives down
