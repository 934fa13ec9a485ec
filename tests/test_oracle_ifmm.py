"""Pins of the oracle's elimination, compression, merge and solve.

E3  exact limit: with eps -> 0 (tau = 64 u sigma_0) every compression is
    lossless, so the IFMM solve equals the dense solve of A~ (and of A for a
    kernel the interpolation reproduces exactly) - Sec. 1 and 5: the accuracy
    is controllable down to machine precision.
E6  error decreases monotonically as eps decreases (Sec. 3.1 trend).
E10 boxes of one colour class commute (independent sets): any order inside a
    class gives the same solution.
Planted mistakes (a dropped redirect term, a missing basis rotation) must make
E3 fail, which shows the pin sees them.
"""
import numpy as np
import pytest

import workloads as W
from oracle import kernels
from oracle.ifmm import IFMM


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


CASES = [(400, 2, 3, 3), (512, 2, 4, 2), (500, 3, 2, 2), (700, 3, 3, 2)]


@pytest.mark.parametrize("n,dim,depth,order", CASES)
def test_exact_limit_matches_dense_solve(n, dim, depth, order):
    wl = W.small_uniform(n, dim, 100 + n, depth, order, 0.0)
    f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, depth, order, 0.0)
    f.factorize()
    Ad = f.h2.dense()
    b = wl.rhs[:, 0]
    xd = np.linalg.solve(Ad, b)
    x = f.solve(b)
    kappa = np.linalg.cond(Ad)
    assert rel(x, xd) <= 1e-13 * kappa


def test_exact_limit_reproduces_Ainv_b_for_poly_kernel():
    pts = W.uniform_cube(300, 2, 61)
    A = kernels.dense("poly2", 0.0, 1.0, pts)
    f = IFMM(pts, "poly2", 0.0, 1.0, 3, 3, 0.0)
    f.factorize()
    b = W.normal_rhs(300, 2, 62)
    x = f.solve(b)
    xd = np.linalg.solve(A, b)
    assert rel(x, xd) <= 1e-13 * np.linalg.cond(A)


def test_error_monotone_in_eps():
    wl = W.small_uniform(1024, 2, 71, 4, 4, 1e-8)
    base = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 4, 4, 1e-8)
    xd = np.linalg.solve(base.h2.dense(), wl.rhs[:, 0])
    errs = []
    for eps in (1e-2, 1e-4, 1e-6, 1e-8, 1e-10):
        f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 4, 4, eps, sigma0=base.r2.sigma0)
        f.factorize()
        errs.append(rel(f.solve(wl.rhs[:, 0]), xd))
    assert all(errs[k + 1] < errs[k] for k in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-7


def test_colour_class_order_irrelevant():
    wl = W.small_uniform(800, 3, 73, 3, 2, 1e-6)
    a = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 3, 2, 1e-6)
    b = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 3, 2, 1e-6, sigma0=a.r2.sigma0,
             class_shuffle_seed=5)
    a.factorize()
    b.factorize()
    assert a.final_r == b.final_r
    assert rel(b.solve(wl.rhs[:, 0]), a.solve(wl.rhs[:, 0])) <= 1e-12


def test_many_rhs_equals_single():
    wl = W.small_uniform(400, 2, 75, 3, 3, 1e-6, nrhs=4)
    f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6)
    f.factorize()
    X = f.solve(wl.rhs)
    for k in range(4):
        assert np.allclose(f.solve(wl.rhs[:, k]), X[:, k], rtol=0, atol=1e-13 * np.abs(X).max())


def test_ranks_never_exceed_box_size():
    wl = W.small_cluster(60, 81, 4, 3, 1e-8)
    f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-8)
    f.factorize()
    L = f.tree.L
    for i, r in enumerate(f.final_r[L]):
        s = f.tree.leaf_points(i)
        assert r <= s.stop - s.start


def _planted(monkeypatch, what):
    import oracle.ifmm as mod
    if what == "no_redirect":
        monkeypatch.setattr(mod.IFMM, "_redirect_add", lambda self, st, a, c, B: None)
    elif what == "no_rotation":
        def nop(self, st, new_basis):
            for j, (Uh, sU, Vh, sV) in new_basis.items():
                st.U[j], st.V[j] = Uh, Vh
                st.r[j] = Uh.shape[1]
        monkeypatch.setattr(mod.IFMM, "_apply_basis_change", nop)
    elif what == "wrong_sign_fill":
        orig = mod.LevelState.setk
        monkeypatch.setattr(mod.IFMM, "_redirect_add",
                            lambda self, st, a, c, B: orig(st, a, c, st.k(a, c) - B))


@pytest.mark.parametrize("what", ["no_redirect", "no_rotation", "wrong_sign_fill"])
def test_planted_mistakes_break_exact_limit(monkeypatch, what):
    _planted(monkeypatch, what)
    wl = W.small_uniform(400, 2, 91, 3, 3, 0.0)
    f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 3, 3, 0.0)
    try:
        f.factorize()
        x = f.solve(wl.rhs[:, 0])
    except Exception:
        return                      # a crash also counts as detected
    xd = np.linalg.solve(f.h2.dense(), wl.rhs[:, 0])
    assert rel(x, xd) > 1e-6


def test_preconditioned_gmres_iterations_grow_with_eps():
    from oracle.gmres import gmres_right
    wl = W.small_uniform(600, 2, 93, 4, 3, 1e-8)
    its = []
    s0 = None
    for eps in (0.0, 1e-6, 1e-2):
        f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 4, 3, eps, sigma0=s0)
        s0 = f.r2.sigma0
        f.factorize()
        x, it, res, _ = gmres_right(f.matvec, f.solve, wl.rhs[:, 0], tol=1e-10, maxit=100)
        assert res <= 1e-10
        its.append(it)
    assert its[0] == 1
    assert its[0] <= its[1] <= its[2] and its[2] > its[0]


def test_left_preconditioned_gmres_iterations_grow_with_eps():
    """App. B with the oracle's own factorization: at eps = 0 the factorization is the exact inverse of the
    H2 operator, so left-preconditioned GMRES takes one step; coarser eps needs more, and the reported
    (preconditioned) residual and the true residual both end small."""
    from oracle.gmres import gmres_left
    wl = W.small_uniform(600, 2, 93, 4, 3, 1e-8)
    its = []
    s0 = None
    for eps in (0.0, 1e-6, 1e-2):
        f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 4, 3, eps, sigma0=s0)
        s0 = f.r2.sigma0
        f.factorize()
        x, it, rp, rt, _ = gmres_left(f.matvec, f.solve, wl.rhs[:, 0], tol=1e-10, maxit=100)
        assert rp <= 2e-10 and rt <= 1e-8
        its.append(it)
    assert its[0] == 1
    assert its[0] <= its[1] <= its[2] and its[2] > its[0]


@pytest.mark.parametrize("n,dim,depth,order", [(400, 2, 3, 3), (500, 3, 2, 2)])
def test_literal_mode_exact_limit(n, dim, depth, order):
    """The paper's own pairwise route (Alg. 2 and 3: truncated SVD of each well-separated fill, then
    recompression of [U Sigma | U' S'] and the redirect) is exact at eps -> 0, like the aggregated one."""
    wl = W.small_uniform(n, dim, 100 + n, depth, order, 0.0)
    f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, depth, order, 0.0, mode="literal")
    f.factorize()
    Ad = f.h2.dense()
    b = wl.rhs[:, 0]
    assert rel(f.solve(b), np.linalg.solve(Ad, b)) <= 1e-13 * np.linalg.cond(Ad)


def test_literal_and_aggregated_modes_agree_to_order_eps():
    """Aggregated recompression (one recompression per affected box and elimination) against the paper's
    pairwise route on the same sigma_0: both solutions are within a small multiple of eps of the dense
    solve of A~ and of each other, and their difference shrinks with eps."""
    wl = W.small_uniform(600, 2, 301, 4, 3, 1e-6)
    b = wl.rhs[:, 0]
    base = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-6)
    xd = np.linalg.solve(base.h2.dense(), b)
    diffs = []
    for eps in (1e-4, 1e-6, 1e-8):
        xs = {}
        for mode in ("aggregated", "literal"):
            f = IFMM(wl.points, wl.kernel, wl.kparam, wl.shift, 4, 3, eps, sigma0=base.r2.sigma0, mode=mode)
            f.factorize()
            xs[mode] = f.solve(b)
        ea, el = rel(xs["aggregated"], xd), rel(xs["literal"], xd)
        d = rel(xs["literal"], xs["aggregated"])
        assert ea <= 10 * eps and el <= 10 * eps, (eps, ea, el)
        assert d <= 10 * eps, (eps, d)
        diffs.append(d)
    assert diffs[0] > diffs[1] > diffs[2]
