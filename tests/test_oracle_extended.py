"""Pins of the oracle's extended sparse system E and of sigma_0.

Paper: Sec. 2.1, eq. (Ax=b_extended): solving E [x; 0] = [b; 0] gives the
solution of A x = b; E is symmetric for symmetric A thanks to the ordering
of the equations. Sec. 2.4: sigma_0(E) is the largest singular value of E.
"""
import numpy as np
import pytest

import workloads as W
from oracle.extended import R2
from oracle.h2 import H2
from oracle.tree import Tree


def build(n, dim, depth, order, eps, kernel="imq", kp=0.02, shift=1.0, seed=41, sigma0=None):
    pts = W.uniform_cube(n, dim, seed)
    tr = Tree(pts, depth)
    h = H2(tr, kernel, kp, shift, order)
    return pts, tr, h, R2(h, eps, sigma0=sigma0)


@pytest.mark.parametrize("dim,depth,order", [(2, 3, 3), (3, 2, 2), (2, 4, 2)])
def test_extended_solve_reproduces_Atilde(dim, depth, order):
    pts, tr, h, r2 = build(300, dim, depth, order, 1e-15)
    # bases are still complete at this tolerance, so E represents A~ exactly
    E = r2.dense_E()
    b = W.normal_rhs(300, 1, 5)[:, 0]
    rhs = np.zeros(E.shape[0])
    rhs[:300] = b[tr.perm]
    xt = np.linalg.solve(E, rhs)[:300]
    x = np.empty(300)
    x[tr.perm] = xt
    xd = np.linalg.solve(h.dense(), b)
    assert np.linalg.norm(x - xd) <= 1e-12 * np.linalg.norm(xd)


def test_E_symmetric_for_symmetric_kernel():
    _, _, _, r2 = build(250, 2, 3, 3, 1e-15)
    E = r2.dense_E()
    assert np.linalg.norm(E - E.T) <= 1e-13 * np.linalg.norm(E)


def test_bases_orthonormal_and_transfers_nested():
    pts = W.uniform_cube(400, 3, 43)
    tr = Tree(pts, 3)
    h = H2(tr, "imq", 0.02, 1.0, 3)
    r2 = R2(h, 1e-15, sigma0=1.0, weights=False)
    r2.r_pre = r2.r
    for i, U in r2.U.items():
        assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-12)
    # the effective basis of a level-2 box on its points, blockdiag(U_c) stack(PU_c), is orthonormal
    L = tr.L
    assert L == 3
    lev2 = tr.levels[2]
    for p in range(lev2.nb):
        cs = lev2.children[p]
        rows = sum(r2.U[c].shape[0] for c in cs)
        Ueff = np.zeros((rows, r2.r_pre[2][p]))
        o = 0
        for c in cs:
            Ueff[o:o + r2.U[c].shape[0]] = r2.U[c] @ r2.PU[L][c]
            o += r2.U[c].shape[0]
        assert np.allclose(Ueff.T @ Ueff, np.eye(Ueff.shape[1]), atol=1e-11)


@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_sigma0_matches_dense_svd(kind):
    # brute force: largest singular value of the dense E (unrotated operators); the clustered cloud has
    # several nearly equal top singular values (one per cluster), where a power iteration stalls
    if kind == "uniform":
        pts = W.uniform_cube(200, 2, 47)
        h = H2(Tree(pts, 3), "imq", 0.02, 1.0, 2)
    else:
        pts = W.clustered(8, 40, 0.05, 49, 50)
        h = H2(Tree(pts, 3), "gauss", 0.1, 0.1, 2)
    r2 = R2(h, 1e-15, weights=False)
    sig = np.linalg.norm(r2.dense_E(), 2)
    assert abs(r2.sigma0 - sig) <= 1e-10 * sig
    assert r2.sigma0 >= 1.0
    assert r2.sigma0_steps < 300


def test_truncation_rank_rule_strict():
    # tau scales with eps; a larger eps can only keep fewer directions
    _, _, _, a = build(400, 2, 3, 4, 1e-2, seed=45)
    _, _, _, b = build(400, 2, 3, 4, 1e-8, seed=45, sigma0=a.sigma0)
    for l in a.k_init:
        assert all(x <= y for x, y in zip(a.k_init[l], b.k_init[l]))
    assert sum(map(sum, a.k_init.values())) < sum(map(sum, b.k_init.values()))


def _box_points(tr, l, i):
    """Tree-order indices of the points in box i of level l (leaf coordinates shifted to level l)."""
    levL = tr.levels[tr.L]
    shift = tr.L - l
    box = tr.levels[l].coords[i]
    idx = []
    for j in range(levL.nb):
        if np.all((levL.coords[j] >> shift) == box):
            s = tr.leaf_points(j)
            idx.extend(range(s.start, s.stop))
    return np.array(idx, dtype=np.int64)


@pytest.mark.parametrize("dim,n,depth,order,kernel,kp", [(2, 600, 4, 3, "imq", 0.02), (3, 600, 3, 3, "gauss", 0.3)])
def test_weights_are_far_field_singular_values(dim, n, depth, order, kernel, kp):
    """Sec. 2.2 footnote on initial weights: the weights of a box are the singular values of the block row
    of U K V^T over its far field. Pinned against the dense A~ itself: for every box i of every level, the
    kept weights Sigma_U equal the leading singular values of A~(points of i, points outside N(i)), and
    Sigma_V those of A~(points outside N(i), points of i)^T. The far field outside N(i) holds the interaction
    list and every ancestor's far field, so weights built from the level's interaction list alone fail."""
    pts = W.uniform_cube(n, dim, 51)
    tr = Tree(pts, depth)
    h = H2(tr, kernel, kp, 1.0, order)
    r2 = R2(h, 1e-9)
    Ad = h.dense()
    A = Ad[np.ix_(tr.perm, tr.perm)]             # tree order
    for l in range(2, depth + 1):
        lev = tr.levels[l]
        for i in range(lev.nb):
            rows = _box_points(tr, l, i)
            near = np.concatenate([_box_points(tr, l, j) for j in lev.nbrs[i]])
            far = np.setdiff1d(np.arange(tr.n), near)
            k = r2.k_init[l][i]
            for side, M in (("U", A[np.ix_(rows, far)]), ("V", A[np.ix_(far, rows)].T)):
                s = np.linalg.svd(M, compute_uv=False) if M.size else np.zeros(0)
                want = np.zeros(k)
                want[:min(k, s.shape[0])] = s[:k]
                got = (r2.SU if side == "U" else r2.SV)[l][i]
                assert np.allclose(got, want, rtol=0, atol=1e-12 * r2.sigma0), (l, i, side)
                # every dropped direction is at or below tau
                if s.shape[0] > k:
                    assert s[k] <= r2.tau * (1 + 1e-10), (l, i, side)
