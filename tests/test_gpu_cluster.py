"""Scaled-down version of the 3D clustered workload (8 Gaussian clusters, sigma 0.05, Gaussian kernel
exp(-r^2/0.1^2) + 0.1 I, Chebyshev order 4) against the oracle.

* FP64 factors at eps 1e-10 (the accuracy of the plain FP64 path): ranks box by box, solve <= 1e-10.
  Box sizes reach a few hundred unknowns at the top levels, ranks above 32 (the redirect by batched
  products) and boxes whose bases grow past their first capacity.
* The same with IFMM_FORCE_STREAMED: the variants meant for large blocks (LU panels streamed from memory,
  block-Jacobi SVD, one-workgroup pivoted QR, redirect by batched products) on every size, checked against
  the oracle in the same way.
* FP32 factors at eps 1e-5 precondition FP64 GMRES to 1e-10; the error of the FP32 solve and of the GMRES
  solution against the oracle's FP64 results is printed and bounded.
"""
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

_CACHE = {}


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def case(eps):
    if eps not in _CACHE:
        from oracle.ifmm import IFMM as Oracle
        wl = W.cluster3d(256, 4, eps)      # 2048 points, depth 4
        o = Oracle(wl.points, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, eps)
        o.factorize()
        _CACHE[eps] = (wl, o)
    return _CACHE[eps]


@pytest.mark.parametrize("forced", [False, True])
def test_clustered_fp64_eps1e10_matches_oracle(forced, monkeypatch):
    from paper_1508_01835_amd import IFMM
    wl, o = case(1e-10)
    monkeypatch.setenv("IFMM_KTIMING", "1")
    if forced:
        monkeypatch.setenv("IFMM_FORCE_STREAMED", "1")
    else:
        monkeypatch.delenv("IFMM_FORCE_STREAMED", raising=False)
    print("clustered 2048 points, order 4, eps 1e-10, forced=%s" % forced, flush=True)
    g = IFMM(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, 1e-10, sigma0=o.r2.sigma0)
    g.factorize()
    for l, r in o.final_r.items():
        assert g.ranks(l) == list(r), "ranks differ at level %d" % l
    x = g.solve(to_dev(wl.rhs[:, 0])).cpu().numpy()
    xo = o.solve(wl.rhs[:, 0])
    st = g.stats()
    fam = dict(zip(["schur_gemm", "pivot_lu", "trsm_w", "qr", "jacobi_svd", "edge_update", "solve", "matvec", "other",
                    "svd_round", "qr_panel", "qrcp", "svd_small", "row_xform", "col_xform", "qrcp_step"],
                   st["kfam_launches"]))
    print("max ranks", st["max_rank"], "solve diff %.2e" % rel(x, xo), "launches", fam, flush=True)
    g.close()
    assert max(max(r) for r in o.final_r.values()) > 32
    assert rel(x, xo) <= 1e-10
    if forced:
        assert fam["svd_round"] > 0 and fam["qrcp"] > 0 and fam["svd_small"] == 0 and fam["qrcp_step"] == 0


def test_clustered_fp32_factors_error_against_fp64_oracle():
    from paper_1508_01835_amd import IFMM
    wl, o = case(1e-5)
    b = wl.rhs[:, 0]
    pts = to_dev(wl.points)
    op = IFMM(pts, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, 1e-10, sigma0=o.r2.sigma0)
    pr = IFMM(pts, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, 1e-5, precision=32, sigma0=o.r2.sigma0)
    pr.factorize()
    x32 = pr.solve(to_dev(b)).cpu().numpy()
    xo = o.solve(b)                                   # the oracle's FP64 factorization at the same eps
    xg, it, rr = op.gmres(to_dev(b), tol=1e-10, maxit=200, prec=pr)
    xd = np.linalg.solve(o.h2.dense(), b)             # A~^-1 b
    e_solve, e_gmres = rel(x32, xo), rel(xg.cpu().numpy(), xd)
    print("fp32 factors eps 1e-5: solve vs fp64 oracle %.2e; GMRES %d it, relres %.2e, error vs A~^-1 b %.2e"
          % (e_solve, it, rr, e_gmres), flush=True)
    op.close()
    pr.close()
    assert rr <= 1e-10
    assert e_gmres <= 1e-8
    assert e_solve <= 1e-2
