"""Parity of the HIP library (through the C ABI) with the FP64 oracle.

Sizes are small enough for the oracle to finish in seconds and still span
several tiles, colour classes and levels with ragged box sizes. The floating
point bar is the one the build targets: relative solve difference <= 1e-10
for the FP64 path (both sides use the same sigma_0 so the truncation
decisions are taken against the same tau; ranks must then agree box by box),
and GMRES relative residual <= 1e-10 for the FP32-factor path.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def gpu():
    from paper_1508_01835_amd import IFMM
    return IFMM


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


CASES = {
    # name: (workload factory)
    "uniform2d_2048": lambda: W.uniform2d_2048(),
    "uniform3d_3000_d3": lambda: W.small_uniform(3000, 3, 201, 3, 3, 1e-6, kparam=0.005, nrhs=2),
    "uniform2d_1500_d5": lambda: W.small_uniform(1500, 2, 203, 5, 3, 1e-7),
    "cluster3d_1600_d4": lambda: W.small_cluster(200, 205, 4, 3, 1e-8),
    "uniform3d_1200_o4": lambda: W.small_uniform(1200, 3, 207, 3, 4, 1e-9, kernel="gauss", kparam=0.3, shift=0.1),
}

_ORACLES = {}


def oracle(name):
    if name not in _ORACLES:
        from oracle.ifmm import IFMM as Oracle
        wl = CASES[name]()
        o = Oracle(wl.points, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps)
        o.factorize()
        _ORACLES[name] = (wl, o)
    return _ORACLES[name]


@pytest.mark.parametrize("name", list(CASES))
def test_matvec_matches_oracle(name):
    wl, o = oracle(name)
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps,
              sigma0=o.r2.sigma0)
    y = g.matvec(to_dev(wl.rhs)).cpu().numpy()
    yo = o.matvec(wl.rhs)
    assert rel(y, yo) <= 1e-13
    g.close()


@pytest.mark.parametrize("name", list(CASES))
def test_sigma0_estimate_matches_oracle(name):
    wl, o = oracle(name)
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps)
    s = g.stats()["sigma0"]
    g.close()
    assert abs(s - o.r2.sigma0) <= 1e-8 * o.r2.sigma0


@pytest.mark.parametrize("name", list(CASES))
def test_factor_solve_matches_oracle(name):
    wl, o = oracle(name)
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps,
              sigma0=o.r2.sigma0)
    g.factorize()
    for l, r in o.final_r.items():
        assert g.ranks(l) == list(r), "ranks differ at level %d" % l
    x = g.solve(to_dev(wl.rhs)).cpu().numpy()
    xo = o.solve(wl.rhs)
    assert rel(x, xo) <= 1e-10
    g.close()


def test_exact_limit_equals_dense_solve():
    from oracle.h2 import H2
    from oracle.tree import Tree
    wl = W.small_uniform(700, 2, 211, 4, 3, 0.0)
    tr = Tree(wl.points, 4)
    Ad = H2(tr, wl.kernel, wl.kparam, wl.shift, 3).dense()
    xd = np.linalg.solve(Ad, wl.rhs[:, 0])
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 4, 3, 0.0)
    g.factorize()
    x = g.solve(to_dev(wl.rhs[:, 0])).cpu().numpy()
    g.close()
    assert rel(x, xd) <= 1e-13 * np.linalg.cond(Ad)


def test_poly_kernel_reproduces_Ainv_b():
    from oracle import kernels
    pts = W.uniform_cube(500, 3, 213)
    A = kernels.dense("poly2", 0.0, 1.0, pts)
    b = W.normal_rhs(500, 1, 214)[:, 0]
    g = gpu()(to_dev(pts), "poly2", 0.0, 1.0, 3, 3, 0.0)
    g.factorize()
    x = g.solve(to_dev(b)).cpu().numpy()
    g.close()
    assert rel(x, np.linalg.solve(A, b)) <= 1e-12 * np.linalg.cond(A)


def test_many_rhs_equal_single_rhs_bitwise():
    wl = W.small_uniform(900, 3, 215, 3, 3, 1e-6, nrhs=5)
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6)
    g.factorize()
    X = g.solve(to_dev(wl.rhs)).cpu().numpy()
    for k in range(5):
        xk = g.solve(to_dev(wl.rhs[:, k])).cpu().numpy()
        assert np.array_equal(xk, X[:, k])
    g.close()


def test_refactorization_is_deterministic():
    wl = W.small_cluster(150, 217, 4, 3, 1e-7)
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-7)
    g.factorize()
    x1 = g.solve(to_dev(wl.rhs[:, 0])).cpu().numpy()
    g.factorize()
    x2 = g.solve(to_dev(wl.rhs[:, 0])).cpu().numpy()
    g.close()
    assert np.array_equal(x1, x2)


def test_gmres_fp64_preconditioner_matches_oracle_iterations():
    from oracle.gmres import gmres_right
    wl, o = oracle("uniform2d_1500_d5")
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, 1e-3,
              sigma0=o.r2.sigma0)
    g.factorize()
    x, it, rr = g.gmres(to_dev(wl.rhs[:, 0]), tol=1e-10, maxit=100)
    from oracle.ifmm import IFMM as Oracle
    o3 = Oracle(wl.points, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, 1e-3, sigma0=o.r2.sigma0)
    o3.factorize()
    xo, ito, rro, _ = gmres_right(o3.matvec, o3.solve, wl.rhs[:, 0], tol=1e-10, maxit=100)
    g.close()
    assert rr <= 1e-10 and rro <= 1e-10
    assert abs(it - ito) <= 1
    assert rel(x.cpu().numpy(), xo) <= 1e-8


def test_fp32_factors_precondition_fp64_gmres():
    wl = W.small_cluster(250, 219, 4, 3, 1e-5, nrhs=2)
    pts = to_dev(wl.points)
    op = gpu()(pts, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-5)
    pr = gpu()(pts, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-5, precision=32)
    pr.factorize()
    x, it, rr = op.gmres(to_dev(wl.rhs), tol=1e-10, maxit=200, prec=pr)
    assert rr <= 1e-10
    # the FP32 factorization alone is an approximate solve (error ~ cond * eps)
    x32 = pr.solve(to_dev(wl.rhs)).cpu().numpy()
    assert rel(x32, x.cpu().numpy()) <= 1e-2
    # FP32 and FP64 factorizations at the same eps keep the same ranks here
    f64 = gpu()(pts, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-5, sigma0=pr.stats()["sigma0"])
    f64.factorize()
    assert f64.stats()["max_rank"] == pr.stats()["max_rank"]
    f64.close()
    op.close()
    pr.close()


def test_error_paths():
    from paper_1508_01835_amd import IFMMError
    IFMM = gpu()
    wl = W.small_uniform(300, 2, 221, 3, 3, 1e-6)
    g = IFMM(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6)
    with pytest.raises(IFMMError) as e:
        g.solve(to_dev(wl.rhs[:, 0]))
    assert e.value.code == 5          # IFMM_ERR_STATE
    g.close()
    bad = wl.points.copy()
    bad[3, 0] = np.nan
    with pytest.raises(IFMMError) as e:
        IFMM(to_dev(bad), wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6)
    assert e.value.code == 1          # IFMM_ERR_ARG
    with pytest.raises(IFMMError) as e:
        IFMM(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6, hbm_budget_bytes=4096)
    assert e.value.code == 2          # IFMM_ERR_OOM (budget)
    with pytest.raises(IFMMError) as e:
        IFMM(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 1, 3, 1e-6)
    assert e.value.code == 1


def test_paper_kernel_gmres_with_and_without_preconditioner():
    """The paper's GMRES comparison (Sec. 3.2) at a size the oracle runs: the same H2 operator without a
    preconditioner and with the IFMM preconditioner (eps 1e-3). Iteration counts follow the oracle's runs
    of the same method; the preconditioned run needs far fewer."""
    from oracle.gmres import gmres_right
    from oracle.ifmm import IFMM as Oracle
    wl = W.paper_cube(n=2000, d=1e-2, order=3, depth=3, eps=1e-3, seed=6101)
    b = wl.rhs[:, 0]
    o = Oracle(wl.points, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps)
    o.factorize()
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps,
              sigma0=o.r2.sigma0)
    xn, itn, rrn = g.gmres(to_dev(b), tol=1e-10, maxit=500, precondition=False)   # before factorize
    xo_n, ito_n, rro_n, _ = gmres_right(o.matvec, lambda v: v, b, tol=1e-10, maxit=500)
    g.factorize()
    xp, itp, rrp = g.gmres(to_dev(b), tol=1e-10, maxit=500)
    xo_p, ito_p, rro_p, _ = gmres_right(o.matvec, o.solve, b, tol=1e-10, maxit=500)
    g.close()
    print("unpreconditioned", itn, ito_n, "preconditioned", itp, ito_p, flush=True)
    assert max(rrn, rrp, rro_n, rro_p) <= 1e-10
    assert abs(itn - ito_n) <= 1 and abs(itp - ito_p) <= 1
    assert itp * 3 <= itn
    assert rel(xn.cpu().numpy(), xo_n) <= 1e-8 and rel(xp.cpu().numpy(), xo_p) <= 1e-8


def test_paper_kernel_left_preconditioning_matches_oracle():
    """App. B: the IFMM as a left preconditioner on the paper's kernel (eps 1e-3). The iteration count,
    the solution and both residuals follow the oracle's run of the same method; with P = I the left
    variant is the unpreconditioned method itself."""
    from oracle.gmres import gmres_left
    from oracle.ifmm import IFMM as Oracle
    wl = W.paper_cube(n=2000, d=1e-2, order=3, depth=3, eps=1e-3, seed=6101)
    b = wl.rhs[:, 0]
    o = Oracle(wl.points, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps)
    o.factorize()
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps,
              sigma0=o.r2.sigma0)
    xi, iti, rpi, rti = g.gmres_left(to_dev(b), tol=1e-10, maxit=500, precondition=False)
    xr, itr, rrr = g.gmres(to_dev(b), tol=1e-10, maxit=500, precondition=False)
    g.factorize()
    xl, itl, rpl, rtl = g.gmres_left(to_dev(b), tol=1e-10, maxit=500)
    xo, ito, rpo, rto, _ = gmres_left(o.matvec, o.solve, b, tol=1e-10, maxit=500)
    g.close()
    print("left", itl, ito, rpl, rpo, rtl, rto, "identity", iti, itr, flush=True)
    assert iti == itr and rpi == rti == rrr and torch.equal(xi, xr)
    assert abs(itl - ito) <= 1
    assert max(rpl, rpo) <= 1.5e-10           # recomputed; the Arnoldi estimate stopped at 1e-10
    assert rtl <= 1e-8 and rto <= 1e-8
    assert rel(xl.cpu().numpy(), xo) <= 1e-8


def test_nonfinite_inputs_and_overlap_rejected():
    """IFMM_ERR_NUMERICAL for a NaN or infinity in b (solve and GMRES); IFMM_ERR_ARG when GMRES's x overlaps b."""
    import ctypes
    from paper_1508_01835_amd import IFMMError
    from paper_1508_01835_amd import ifmm as binding
    wl = W.small_uniform(400, 2, 223, 3, 3, 1e-6)
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6)
    g.factorize()
    for v in (np.nan, np.inf):
        b = wl.rhs[:, 0].copy()
        b[17] = v
        with pytest.raises(IFMMError) as e:
            g.solve(to_dev(b))
        assert e.value.code == 4      # IFMM_ERR_NUMERICAL
        with pytest.raises(IFMMError) as e:
            g.gmres(to_dev(b), tol=1e-10, maxit=20)
        assert e.value.code == 4
    # the handle still works after the rejected calls
    x = g.solve(to_dev(wl.rhs[:, 0])).cpu().numpy()
    assert np.all(np.isfinite(x))
    B = to_dev(np.concatenate([wl.rhs[:, 0], wl.rhs[:, 0]]))
    n = wl.n
    it, rr = ctypes.c_int(), ctypes.c_double()
    for xoff in (0, n // 2):
        rc = binding.lib().ifmm_gmres(g.h, g.h, ctypes.c_void_p(B.data_ptr()),
                                      ctypes.c_void_p(B.data_ptr() + 8 * xoff), 1, n, 1e-10, 20,
                                      ctypes.byref(it), ctypes.byref(rr))
        assert rc == 1                # IFMM_ERR_ARG: x overlaps b
    g.close()


def test_gmres_op_and_prec_on_different_streams():
    """op and prec on distinct streams give the same result as on one stream (the calls order the streams)."""
    wl = W.small_cluster(250, 225, 4, 3, 1e-5, nrhs=3)
    pts = to_dev(wl.points)
    b = to_dev(wl.rhs)
    IFMM = gpu()
    op = IFMM(pts, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-5)
    pr = IFMM(pts, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-5, precision=32)
    pr.factorize()
    x1, it1, rr1 = op.gmres(b, tol=1e-10, maxit=200, prec=pr)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    op2 = IFMM(pts, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-5, stream=sa)
    pr2 = IFMM(pts, wl.kernel, wl.kparam, wl.shift, 4, 3, 1e-5, precision=32, stream=sb)
    pr2.factorize()
    x2, it2, rr2 = op2.gmres(b, tol=1e-10, maxit=200, prec=pr2)
    sa.synchronize()
    assert rr1 <= 1e-10 and it1 == it2 and rr1 == rr2
    assert torch.equal(x1, x2)
    for h in (op, pr, op2, pr2):
        h.close()


def test_solve_graph_replays_equal_eager_launches(monkeypatch):
    """The substitution replayed as a HIP graph gives bitwise the result of launching its kernels one by one,
    on every replay, with other device work and synchronisations between the replays, for several
    right-hand-side counts (one graph each)."""
    wl = W.small_uniform(1500, 3, 227, 3, 3, 1e-6, kparam=0.005, nrhs=4)
    g = gpu()(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6)
    g.factorize()
    monkeypatch.setenv("IFMM_SOLVE_GRAPH", "0")
    ref = {k: g.solve(to_dev(wl.rhs[:, :k])).cpu() for k in (1, 2, 4)}
    monkeypatch.delenv("IFMM_SOLVE_GRAPH")
    for rep in range(4):
        for k in (1, 2, 4):
            x = g.solve(to_dev(wl.rhs[:, :k])).cpu()
            assert torch.equal(x, ref[k]), (rep, k)
            y = g.matvec(to_dev(wl.rhs[:, :k]))      # other work between replays
            torch.cuda.synchronize()
            assert torch.isfinite(y).all()
    g.close()
