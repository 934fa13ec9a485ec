"""Edge cases of the HIP path against the oracle, through the C ABI.

Degenerate point clouds the method has to handle:
  * a single point, and three points in a depth-2 octree (almost every box empty);
  * every point doubled (coincident pairs; the diagonal shift keeps A nonsingular);
  * points on a line and on a plane inside a 3D octree (most boxes empty, ragged occupancy).
The bar is that of the other parity cases: identical ranks box by box and the solution within 1e-10 of the
oracle's (both sides use the oracle's sigma_0).

Then the layout rules of the boundary: a leading dimension ld > n for solve, matvec and GMRES (results
bitwise equal to ld = n, padding rows untouched), a solve in place (x aliasing b), and the argument errors.
"""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a))


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def _line(n):
    return np.stack([np.linspace(0.0, 1.0, n), np.full(n, 0.5), np.full(n, 0.25)], axis=1)


DEGENERATE = {
    "single_point": (lambda: np.array([[0.3, 0.4, 0.5]]), 2),
    "three_points_depth2": (lambda: W.uniform_cube(3, 3, 9), 2),
    "coincident_pairs": (lambda: np.repeat(W.uniform_cube(200, 3, 10), 2, axis=0), 3),
    "line_in_octree": (lambda: _line(700), 4),
    "plane_in_octree": (lambda: np.concatenate([W.uniform_cube(900, 2, 11), np.zeros((900, 1))], axis=1), 4),
}


@pytest.mark.parametrize("name", list(DEGENERATE))
def test_degenerate_point_clouds_match_oracle(name):
    from oracle.ifmm import IFMM as Oracle
    from paper_1508_01835_amd import IFMM
    mk, depth = DEGENERATE[name]
    P = mk()
    n = P.shape[0]
    b = W.normal_rhs(n, 2, 77)
    print("case", name, "n", n, "depth", depth, flush=True)
    o = Oracle(P, "imq", 0.01, 1.0, depth, 3, 1e-8)
    o.factorize()
    g = IFMM(to_dev(P), "imq", 0.01, 1.0, depth, 3, 1e-8, sigma0=o.r2.sigma0)
    y = g.matvec(to_dev(b)).cpu().numpy()
    assert rel(y, o.matvec(b)) <= 1e-13
    g.factorize()
    for l, r in o.final_r.items():
        assert g.ranks(l) == list(r), "ranks differ at level %d" % l
    x = g.solve(to_dev(b)).cpu().numpy()
    g.close()
    assert rel(x, o.solve(b)) <= 1e-10


@pytest.fixture(scope="module")
def handle():
    from paper_1508_01835_amd import IFMM
    wl = W.small_uniform(700, 3, 219, 3, 3, 1e-6, nrhs=3)
    g = IFMM(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6)
    g.factorize()
    yield wl, g
    g.close()


def _padded(rhs, ld, fill):
    """Column-major n x k block with leading dimension ld: a (k, ld) buffer, rows n..ld-1 set to fill."""
    n, k = rhs.shape
    B = torch.full((k, ld), fill, dtype=torch.float64, device="cuda")
    B[:, :n] = to_dev(rhs.T)
    return B


def test_leading_dimension_larger_than_n(handle):
    from paper_1508_01835_amd.ifmm import lib
    wl, g = handle
    n, k = wl.rhs.shape
    ld = n + 37
    B = _padded(wl.rhs, ld, 7.0)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    torch.cuda.synchronize()
    # solve
    X = torch.full((k, ld), -3.0, dtype=torch.float64, device="cuda")
    assert lib().ifmm_solve(g.h, p(B), p(X), k, ld) == 0
    ref = g.solve(to_dev(wl.rhs))
    assert torch.equal(X[:, :n].t(), ref) and bool(torch.all(X[:, n:] == -3.0))
    # matvec
    Y = torch.full((k, ld), -3.0, dtype=torch.float64, device="cuda")
    assert lib().ifmm_matvec(g.h, p(B), p(Y), k, ld) == 0
    assert torch.equal(Y[:, :n].t(), g.matvec(to_dev(wl.rhs))) and bool(torch.all(Y[:, n:] == -3.0))
    # GMRES
    Z = torch.full((k, ld), -3.0, dtype=torch.float64, device="cuda")
    it = ctypes.c_int()
    rr = ctypes.c_double()
    assert lib().ifmm_gmres(g.h, g.h, p(B), p(Z), k, ld, 1e-10, 50, ctypes.byref(it), ctypes.byref(rr)) == 0
    Zr, itr, rrr = g.gmres(to_dev(wl.rhs), tol=1e-10, maxit=50)
    assert it.value == itr and rr.value == rrr
    assert torch.equal(Z[:, :n].t(), Zr) and bool(torch.all(Z[:, n:] == -3.0))
    assert bool(torch.all(B[:, n:] == 7.0))             # inputs untouched


def test_solve_in_place(handle):
    from paper_1508_01835_amd.ifmm import lib
    wl, g = handle
    n, k = wl.rhs.shape
    X = to_dev(wl.rhs.T)                                  # (k, n) = column-major n x k
    torch.cuda.synchronize()
    assert lib().ifmm_solve(g.h, ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(X.data_ptr()), k, n) == 0
    assert torch.equal(X.t(), g.solve(to_dev(wl.rhs)))


def test_argument_errors_of_the_products(handle):
    from paper_1508_01835_amd.ifmm import lib
    wl, g = handle
    n, k = wl.rhs.shape
    B = to_dev(wl.rhs.T)
    Y = torch.empty_like(B)
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    it = ctypes.c_int()
    rr = ctypes.c_double()
    assert lib().ifmm_solve(g.h, p(B), p(Y), 0, n) == 1                     # nrhs < 1
    assert lib().ifmm_solve(g.h, p(B), p(Y), k, n - 1) == 1                 # ld < n
    assert lib().ifmm_matvec(g.h, p(B), p(B), k, n) == 1                    # aliasing not allowed
    assert lib().ifmm_gmres(g.h, g.h, p(B), p(Y), k, n, 0.0, 10, ctypes.byref(it), ctypes.byref(rr)) == 1
    assert lib().ifmm_gmres(g.h, g.h, p(B), p(Y), k, n, 1e-10, 1001, ctypes.byref(it), ctypes.byref(rr)) == 1
    assert lib().ifmm_gmres_left(g.h, g.h, p(B), p(Y), k, n, 1e-10, 0, ctypes.byref(it), ctypes.byref(rr),
                                 None) == 1
