"""ifmm_solve_noalloc (the solve with the library's fixed device array as work storage) through the C ABI:
bitwise the result of ifmm_solve, on two calls in a row (the second with a smaller input) and in place;
a call whose work exceeds the array fails with IFMM_ERR_ARG."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


def colmajor(a):
    """(n, k) host array -> device buffer holding it column-major (a (k, n) contiguous tensor)."""
    return to_dev(np.ascontiguousarray(np.asarray(a).T))


def noalloc(g, B, X, nrhs):
    from paper_1508_01835_amd import ifmm as binding
    rc = binding.lib().ifmm_solve_noalloc(g.h, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                          nrhs, g.n)
    g.stream.synchronize()
    return rc


def reference(g, B, nrhs):
    from paper_1508_01835_amd import ifmm as binding
    X = torch.empty_like(B)
    rc = binding.lib().ifmm_solve(g.h, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()), nrhs, g.n)
    assert rc == 0
    return X


def test_noalloc_solve_equals_solve_on_consecutive_calls():
    from paper_1508_01835_amd import IFMM
    big = W.small_uniform(3000, 3, 231, 3, 3, 1e-6, kparam=0.005, nrhs=5)
    small = W.small_uniform(800, 2, 233, 4, 3, 1e-7, nrhs=2)
    g1 = IFMM(to_dev(big.points), big.kernel, big.kparam, big.shift, big.depth, big.order, big.eps)
    g2 = IFMM(to_dev(small.points), small.kernel, small.kparam, small.shift, small.depth, small.order, small.eps,
              precision=32)
    g1.factorize()
    g2.factorize()
    print("noalloc: call 1 (3000 points, 5 rhs, fp64)", flush=True)
    B1 = colmajor(big.rhs)
    X1 = torch.full_like(B1, np.nan)
    assert noalloc(g1, B1, X1, 5) == 0
    assert torch.equal(X1, reference(g1, B1, 5))
    print("noalloc: call 2 (800 points, 2 rhs, fp32 factors)", flush=True)
    B2 = colmajor(small.rhs)
    X2 = torch.full_like(B2, np.nan)
    assert noalloc(g2, B2, X2, 2) == 0
    assert torch.equal(X2, reference(g2, B2, 2))
    print("noalloc: in place, one rhs", flush=True)
    B3 = colmajor(big.rhs[:, 1:2])
    ref = reference(g1, B3, 1)
    assert noalloc(g1, B3, B3, 1) == 0
    assert torch.equal(B3, ref)
    g1.close()
    g2.close()


def test_noalloc_rejects_work_beyond_the_array():
    from paper_1508_01835_amd import IFMM
    from paper_1508_01835_amd import ifmm as binding
    wl = W.small_uniform(2000, 2, 235, 4, 3, 1e-6)
    g = IFMM(to_dev(wl.points), wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps)
    g.factorize()
    nrhs = 4200    # at least 2000 * 4200 * 8 bytes of work vector: above 64 MiB
    B = torch.zeros((nrhs, wl.n), dtype=torch.float64, device="cuda")
    X = torch.zeros_like(B)
    print("noalloc: oversized call", flush=True)
    assert noalloc(g, B, X, nrhs) == 1
    assert b"needs" in binding.lib().ifmm_last_error()
    g.close()
