"""Serving loop: resident FP32 factors, coalesced FP64 GMRES solves.

A burst of requests makes several solves pend on one factor, so they are
served by one multi-column GMRES call. Each request must still get exactly
the result it gets alone (same factor, GMRES on its own right-hand sides),
reach the tolerance, and be accounted with a completion time.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_mixed_requests_equal_alone():
    from paper_1508_01835_amd import IFMM
    from paper_1508_01835_amd.serve import Server, synthetic_requests
    # a burst of mixed sizes (1000 to 12000 points): factorizations overlap each other and the solves
    reqs = synthetic_requests(16, rate=400.0, n_lo=1000, n_hi=12000, seed=5101, factorize_frac=0.3, nrhs_max=6)
    srv = Server(hbm_budget_bytes=1 << 36, keep_results=True, factor_workers=2)
    res = srv.run(reqs)
    print("serve", res, flush=True)
    assert res["requests"] == len(reqs)
    assert res["gmres_calls"] < len(reqs)           # some solves were coalesced
    assert res["factorizations_in_flight_max"] == 2
    assert res["max_relres"] <= 1e-10
    assert all(r.t_done >= r.arrival for r in reqs)
    pts = {r.rid: r.points for r in reqs if r.kind == "factorize"}
    for r in reqs:
        h = IFMM(torch.tensor(pts[r.factor], device="cuda"), "imq", 0.01, 1.0, 0, 3, 1e-5, precision=32,
                 leaf_max=64)
        h.factorize()
        B = torch.tensor(np.random.default_rng(r.seed).standard_normal((h.n, r.nrhs)), device="cuda")
        X, it, rr = h.gmres(B, tol=1e-10, maxit=200)
        h.close()
        assert np.array_equal(X.cpu().numpy(), r.x), "request %d differs from its solve alone" % r.rid


def test_admission_evicts_least_recently_used():
    from paper_1508_01835_amd.serve import Server, synthetic_requests
    reqs = synthetic_requests(10, rate=50.0, n_lo=1500, n_hi=2500, seed=5102, factorize_frac=0.6, nrhs_max=2)
    nf = sum(r.kind == "factorize" for r in reqs)
    srv = Server(hbm_budget_bytes=1)                # room for one factor at a time
    res = srv.run(reqs)
    print("serve", res, flush=True)
    assert res["requests"] == len(reqs)
    assert res["evicted"] >= nf - 1 - 1
    assert res["max_relres"] <= 1e-10
