"""Serving loop: resident factors (FP32, or FP64 where the FP32 ones fail the probe), coalesced FP64 GMRES
solves.

A burst of requests makes several solves pend on one factor, so they are
served by one multi-column GMRES call. Each request must still get exactly
the result it gets alone (the same factor by the same probe, GMRES on its own
right-hand sides), reach the tolerance, and be accounted with a completion time.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _alone(pts, fac_req, r):
    """Request r served alone: its factor built by the same probe from the factorize request, then r's own
    GMRES (a factorize request's result is the probe's)."""
    from paper_1508_01835_amd.serve import factor_with_probe
    p = torch.tensor(pts, device="cuda")
    b0 = torch.tensor(np.random.default_rng(fac_req.seed).standard_normal((p.shape[0], fac_req.nrhs)),
                      device="cuda")
    h, x, it, rr = factor_with_probe(p, b0, ("imq", 0.01, 1.0), 3, 1e-5, 64, 1e-10, 200)
    prec = h.stats()["precision"]
    if r.kind == "solve":
        B = torch.tensor(np.random.default_rng(r.seed).standard_normal((h.n, r.nrhs)), device="cuda")
        x, it, rr = h.gmres(B, tol=1e-10, maxit=200)
    h.close()
    return x.cpu().numpy(), prec


def test_mixed_requests_equal_alone():
    from paper_1508_01835_amd.serve import Server, synthetic_requests
    # a burst of mixed sizes (1000 to 12000 points): factorizations overlap each other and the solves
    reqs = synthetic_requests(16, rate=400.0, n_lo=1000, n_hi=12000, seed=5101, factorize_frac=0.3, nrhs_max=6)
    srv = Server(hbm_budget_bytes=1 << 36, keep_results=True, factor_workers=2)
    res = srv.run(reqs)
    print("serve", res, flush=True)
    assert res["requests"] == len(reqs)
    assert res["gmres_calls"] < res["solve_requests"]   # some solves were coalesced
    assert res["factorizations_in_flight_max"] == 2
    assert res["max_relres"] <= 1e-10
    assert all(r.t_done >= r.arrival for r in reqs)
    fac = {r.rid: r for r in reqs if r.kind == "factorize"}
    precs = set()
    for r in reqs:
        x, prec = _alone(fac[r.factor].points, fac[r.factor], r)
        precs.add(prec)
        assert np.array_equal(x, r.x), "request %d differs from its solve alone" % r.rid
    print("factor precisions", sorted(precs), flush=True)


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
