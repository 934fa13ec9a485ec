"""Batched factorization of independent problems (ifmm_factorize_batch).

Each problem of the batch must give exactly the result it gives when built
and factorized alone: the batch only overlaps independent problems on their
own streams, it changes no arithmetic. Problems follow the uneven-batch
recipe (sizes log-uniform, sphere surface / unit cube alternating, IMQ
c = 0.01 + 1.0 I, Chebyshev order 3, eps 1e-6, depth from <= 64 points per
leaf), at sizes small enough for a test.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _problems(count=10, lo=600, hi=5000):
    sizes = W.batch_sizes(count, lo, hi, seed=4001)
    return [(k, int(n), W.batch_problem(k, int(n))) for k, n in enumerate(sizes)]


def _build(pts, precision, stream=None):
    from paper_1508_01835_amd import IFMM
    return IFMM(torch.tensor(pts, device="cuda"), "imq", 0.01, 1.0, 0, 3, 1e-6, precision=precision,
                leaf_max=64, stream=stream)


@pytest.mark.parametrize("precision", [32, 64])
def test_batch_equals_one_by_one(precision):
    from paper_1508_01835_amd import factorize_batch
    probs = _problems()
    print("batch sizes", [n for _, n, _ in probs], flush=True)
    alone = []
    for k, n, pts in probs:
        g = _build(pts, precision)
        g.factorize()
        b = torch.tensor(W.normal_rhs(n, 2, 4500 + k), device="cuda")
        alone.append((g.solve(b).cpu().numpy(), g.stats()["max_rank"]))
        g.close()
    streams = [torch.cuda.Stream() for _ in probs]
    hs = [_build(pts, precision, stream=s) for (_, _, pts), s in zip(probs, streams)]
    st = factorize_batch(hs, nthreads=4)
    assert st == [0] * len(hs)
    for (k, n, _), g, (xa, ra) in zip(probs, hs, alone):
        b = torch.tensor(W.normal_rhs(n, 2, 4500 + k), device="cuda")
        x = g.solve(b).cpu().numpy()
        assert g.stats()["max_rank"] == ra
        assert np.array_equal(x, xa), "problem %d differs from its single factorization" % k
        g.close()


def test_batch_argument_errors():
    from paper_1508_01835_amd import IFMMError, factorize_batch
    assert factorize_batch([], nthreads=2) == []
    k, n, pts = _problems(1)[0]
    g = _build(pts, 32)
    with pytest.raises(IFMMError) as e:
        factorize_batch([g, g], nthreads=2)
    assert e.value.code == 1   # IFMM_ERR_ARG: a handle twice
    with pytest.raises(IFMMError):
        factorize_batch([g], nthreads=0)
    g.close()
