"""Caller-supplied device allocator (dev_alloc / dev_free in ifmm_options).

A handle whose device buffers come from PyTorch's caching allocator must
compute exactly what a handle on the library's own block cache computes
(the allocator changes where buffers live, no arithmetic), must return every
block it took by the time it is destroyed, also when a build fails part way,
and must work from the worker threads of a batched factorization. The cache
is filled with NaN blocks first, so a read of a freed or unwritten buffer
cannot pass unnoticed.
"""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def to_dev(a):
    return torch.tensor(np.ascontiguousarray(a), device="cuda")


@pytest.mark.parametrize("precision", [64, 32])
def test_torch_allocator_equals_own_pool(precision):
    from paper_1508_01835_amd import IFMM
    wl = W.small_uniform(3000, 3, 241, 3, 3, 1e-6, kparam=0.005, nrhs=3)
    pts, b = to_dev(wl.points), to_dev(wl.rhs)
    res = []
    for torch_alloc in (False, True):
        if torch_alloc:
            # PyTorch's cache then holds NaN-filled blocks of many sizes: a buffer read before it is written, or
            # through a pointer that a re-upload moved, gives NaN or a wild offset instead of the old contents
            junk = [torch.full((1 << k,), float("nan"), dtype=torch.float64, device="cuda") for k in list(range(5, 22)) * 2]
            del junk
        torch.cuda.synchronize()
        before = torch.cuda.memory_allocated()
        g = IFMM(pts, wl.kernel, wl.kparam, wl.shift, 3, 3, 1e-6, precision=precision, torch_alloc=torch_alloc)
        g.factorize()
        x = g.solve(b)
        y = g.matvec(b)
        xg, it, rr = g.gmres(b, tol=1e-10, maxit=100, prec=g)
        res.append((x.cpu(), y.cpu(), xg.cpu(), it, rr, g.stats()["max_rank"]))
        held = torch.cuda.memory_allocated() - before
        counts = g.alloc_counts
        print("torch_alloc", torch_alloc, "torch-held bytes", held, "counts", counts, flush=True)
        if torch_alloc:
            assert counts["alloc"] > 10 and counts["live_bytes"] > 0
            assert held >= counts["live_bytes"]          # the handle's buffers are PyTorch's blocks
        g.close()
        if torch_alloc:
            assert counts["free"] == counts["alloc"] and counts["live_bytes"] == 0
    (x0, y0, g0, i0, r0, k0), (x1, y1, g1, i1, r1, k1) = res
    assert torch.equal(x0, x1) and torch.equal(y0, y1) and torch.equal(g0, g1)
    assert i0 == i1 and r0 == r1 and k0 == k1


def test_failing_allocator_gives_oom_and_returns_every_block():
    """dev_alloc succeeds a few times, then returns NULL: the build fails with IFMM_ERR_OOM and the library
    hands back every block it had taken."""
    from paper_1508_01835_amd import ifmm as binding
    wl = W.small_uniform(2000, 3, 243, 3, 3, 1e-6)
    pts = to_dev(wl.points)
    lib = binding.lib()
    stream = torch.cuda.current_stream()
    for allow in (0, 3, 12):
        live = {}

        def _alloc(nbytes, ctx):
            if len(live) >= allow:
                return None
            p = torch.cuda.caching_allocator_alloc(int(nbytes), pts.device.index, stream)
            live[p] = int(nbytes)
            return p

        def _free(ptr, nbytes, ctx):
            assert live.pop(ptr) == nbytes
            torch.cuda.caching_allocator_delete(ptr)

        fa, ff = binding.DevAllocFn(_alloc), binding.DevFreeFn(_free)
        opt = binding.Options()
        lib.ifmm_default_options(ctypes.byref(opt))
        opt.stream = ctypes.c_void_p(stream.cuda_stream)
        opt.dev_alloc, opt.dev_free = fa, ff
        h = ctypes.c_void_p()
        rc = lib.ifmm_build(ctypes.c_void_p(pts.data_ptr()), wl.points.shape[0], 3,
                            binding.Kernel(binding.KERNELS[wl.kernel], wl.kparam, wl.shift), 3, 3, 1e-6,
                            ctypes.byref(opt), ctypes.byref(h))
        print("allow", allow, "rc", rc, lib.ifmm_last_error(), flush=True)
        assert rc == 2 and not h.value               # IFMM_ERR_OOM
        assert live == {}


def test_torch_allocator_in_batched_factorization():
    """Worker threads of ifmm_factorize_batch call the Python callbacks; results equal the one-by-one run."""
    from paper_1508_01835_amd import IFMM, factorize_batch
    sizes = W.batch_sizes(6, 600, 4000, seed=4003)
    probs = [(k, int(n), W.batch_problem(k, int(n))) for k, n in enumerate(sizes)]
    alone = []
    for k, n, pts in probs:
        g = IFMM(to_dev(pts), "imq", 0.01, 1.0, 0, 3, 1e-6, precision=32, leaf_max=64)
        g.factorize()
        alone.append(g.solve(to_dev(W.normal_rhs(n, 2, 4600 + k))).cpu())
        g.close()
    streams = [torch.cuda.Stream() for _ in probs]
    hs = [IFMM(to_dev(pts), "imq", 0.01, 1.0, 0, 3, 1e-6, precision=32, leaf_max=64, stream=s, torch_alloc=True)
          for (_, _, pts), s in zip(probs, streams)]
    assert factorize_batch(hs, nthreads=3) == [0] * len(hs)
    for (k, n, _), g, xa in zip(probs, hs, alone):
        x = g.solve(to_dev(W.normal_rhs(n, 2, 4600 + k))).cpu()
        assert torch.equal(x, xa), "problem %d differs" % k
        counts = g.alloc_counts
        g.close()
        assert counts["free"] == counts["alloc"] and counts["live_bytes"] == 0
