"""Thin ctypes binding of the IFMM C ABI (include/ifmm.h).

Argument marshalling only: every step runs in the HIP library libifmm.so.
PyTorch provides the device memory and the stream. There is no fallback: if
the library is missing, importing this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libifmm.so")

KERNELS = {"imq": 0, "gauss": 1, "paper": 2, "poly2": 3}

IFMM_OK = 0
STATUS = {0: "IFMM_OK", 1: "IFMM_ERR_ARG", 2: "IFMM_ERR_OOM", 3: "IFMM_ERR_SINGULAR",
          4: "IFMM_ERR_NUMERICAL", 5: "IFMM_ERR_STATE", 6: "IFMM_ERR_HIP", 7: "IFMM_ERR_INTERNAL"}


class Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("param", ctypes.c_double), ("diag_shift", ctypes.c_double)]


DevAllocFn = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
DevFreeFn = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("leaf_max", ctypes.c_int), ("rank_max", ctypes.c_int),
                ("sigma0_override", ctypes.c_double), ("hbm_budget_bytes", ctypes.c_int64),
                ("stream", ctypes.c_void_p), ("dev_alloc", DevAllocFn), ("dev_free", DevFreeFn),
                ("alloc_ctx", ctypes.c_void_p)]


def torch_allocator(stream):
    """dev_alloc / dev_free callbacks that take the handle's device buffers from PyTorch's caching
    allocator on `stream` (the handle's stream), so that the library and PyTorch share one pool.
    The allocator reuses a freed block only for work ordered after it on that stream, which is what the
    library's stream-ordered frees need. Keep the returned pair alive as long as the handle."""
    import torch
    dev = stream.device.index if stream.device.index is not None else torch.cuda.current_device()
    counts = {"alloc": 0, "free": 0, "live_bytes": 0}

    def _alloc(nbytes, ctx):
        try:
            p = torch.cuda.caching_allocator_alloc(int(nbytes), dev, stream)
        except Exception:   # out of memory or a torch error: the library fails the call with IFMM_ERR_OOM
            return None
        counts["alloc"] += 1
        counts["live_bytes"] += int(nbytes)
        return p

    def _free(ptr, nbytes, ctx):
        try:
            torch.cuda.caching_allocator_delete(ptr)
            counts["free"] += 1
            counts["live_bytes"] -= int(nbytes)
        except Exception:   # interpreter shutdown: the process is ending anyway
            pass

    return DevAllocFn(_alloc), DevFreeFn(_free), counts


class Stats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("dim", ctypes.c_int), ("depth", ctypes.c_int),
                ("cheb_order", ctypes.c_int), ("precision", ctypes.c_int),
                ("eps", ctypes.c_double), ("sigma0", ctypes.c_double), ("tau", ctypes.c_double),
                ("levels", ctypes.c_int), ("max_rank", ctypes.c_int * 32),
                ("mean_rank", ctypes.c_double * 32), ("boxes", ctypes.c_int64 * 32),
                ("t_build_ms", ctypes.c_double), ("t_sigma0_ms", ctypes.c_double),
                ("t_factor_ms", ctypes.c_double), ("t_last_solve_ms", ctypes.c_double),
                ("t_last_matvec_ms", ctypes.c_double), ("factor_flops", ctypes.c_double),
                ("schur_flops", ctypes.c_double), ("factor_bytes", ctypes.c_int64),
                ("device_bytes", ctypes.c_int64), ("device_bytes_peak", ctypes.c_int64),
                ("error_level", ctypes.c_int), ("error_box", ctypes.c_int),
                ("gmres_iters", ctypes.c_int), ("gmres_relres", ctypes.c_double),
                ("kfam_ms", ctypes.c_double * 24), ("kfam_flops", ctypes.c_double * 24),
                ("kfam_bytes", ctypes.c_double * 24), ("kfam_launches", ctypes.c_int64 * 24),
                ("gmres_restarts", ctypes.c_int)]

KFAMILIES = ["schur_gemm", "pivot_lu", "trsm_w", "qr", "jacobi_svd", "edge_update", "solve", "matvec", "other",
             "svd_round", "qr_panel", "qrcp", "svd_small", "row_xform", "col_xform", "qrcp_step", "qr_narrow",
             "kpre", "unused18", "unused19", "unused20", "unused21", "unused22", "unused23"]
# families holding exactly one kernel (per-launch timing), with its name
# families whose timed ranges each hold one launch of one kernel (rocprof name, templated on the element
# type or not); the other families span several kernels
KERNEL_OF_FAMILY = {"svd_round": "k_svd_round", "qr_panel": "k_qr_panel", "kpre": "k_kpre_tile"}
KERNEL_TYPED = {"svd_round": True, "qr_panel": True, "kpre": False}


EXPORTS = ["ifmm_default_options", "ifmm_build", "ifmm_factorize", "ifmm_factorize_batch", "ifmm_solve",
           "ifmm_solve_noalloc", "ifmm_matvec", "ifmm_gmres", "ifmm_gmres_left", "ifmm_query", "ifmm_query_ranks",
           "ifmm_destroy", "ifmm_strerror", "ifmm_last_error"]


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    if not os.path.exists(path):
        raise RuntimeError("libifmm.so is not built (%s); run __graft_entry__.build()" % path)
    lib = ctypes.CDLL(path)
    lib.ifmm_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.ifmm_default_options.restype = None
    lib.ifmm_build.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, Kernel, ctypes.c_int,
                               ctypes.c_int, ctypes.c_double, ctypes.POINTER(Options),
                               ctypes.POINTER(ctypes.c_void_p)]
    lib.ifmm_factorize.argtypes = [ctypes.c_void_p]
    lib.ifmm_factorize_batch.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_int,
                                         ctypes.POINTER(ctypes.c_int)]
    lib.ifmm_solve.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]
    lib.ifmm_solve_noalloc.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                                       ctypes.c_int64]
    lib.ifmm_query_ranks.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
    lib.ifmm_matvec.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int64]
    lib.ifmm_gmres.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                               ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_int),
                               ctypes.POINTER(ctypes.c_double)]
    lib.ifmm_gmres_left.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                    ctypes.c_int, ctypes.c_int64, ctypes.c_double, ctypes.c_int,
                                    ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.ifmm_query.argtypes = [ctypes.c_void_p, ctypes.POINTER(Stats)]
    lib.ifmm_destroy.argtypes = [ctypes.c_void_p]
    lib.ifmm_strerror.argtypes = [ctypes.c_int]
    lib.ifmm_strerror.restype = ctypes.c_char_p
    lib.ifmm_last_error.argtypes = []
    lib.ifmm_last_error.restype = ctypes.c_char_p
    for name in ["ifmm_build", "ifmm_factorize", "ifmm_factorize_batch", "ifmm_solve", "ifmm_solve_noalloc",
                 "ifmm_matvec", "ifmm_gmres", "ifmm_gmres_left", "ifmm_query", "ifmm_query_ranks", "ifmm_destroy"]:
        getattr(lib, name).restype = ctypes.c_int
    return lib


_LIB = None


def lib() -> ctypes.CDLL:
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


class IFMMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s: %s" % (STATUS.get(code, str(code)), msg))
        self.code = code


def _check(rc: int) -> None:
    if rc != IFMM_OK:
        raise IFMMError(rc, lib().ifmm_last_error().decode())


def _colmajor(t, n):
    """(n,) or (n, k) float64 CUDA tensor -> contiguous (k, n) buffer = column-major n x k."""
    import torch
    if t.dim() == 1:
        t = t[:, None]
    if t.shape[0] != n:
        raise ValueError("first dimension must be n = %d" % n)
    return t.to(torch.float64).t().contiguous()


class IFMM:
    """One IFMM handle: build on construction, then factorize / solve / matvec / gmres."""

    def __init__(self, points, kernel: str, param: float, shift: float, depth: int, order: int, eps: float,
                 precision: int = 64, rank_max: int = 0, sigma0: float = 0.0, leaf_max: int = 64,
                 hbm_budget_bytes: int = 0, stream=None, torch_alloc: bool = False):
        import torch
        if not points.is_cuda:
            raise ValueError("points must be a CUDA tensor")
        pts = points.to(torch.float64).contiguous()
        self.n, self.dim = pts.shape
        opt = Options()
        lib().ifmm_default_options(ctypes.byref(opt))
        opt.precision = precision
        opt.leaf_max = leaf_max
        opt.rank_max = rank_max
        opt.sigma0_override = sigma0
        opt.hbm_budget_bytes = hbm_budget_bytes
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        opt.stream = ctypes.c_void_p(self.stream.cuda_stream)
        self.alloc_counts = None
        if torch_alloc:   # device buffers from PyTorch's caching allocator, on the handle's stream
            fa, ff, self.alloc_counts = torch_allocator(self.stream)
            self._alloc_fns = (fa, ff)   # the callbacks outlive every library call of the handle
            opt.dev_alloc = fa
            opt.dev_free = ff
        k = Kernel(KERNELS[kernel], float(param), float(shift))
        h = ctypes.c_void_p()
        torch.cuda.current_stream().synchronize()   # the points are ready before the handle's stream reads them
        _check(lib().ifmm_build(ctypes.c_void_p(pts.data_ptr()), self.n, self.dim, k, depth, order, float(eps),
                                ctypes.byref(opt), ctypes.byref(h)))
        self.h = h
        self.precision = precision

    def factorize(self) -> None:
        _check(lib().ifmm_factorize(self.h))

    def _inputs_ready(self) -> None:
        """Inputs are written on the caller's current stream; the library reads them on the handle's."""
        import torch
        cur = torch.cuda.current_stream()
        if cur.cuda_stream != self.stream.cuda_stream:
            cur.synchronize()

    def solve(self, b):
        B = _colmajor(b, self.n)
        X = B.clone()
        self._inputs_ready()
        _check(lib().ifmm_solve(self.h, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                B.shape[0], self.n))
        out = X.t()
        return out[:, 0] if b.dim() == 1 else out

    def solve_noalloc(self, b):
        """ifmm_solve_noalloc: the same result as solve(), with the library's fixed device array as work
        storage. The call only enqueues work on the handle's stream; the returned tensor is ready once that
        stream has been synchronised (this wrapper does so)."""
        B = _colmajor(b, self.n)
        X = B.clone()
        self._inputs_ready()
        _check(lib().ifmm_solve_noalloc(self.h, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                        B.shape[0], self.n))
        self.stream.synchronize()
        out = X.t()
        return out[:, 0] if b.dim() == 1 else out

    def ranks(self, level: int) -> list:
        """Final rank of every box of a level (ifmm_query_ranks), boxes in Morton order."""
        nb = self.stats()["boxes"][level]
        out = (ctypes.c_int * max(nb, 1))()
        _check(lib().ifmm_query_ranks(self.h, int(level), out, int(nb)))
        return [out[i] for i in range(nb)]

    def matvec(self, x):
        Xc = _colmajor(x, self.n)
        Y = Xc.new_empty(Xc.shape)
        self._inputs_ready()
        _check(lib().ifmm_matvec(self.h, ctypes.c_void_p(Xc.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                 Xc.shape[0], self.n))
        out = Y.t()
        return out[:, 0] if x.dim() == 1 else out

    def gmres(self, b, tol: float = 1e-10, maxit: int = 500, prec: "IFMM | None" = None,
              precondition: bool = True):
        """GMRES on this handle's H2 operator; preconditioner: prec's factorization, else this handle's,
        none with precondition=False."""
        B = _colmajor(b, self.n)
        X = B.new_zeros(B.shape)
        it = ctypes.c_int()
        rr = ctypes.c_double()
        p = None if not precondition else (prec.h if prec is not None else self.h)
        self._inputs_ready()
        _check(lib().ifmm_gmres(self.h, p, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                B.shape[0], self.n, float(tol), int(maxit), ctypes.byref(it), ctypes.byref(rr)))
        out = X.t()
        return (out[:, 0] if b.dim() == 1 else out), it.value, rr.value

    def gmres_left(self, b, tol: float = 1e-10, maxit: int = 500, prec: "IFMM | None" = None,
                   precondition: bool = True):
        """Left-preconditioned GMRES on this handle's H2 operator (preconditioner chosen as in gmres).
        Returns (x, iterations, preconditioned relative residual, true relative residual)."""
        B = _colmajor(b, self.n)
        X = B.new_zeros(B.shape)
        it = ctypes.c_int()
        rr = ctypes.c_double()
        rt = ctypes.c_double()
        p = None if not precondition else (prec.h if prec is not None else self.h)
        self._inputs_ready()
        _check(lib().ifmm_gmres_left(self.h, p, ctypes.c_void_p(B.data_ptr()), ctypes.c_void_p(X.data_ptr()),
                                     B.shape[0], self.n, float(tol), int(maxit), ctypes.byref(it), ctypes.byref(rr),
                                     ctypes.byref(rt)))
        out = X.t()
        return (out[:, 0] if b.dim() == 1 else out), it.value, rr.value, rt.value

    def stats(self) -> dict:
        s = Stats()
        _check(lib().ifmm_query(self.h, ctypes.byref(s)))
        d = {}
        for name, _ in Stats._fields_:
            v = getattr(s, name)
            if isinstance(v, ctypes.Array):
                v = list(v)
            d[name] = v
        L = d["depth"]
        d["max_rank"] = {l: d["max_rank"][l] for l in range(2, L + 1)}
        d["mean_rank"] = {l: d["mean_rank"][l] for l in range(2, L + 1)}
        d["boxes"] = {l: d["boxes"][l] for l in range(2, L + 1)}
        return d

    def close(self) -> None:
        if getattr(self, "h", None):
            lib().ifmm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def factorize_batch(handles, nthreads: int = 8) -> list:
    """Factorize independent handles concurrently (ifmm_factorize_batch); per-problem status codes.

    Give each handle its own stream (IFMM(..., stream=torch.cuda.Stream())) so that the problems overlap on
    the device. Raises IFMMError if any problem failed."""
    n = len(handles)
    arr = (ctypes.c_void_p * max(n, 1))(*[h.h for h in handles])
    st = (ctypes.c_int * max(n, 1))()
    rc = lib().ifmm_factorize_batch(arr, n, int(nthreads), st)
    _check(rc)
    return [st[i] for i in range(n)]
