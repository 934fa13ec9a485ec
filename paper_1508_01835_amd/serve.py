"""Serving loop on one GPU: resident IFMM factors, continuous batching of solves.

Two request kinds:
  * factorize: points (+ one right-hand side): build and factorize a handle
    (FP32 factors, FP64 when the FP32 ones fail the probe below), solve the
    right-hand side on the factorization's worker, keep the factor resident;
  * solve: right-hand sides for a resident factor: FP64 GMRES to the
    tolerance, preconditioned by the FP32 factors (Sec. 3.2 of the paper:
    the IFMM as a preconditioner).

Precision of a factor (factor_with_probe): FP32 factors first. The
factorize request's own solve is the probe: FP64 GMRES preconditioned by
them, at most `probe_maxit` iterations. When it does not reach the
tolerance, the handle is built again with FP64 factors (sigma_0 passed in)
and eps lowered so that tau = eps sigma_0 is at most shift / 20. The probe
is needed because the FP32 error depends on the cloud, not on a bound: on
clustered clouds the FP32 factors lose far more than FP32 rounding at the
same truncation level as FP64. Measured at 131072 clustered points, the
FP32 and FP64 solves differ by 4e-5, 8e-3 and 2.4 at shifts 10, 1 and 0.1.
On the uniform cube the FP32 factors still precondition at sigma_0 / shift
near 1e5. The kernels served are positive definite, so the shift bounds the
smallest eigenvalue from below. A tau at or above it leaves GMRES stalled.

Scheduling (host side; every step of a request runs in the HIP library):
  * admission: a factorization starts only when the device bytes of the
    resident factors, of the factorizations in flight and of the solve
    lane's GMRES workspace, plus its own estimate, fit the budget;
    least-recently-used factors with no pending work are evicted to make
    room. A factor's bytes are re-read after every call on it;
  * up to `factor_workers` factorizations run at once, each on a worker
    thread and a stream of its own, overlapping each other and the solves;
  * continuous batching: when the solve lane is free it takes the factor of
    the oldest pending solve and runs all pending solves of that factor as one
    multi-column GMRES call. Columns are independent GMRES runs, so a request
    gets the same result alone or in a mix;
  * latency = completion - arrival, per request.
"""
from __future__ import annotations

import sys
import threading
import time
from collections import OrderedDict
from dataclasses import dataclass, field

import numpy as np

from .ifmm import IFMM


TAU_SHIFT_FRAC = 0.05    # FP64 fallback: tau = eps sigma_0 at most this fraction of the shift


def factor_with_probe(points, b, kernel, order: int, eps: float, leaf_max: int, tol: float, maxit: int,
                      probe_maxit: int = 40, stream=None, depth: int = 0):
    """Build, factorize and solve one problem: FP32 factors, and if FP64 GMRES preconditioned by them does
    not reach `tol` within `probe_maxit` iterations, FP64 factors at min(eps, TAU_SHIFT_FRAC shift / sigma_0)
    and GMRES again with `maxit`. points: CUDA tensor n x 3; b: CUDA tensor (n,) or (n, k); depth 0: from
    leaf_max. Returns (handle, x, iterations of both GMRES runs, relres)."""
    k, c, s = kernel
    h = IFMM(points, k, c, s, depth, order, eps, precision=32, leaf_max=leaf_max, stream=stream)
    h.factorize()
    x, it, rr = h.gmres(b, tol=tol, maxit=min(probe_maxit, maxit))
    if rr <= tol:
        return h, x, it, rr
    sigma0 = h.stats()["sigma0"]
    h.close()
    eps64 = min(eps, TAU_SHIFT_FRAC * s / sigma0) if s > 0 else eps
    h = IFMM(points, k, c, s, depth, order, eps64, precision=64, leaf_max=leaf_max, stream=stream,
             sigma0=sigma0)
    h.factorize()
    x, it2, rr = h.gmres(b, tol=tol, maxit=maxit)
    return h, x, it + it2, rr


@dataclass
class Request:
    rid: int
    arrival: float                       # seconds from the start of the run
    kind: str                            # "factorize" or "solve"
    points: np.ndarray | None = None     # factorize: n x 3
    cluster: bool = False
    nrhs: int = 1                        # solve: right-hand sides
    seed: int = 0
    # filled in by the server
    factor: int = -1
    t_done: float = -1.0
    iters: int = 0
    relres: float = 0.0
    x: np.ndarray | None = None


@dataclass
class _Factor:
    fid: int
    handle: IFMM
    n: int
    bytes: int
    last_use: float
    pending: list = field(default_factory=list)


class Server:
    def __init__(self, hbm_budget_bytes: int, kernel=("imq", 0.01, 1.0), order: int = 3, eps: float = 1e-5,
                 leaf_max: int = 64, tol: float = 1e-10, maxit: int = 200, keep_results: bool = False,
                 factor_workers: int = 2, gmres_iters_estimate: int = 40, progress: bool = False):
        import torch
        self.torch = torch
        self.budget = int(hbm_budget_bytes)
        self.kernel, self.order, self.eps, self.leaf_max = kernel, order, eps, leaf_max
        self.tol, self.maxit, self.keep = tol, maxit, keep_results
        self.factor_workers = max(1, int(factor_workers))
        self.gmres_iters_estimate = gmres_iters_estimate
        self.progress = progress          # a line on stderr for every finished solve batch
        self.factors: "OrderedDict[int, _Factor]" = OrderedDict()
        self.bytes_per_point = 4.0e4      # first estimate; replaced by what factorizations use
        self.solve_stream = torch.cuda.Stream()
        self.stats = {"factorized_points": 0, "factor_busy_s": 0.0, "solve_busy_s": 0.0, "evicted": 0,
                      "gmres_calls": 0, "rhs": 0, "fp64_factors": 0}

    # ------------------------------------------------------------ factors
    def _resident_bytes(self) -> int:
        return sum(f.bytes for f in self.factors.values())

    def _gmres_bytes(self, n: int, nrhs: int) -> int:
        """Device bytes of one GMRES call: Krylov and preconditioned bases (2 x iterations) plus work vectors."""
        return 8 * n * nrhs * (2 * self.gmres_iters_estimate + 6)

    def _make_room(self, need: int, busy: set) -> bool:
        while self._resident_bytes() + self.inflight + need > self.budget:
            victims = [f for f in self.factors.values() if not f.pending and f.fid not in busy]
            if not victims:
                return False
            v = min(victims, key=lambda f: f.last_use)
            v.handle.close()
            del self.factors[v.fid]
            self.stats["evicted"] += 1
        return True

    def _factorize(self, req: Request, stream, out: dict) -> None:
        torch = self.torch
        t0 = time.perf_counter()
        try:
            with torch.cuda.stream(stream):
                pts = torch.tensor(req.points, device="cuda")
                b = torch.tensor(np.random.default_rng(req.seed).standard_normal((pts.shape[0], req.nrhs)),
                                 device="cuda")
                h, x, it, rr = factor_with_probe(pts, b, self.kernel, self.order, self.eps, self.leaf_max,
                                                 self.tol, self.maxit, stream=stream)
                out["x"] = x.cpu().numpy() if self.keep else None
                out["iters"], out["relres"] = it, rr
            out["handle"] = h
        except Exception as e:   # reported with the request
            out["error"] = e
        out["seconds"] = time.perf_counter() - t0

    # ------------------------------------------------------------ solves
    def _solve_batch(self, f: _Factor, reqs: list, now) -> None:
        torch = self.torch
        cols = [np.random.default_rng(r.seed).standard_normal((f.n, r.nrhs)) for r in reqs]
        B = torch.tensor(np.concatenate(cols, axis=1), device="cuda")
        # the Krylov storage of a call grows to 2 (maxit + 1) vectors per column in the worst case: the
        # columns go in groups that keep it within a quarter of the budget (every column is its own GMRES
        # run, so the grouping changes no result)
        per_col = 16 * f.n * (self.maxit + 1)
        group = max(1, (self.budget // 4) // per_col)
        t0 = time.perf_counter()
        Xs, it, rr = [], 0, 0.0
        with torch.cuda.stream(f.handle.stream):
            for c0 in range(0, B.shape[1], group):
                Xg, itg, rrg = f.handle.gmres(B[:, c0:c0 + group].contiguous(), tol=self.tol, maxit=self.maxit)
                Xs.append(Xg)
                it, rr = max(it, itg), max(rr, rrg)
                self.stats["gmres_calls"] += 1
        X = Xs[0] if len(Xs) == 1 else torch.cat(Xs, dim=1)
        self.stats["solve_busy_s"] += time.perf_counter() - t0
        f.bytes = int(f.handle.stats()["device_bytes"])   # what the handle holds now (the Krylov storage is freed)
        self.stats["rhs"] += B.shape[1]
        t_done = now()
        Xh = X.cpu().numpy() if self.keep else None
        c0 = 0
        for r in reqs:
            r.t_done, r.iters, r.relres = t_done, it, rr
            if Xh is not None:
                r.x = Xh[:, c0:c0 + r.nrhs].copy()
            c0 += r.nrhs
        f.last_use = t_done

    # ------------------------------------------------------------ loop
    def run(self, requests: list) -> dict:
        requests = sorted(requests, key=lambda r: r.arrival)
        t_start = time.perf_counter()

        def now():
            return time.perf_counter() - t_start

        rng = np.random.default_rng(5001)
        arrived = 0
        fq: list = []                 # factorize requests waiting for admission
        orphans: list = []            # solve requests that arrived with no resident factor
        workers: list = []            # (thread, request, out, stream, reserved bytes)
        self.inflight = 0             # bytes reserved by the factorizations in flight
        done = 0
        total = len(requests)
        peak_inflight = 0
        while done < total:
            t = now()
            while arrived < total and requests[arrived].arrival <= t:
                r = requests[arrived]
                arrived += 1
                if r.kind == "factorize":
                    fq.append(r)
                else:
                    orphans.append(r)
            # solve requests pick a resident factor (uniformly) when one exists
            if orphans and self.factors:
                ids = list(self.factors.keys())
                for r in orphans:
                    r.factor = ids[int(rng.integers(len(ids)))]
                    self.factors[r.factor].pending.append(r)
                orphans = []
            # finished factorizations: make them resident, queue their own solves
            for w in [w for w in workers if not w[0].is_alive()]:
                workers.remove(w)
                th, r, out, stream, reserved = w
                self.inflight -= reserved
                self.stats["factor_busy_s"] += out["seconds"]
                if "error" in out:
                    r.t_done, r.relres = now(), float("nan")
                    done += 1
                    continue
                h = out["handle"]
                st = h.stats()
                f = _Factor(r.rid, h, h.n, int(st["device_bytes"]), now())
                # reservation of later factorizations: the peak of this one per point (build and elimination)
                self.bytes_per_point = max(self.bytes_per_point * 0.5, 1.2 * st["device_bytes_peak"] / f.n)
                self.stats["fp64_factors"] += st["precision"] == 64
                self.factors[r.rid] = f
                self.stats["factorized_points"] += f.n
                r.factor = r.rid
                r.t_done, r.iters, r.relres, r.x = now(), out["iters"], out["relres"], out["x"]
                done += 1
                if self.progress:
                    print("[serve] %d / %d requests done, %.1f s (factorization of %d points, FP%d, %d it)"
                          % (done, total, now(), f.n, st["precision"], r.iters), file=sys.stderr, flush=True)
            # start admitted factorizations while workers are free
            while len(workers) < self.factor_workers and fq:
                r = fq[0]
                n = r.points.shape[0]
                need = int(self.bytes_per_point * n) + self._gmres_bytes(n, 1)
                if not (self._make_room(need, set()) or (not self.factors and not workers)):
                    break
                fq.pop(0)
                out: dict = {}
                stream = self.torch.cuda.Stream()
                th = threading.Thread(target=self._factorize, args=(r, stream, out))
                th.start()
                workers.append((th, r, out, stream, need))
                self.inflight += need
                peak_inflight = max(peak_inflight, len(workers))
            # solve lane: the factor of the oldest pending solve, all its pending solves at once
            pend = [f for f in self.factors.values() if f.pending]
            if pend:
                f = min(pend, key=lambda f: min(q.arrival for q in f.pending))
                reqs, f.pending = f.pending, []
                self._solve_batch(f, reqs, now)
                if self.progress:
                    print("[serve] %d / %d requests done, %.1f s (factor of %d points, %d columns)"
                          % (done + len(reqs), total, now(), f.n, sum(r.nrhs for r in reqs)),
                          file=sys.stderr, flush=True)
                done += len(reqs)
                continue
            if not workers and not fq and arrived < total:
                time.sleep(max(0.0, min(0.002, requests[arrived].arrival - now())))
            elif workers:
                workers[0][0].join(timeout=0.002)
        wall = now()
        for f in self.factors.values():
            f.handle.close()
        self.factors.clear()
        lat = np.array([r.t_done - r.arrival for r in requests])
        fl = np.array([r.t_done - r.arrival for r in requests if r.kind == "factorize"])
        sl = np.array([r.t_done - r.arrival for r in requests if r.kind == "solve"])
        res = {
            "requests": total, "wall_s": wall, "req_per_s": total / wall,
            "rhs_per_s": self.stats["rhs"] / wall,
            "factorized_mpts_per_s": self.stats["factorized_points"] / max(self.stats["factor_busy_s"], 1e-9) / 1e6,
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "factorize_p50_ms": float(np.percentile(fl, 50) * 1e3) if fl.size else None,
            "solve_p50_ms": float(np.percentile(sl, 50) * 1e3) if sl.size else None,
            "solve_p99_ms": float(np.percentile(sl, 99) * 1e3) if sl.size else None,
            "max_relres": float(max(r.relres for r in requests)),
            "max_iters": int(max(r.iters for r in requests)),
            "solve_requests": int(sum(r.kind == "solve" for r in requests)),
            "factorizations_in_flight_max": peak_inflight,
        }
        res.update(self.stats)
        return res


def synthetic_requests(count: int, rate: float, n_lo: int, n_hi: int, seed: int = 5001,
                       factorize_frac: float = 0.25, nrhs_max: int = 64) -> list:
    """Poisson arrivals; a fraction of factorize requests (N log-uniform in [n_lo, n_hi], uniform cube or 8
    Gaussian clusters of width 0.05, half each), the rest solve requests with nrhs uniform in 1..nrhs_max.
    The first request is a factorization so that solves have a factor to go to."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(count):
        t += float(rng.exponential(1.0 / rate))
        if k == 0 or rng.random() < factorize_frac:
            n = int(round(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi)))))
            cl = bool(rng.random() < 0.5)
            if cl:
                cen = rng.random((8, 3))
                pts = cen[rng.integers(0, 8, n)] + 0.05 * rng.standard_normal((n, 3))
            else:
                pts = rng.random((n, 3))
            out.append(Request(k, t, "factorize", points=pts, cluster=cl, nrhs=1, seed=seed * 1000 + k))
        else:
            out.append(Request(k, t, "solve", nrhs=int(rng.integers(1, nrhs_max + 1)), seed=seed * 1000 + k))
    return out
