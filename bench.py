"""Benchmark of the IFMM hot path on one MI355X.

Default workload (the precision configuration, the largest single-GPU one):
N = 2^20 points in 3D as 8 Gaussian clusters (sigma 0.05, seeded centres in
[0,1]^3), Gaussian kernel exp(-r^2/0.1^2) with 0.1 on the diagonal, octree
depth 7, Chebyshev order 4 (64 nodes per box), one N(0,1) right-hand side.
Two paths on the same GPU:
  * FP32 factors at eps = 1e-5 preconditioning FP64 GMRES (the timed step);
  * the plain FP64 IFMM at eps = 1e-10 preconditioning FP64 GMRES.
Inputs are seeded synthetic arrays (workloads.py) already resident in HBM
when the timed region starts.

One timed step = the whole path of the FP32 configuration: tree + H2
operators + sigma_0 + weights (build), level-by-level factorization in FP32,
and FP64 GMRES (H2 matvecs, FP32 factor solves) toward relative residual
1e-10 within --maxit iterations. value = the factorization rate N / t_factor
(Mpts/s), the metric's "IFMM factor Mpts/s".

Printed on one JSON line besides: GMRES time-to-1e-10 of both paths (build +
factorization + GMRES, with iterations, residual reached and whether 1e-10
was reached), p50/p99 single-RHS solve latency, the factorization's
utilisation of the matrix-core peak (algorithmic flops / time / peak), the
roofline of the dominant single-kernel family and the CPU oracle timed on a
bounded sample of the same workload. Kernel timing uses HIP events inside
the library: the warm-up step times every family; the timed steps time only
the dominant single-kernel family, every launch on its own.

The timed work is kept to about --time-budget seconds: when K steps of the
warm-up's duration would not fit, fewer are timed and "steps" says how many
("steps_requested" the number asked for).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)
os.environ.setdefault("IFMM_KTIMING", "1")

# HBM bytes per launch of a roofline kernel from rocprofv3 FETCH_SIZE / WRITE_SIZE counter runs, scaled by
# what the counters read for a 512 MiB device copy (--workload calib); valid for the kernel version the
# counters were taken on
MEASURED_TRAFFIC = {"k_qr_panel<float>": 6.698e7}   # HBM bytes per launch, profiles/k_qr_panel_cluster3d_1048576.txt

PEAKS = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp64_TFs": 78.6,      # FP64 vector and FP64 matrix (dense)
    "fp32_vec_TFs": 157.3,
    "fp32_mfma_TFs": 157.3,
}
from paper_1508_01835_amd.ifmm import KERNEL_OF_FAMILY, KERNEL_TYPED, KFAMILIES as FAMILIES  # noqa: E402


def family_roofline(name, flops, ms, launches, steps, precision):
    """Roofline entry of a single-kernel family: the rocprof kernel name and the peak it is held to. K_pre runs
    on the FP64 matrix cores; the other families run on the vector ALUs in the handle's precision (FP32:
    256 CUs x 2.4 GHz x 256 flop/clk = 157.3 TFLOP/s; FP64: 78.6 TFLOP/s)."""
    tname = "<float>" if precision == 32 else "<double>"
    kname = KERNEL_OF_FAMILY[name] + (tname if KERNEL_TYPED[name] else "")
    if name == "kpre":
        bound, peak = "mfma", PEAKS["fp64_TFs"]
    else:
        bound, peak = "alu", PEAKS["fp32_vec_TFs"] if precision == 32 else PEAKS["fp64_TFs"]
    achieved = flops / (ms * 1e-3) / 1e12 if ms > 0 else 0.0
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": "TFLOP/s", "frac": achieved / peak,
            "traffic": MEASURED_TRAFFIC.get(kname), "kernel": kname, "launches_per_step": launches / steps,
            "avg_launch_ms": ms / max(launches, 1), "flops_per_launch": flops / max(launches, 1)}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline():
    """The oracle, as it stands, on a bounded sample of the same workload."""
    import numpy as np

    import workloads as W
    from oracle.gmres import gmres_right
    from oracle.ifmm import IFMM as Oracle
    try:
        from threadpoolctl import threadpool_info
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        cores = 1
    n, depth, nrhs = 1024, 3, 16          # same 2 points per leaf box as the full workload
    pts = W.uniform_cube(n, 3, 2001)
    rhs = W.normal_rhs(n, nrhs, 2002)
    t0 = time.perf_counter()
    o = Oracle(pts, "imq", 0.005, 1.0, depth, 3, 1e-6)
    o.factorize()
    for k in range(nrhs):
        gmres_right(o.matvec, o.solve, rhs[:, k], tol=1e-10, maxit=200)
    t = time.perf_counter() - t0
    return {"value": n / t / 1e6, "unit": "Mpts/s", "cores": int(cores), "kind": "oracle",
            "sample": "N=1024 uniform in [0,1]^3, depth 3 (2 points per leaf as in the full workload), "
                      "order 3, eps 1e-6, build + factorize + GMRES to 1e-10 for 16 RHS; %.1f s" % t}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_cluster():
    """The oracle, as it stands, on a bounded sample of the clustered workload: the same generator, kernel,
    Chebyshev order and FP32-path tolerance at 2048 points (8 clusters of 256, depth 4), timed with every
    host thread the BLAS has and with one thread. value = the oracle's factorization rate (Mpts/s)."""
    import workloads as W
    from oracle.gmres import gmres_right
    from oracle.ifmm import IFMM as Oracle
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threadpool_limits, cores = None, 1
    wl = W.cluster3d(256, 4, 1e-5)

    def one():
        t0 = time.perf_counter()
        o = Oracle(wl.points, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, wl.eps)
        t1 = time.perf_counter()
        o.factorize()
        t2 = time.perf_counter()
        _, it, rr, _ = gmres_right(o.matvec, o.solve, wl.rhs[:, 0], tol=1e-10, maxit=200)
        t3 = time.perf_counter()
        return t1 - t0, t2 - t1, t3 - t2, it

    b_all, f_all, g_all, it = one()
    out = {"value": wl.n / f_all / 1e6, "unit": "Mpts/s", "cores": int(cores), "kind": "oracle",
           "cpu_model": cpu_model(),
           "sample": "clustered 3D, N=%d (8 clusters of 256, sigma 0.05), Gaussian h=0.1 + 0.1 I, depth 4, order 4, "
                     "eps 1e-5, FP64 oracle: build %.1f s, factorize %.1f s, GMRES to 1e-10 %.1f s (%d it); "
                     "value = N / factorize" % (wl.n, b_all, f_all, g_all, it)}
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            b1, f1, g1, _ = one()
        out["one_thread"] = {"value": wl.n / f1 / 1e6, "build_s": b1, "factorize_s": f1, "gmres_s": g1}
    return out


def run_cluster3d(args):
    """The clustered 2^20-point workload: FP32 factors (eps 1e-5) preconditioning FP64 GMRES as the timed
    step, the FP64 IFMM (eps 1e-10) path beside it, solve latency, utilisation and the CPU oracle."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1508_01835_amd import IFMM

    wl = W.cluster3d(args.n_per_cluster, args.depth_cluster)
    dev = torch.device("cuda:0")
    pts = torch.tensor(wl.points, device=dev)
    b = torch.tensor(np.ascontiguousarray(wl.rhs[:, 0]), device=dev)
    n = wl.n
    eps32, eps64 = 1e-5, 1e-10

    def step(precision, eps, maxit):
        t0 = time.perf_counter()
        g = IFMM(pts, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, eps, precision=precision)
        g.factorize()
        x, it, rr = g.gmres(b, tol=1e-10, maxit=maxit)
        torch.cuda.synchronize()
        return g, x, it, rr, time.perf_counter() - t0

    single = [f for f in range(len(FAMILIES)) if FAMILIES[f] in KERNEL_OF_FAMILY]
    os.environ["IFMM_KTIMING"] = "1"
    warm_stats, t_warm = None, None
    for _ in range(max(1, min(args.warmup, 1))):
        g, x, it, rr, t_warm = step(32, eps32, args.maxit)
        warm_stats = g.stats()
        g.close()
        log("warm-up step: %.1f s (factorize %.1f s), GMRES %d it, relres %.2e"
            % (t_warm, warm_stats["t_factor_ms"] * 1e-3, it, rr))
    torch.cuda.synchronize()
    K = max(1, min(args.steps, int(args.time_budget // max(t_warm, 1e-3))))
    dom_w = max(single, key=lambda f: warm_stats["kfam_ms"][f])
    os.environ["IFMM_KTIMING"] = "m%x" % (1 << dom_w)
    runs = []
    keep = None
    t0 = time.perf_counter()
    for k in range(K):
        g, x, it, rr, sec = step(32, eps32, args.maxit)
        runs.append((g.stats(), it, rr))
        log("timed step %d/%d: %.1f s" % (k + 1, K, sec))
        if k == K - 1:
            keep = (g, x, it, rr, sec)   # serves the latency and the FP32 leg below (outside the timed region)
        else:
            g.close()
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    os.environ["IFMM_KTIMING"] = "1"
    stats = [r[0] for r in runs]
    factor_ms = float(np.mean([s_["t_factor_ms"] for s_ in stats]))
    build_ms = float(np.mean([s_["t_build_ms"] for s_ in stats]))
    fam_ms = [sum(s_["kfam_ms"][f] for s_ in stats) for f in range(len(FAMILIES))]
    fam_fl = [sum(s_["kfam_flops"][f] for s_ in stats) for f in range(len(FAMILIES))]
    fam_nl = [sum(s_["kfam_launches"][f] for s_ in stats) for f in range(len(FAMILIES))]
    name = FAMILIES[dom_w]
    roof = family_roofline(name, fam_fl[dom_w], fam_ms[dom_w], fam_nl[dom_w], K, 32)
    breakdown = {FAMILIES[f]: round(warm_stats["kfam_ms"][f], 1) for f in range(len(FAMILIES))
                 if warm_stats["kfam_ms"][f] > 0}
    flops32 = float(np.mean([s_["factor_flops"] for s_ in stats]))
    util32 = flops32 / (factor_ms * 1e-3) / 1e12
    if args.quick:   # counter and trace runs: the timed steps only
        keep[0].close()
        out = {"metric": "IFMM factor Mpts/s (quick run)", "value": n / (factor_ms * 1e-3) / 1e6, "unit": "Mpts/s",
               "steps": K, "ms_per_step": T / K * 1e3, "kernel_ms_warmup_step": breakdown, "roofline": roof}
        if args.calib_copy:
            src = torch.ones(64 << 20, dtype=torch.float64, device=dev)   # 512 MiB
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            out["calib_copy_bytes"] = src.numel() * 8
        print(json.dumps(out))
        return

    # solve latency of the FP32 factors of the last timed step, one right-hand side
    g = keep[0]
    lat = []
    for _ in range(args.latency_reps + 3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.solve(b)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat[3:])
    st_lat = g.stats()

    # time to 1e-10 of both paths (build + factorization + GMRES). The FP32 path continues from the last timed
    # step's handle: its build and factorization times plus a GMRES run of up to --maxit-ttr iterations.
    # the library's GMRES restarts a column whose true residual, recomputed at exit, misses the tolerance
    ttr = {}
    legs = [("fp32", 32, eps32)] + ([] if args.skip_fp64 else [("fp64", 64, eps64)])
    for tag, prec, eps in legs:
        # the FP64 factorization takes minutes at 2^20: the library prints a line per eliminated level
        if prec == 64:
            os.environ["IFMM_PROGRESS"] = "1"
        if tag == "fp32":
            g = keep[0]
            t_g = time.perf_counter()
            x, it, rr = g.gmres(b, tol=1e-10, maxit=args.maxit_ttr)
            torch.cuda.synchronize()
            sg = g.stats()
            sec = sg["t_build_ms"] * 1e-3 + sg["t_factor_ms"] * 1e-3 + (time.perf_counter() - t_g)
        else:
            g, x, it, rr, sec = step(prec, eps, args.maxit_ttr)
            sg = g.stats()
        ttr[tag] = {"seconds": sec, "reached_1e-10": bool(rr <= 1e-10), "iters": it, "relres": rr, "eps": eps,
                    "build_s": sg["t_build_ms"] * 1e-3, "factor_s": sg["t_factor_ms"] * 1e-3,
                    "factor_mpts_s": n / sg["t_factor_ms"] / 1e3, "factor_flops": sg["factor_flops"],
                    "device_bytes_peak": sg["device_bytes_peak"], "factor_bytes": sg["factor_bytes"],
                    "max_rank": sg["max_rank"],
                    "kernel_ms": {FAMILIES[f]: round(sg["kfam_ms"][f], 1) for f in range(len(FAMILIES))
                                  if sg["kfam_ms"][f] > 0}}
        ttr[tag]["matrix_core_utilisation"] = {
            "achieved_TFs": sg["factor_flops"] / (sg["t_factor_ms"] * 1e-3) / 1e12,
            "peak_TFs": PEAKS["fp64_TFs"] if prec == 64 else PEAKS["fp32_mfma_TFs"]}
        ttr[tag]["matrix_core_utilisation"]["frac"] = (ttr[tag]["matrix_core_utilisation"]["achieved_TFs"] /
                                                      ttr[tag]["matrix_core_utilisation"]["peak_TFs"])
        log("%s leg: %.1f s (build %.1f, factorize %.1f), GMRES %d it, relres %.2e"
            % (tag, sec, sg["t_build_ms"] * 1e-3, sg["t_factor_ms"] * 1e-3, it, rr))
        if tag == "fp64":
            x64 = x
        else:
            x32 = x
        g.close()
        os.environ.pop("IFMM_PROGRESS", None)
    if not args.skip_probe:
        # FP32 factors at eps 1e-5 with a 40-iteration GMRES probe; when it fails, FP64 factors at
        # eps = min(1e-5, shift / (20 sigma_0)) (the serving loop's rule), all inside the leg's time
        from paper_1508_01835_amd.serve import factor_with_probe
        os.environ["IFMM_PROGRESS"] = "1"
        torch.cuda.synchronize()
        t = time.perf_counter()
        g, xp, it, rr = factor_with_probe(pts, b, (wl.kernel, wl.kparam, wl.shift), wl.order, eps32, 64, 1e-10,
                                          args.maxit_ttr, depth=wl.depth)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        sg = g.stats()
        ttr["probe"] = {"seconds": sec, "reached_1e-10": bool(rr <= 1e-10), "iters": it, "relres": rr,
                        "precision": sg["precision"], "eps": sg["eps"], "tau": sg["tau"],
                        "build_s": sg["t_build_ms"] * 1e-3, "factor_s": sg["t_factor_ms"] * 1e-3,
                        "device_bytes_peak": sg["device_bytes_peak"], "factor_bytes": sg["factor_bytes"],
                        "max_rank": sg["max_rank"]}
        log("probe leg: %.1f s, final factors FP%d eps %.3g, GMRES %d it in all, relres %.2e"
            % (sec, sg["precision"], sg["eps"], it, rr))
        g.close()
        os.environ.pop("IFMM_PROGRESS", None)
        if "fp64" in ttr and ttr["fp64"]["reached_1e-10"]:
            ttr["probe"]["relerr_vs_fp64_path"] = float(torch.linalg.norm(xp - x64) / torch.linalg.norm(x64))
    if "fp64" in ttr and ttr["fp64"]["reached_1e-10"]:
        # error of the FP32-preconditioned result against the FP64 path's converged solution
        ttr["fp32"]["relerr_vs_fp64_path"] = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
    keep[0].close()
    del pts, b
    torch.cuda.empty_cache()

    # the same two paths on the uniform 3D configuration (65536 points, IMQ c = 0.005 + 1.0 I, depth 5,
    # order 3, 16 right-hand sides), where FP32 factors are accurate enough to precondition
    ttr_u = {}
    if not args.skip_uniform:
        wu = W.uniform3d_65536()
        pu = torch.tensor(wu.points, device=dev)
        Bu = torch.tensor(np.ascontiguousarray(wu.rhs), device=dev)
        xs = {}
        for tag, prec, eps in (("fp32", 32, 1e-5), ("fp64", 64, 1e-10)):
            torch.cuda.synchronize()
            t = time.perf_counter()
            g = IFMM(pu, wu.kernel, wu.kparam, wu.shift, wu.depth, wu.order, eps, precision=prec)
            g.factorize()
            X, it, rr = g.gmres(Bu, tol=1e-10, maxit=200)
            torch.cuda.synchronize()
            sec = time.perf_counter() - t
            sg = g.stats()
            xs[tag] = X
            ttr_u[tag] = {"seconds": sec, "reached_1e-10": bool(rr <= 1e-10), "iters": it, "relres": rr, "eps": eps,
                          "build_s": sg["t_build_ms"] * 1e-3, "factor_s": sg["t_factor_ms"] * 1e-3}
            g.close()
            log("uniform3d %s: %.2f s, GMRES %d it, relres %.2e" % (tag, sec, it, rr))
        ttr_u["fp32"]["relerr_vs_fp64_path"] = float(torch.linalg.norm(xs["fp32"] - xs["fp64"]) /
                                                     torch.linalg.norm(xs["fp64"]))

    out = {
        "metric": "IFMM factor Mpts/s, GMRES time-to-1e-10 FP32 vs FP64; p50/p99 solve latency",
        "value": n / (factor_ms * 1e-3) / 1e6,
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": K,
        "steps_requested": args.steps,
        "warmup": 1,
        "ms_per_step": T / K * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cluster3d_%d: 8 Gaussian clusters (sigma 0.05) in 3D, Gaussian kernel h=0.1 + 0.1 I, "
                               "depth %d, Chebyshev order 4; step = build + FP32 factorization (eps 1e-5) + FP64 GMRES "
                               "(1 RHS, tol 1e-10, <= %d it)" % (n, wl.depth, args.maxit),
                   "n": n, "depth": wl.depth, "cheb_order": wl.order, "eps": eps32, "nrhs": 1},
        "factor_ms": factor_ms,
        "build_ms": build_ms,
        "step_gmres": {"iters": max(r[1] for r in runs), "relres": max(r[2] for r in runs)},
        "factor_matrix_core_utilisation": {"achieved_TFs": util32, "peak_TFs": PEAKS["fp32_mfma_TFs"],
                                           "frac": util32 / PEAKS["fp32_mfma_TFs"],
                                           "flops": "LAWN-41 counts of LU, triangular solves, Schur products, "
                                                    "recompressions, edge updates, merge and top (ifmm_stats)"},
        "time_to_1e-10_s": ttr,
        "time_to_1e-10_s_uniform3d_65536": ttr_u,
        "solve_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "nrhs": 1, "factors": "fp32", "factor_bytes": int(st_lat["factor_bytes"]),
                             "hbm_GBs_at_p50": st_lat["factor_bytes"] / (np.percentile(lat, 50) * 1e-3) / 1e9,
                             "hbm_peak_GBs": PEAKS["hbm_GBs"]},
        "max_rank": stats[0]["max_rank"],
        "device_bytes_peak": stats[0]["device_bytes_peak"],
        "kernel_ms_warmup_step": breakdown,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_cluster()
    print(json.dumps(out))


def run_batch(args):
    """Uneven batch: problems with N log-uniform in [1024, 16384] (sphere surface / unit cube alternating),
    IMQ c = 0.01 + 1.0 I, Chebyshev order 3, eps 1e-6, FP32 factors, depth from <= 64 points per leaf.
    Every problem has its own handle and stream; one ifmm_factorize_batch call factorizes them all."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    import torch

    import workloads as W
    from paper_1508_01835_amd import IFMM, factorize_batch

    count = args.batch_count
    sizes = [int(n) for n in W.batch_sizes(count)]
    log("batch: %d problems, %d points" % (count, sum(sizes)))
    streams = [torch.cuda.Stream() for _ in range(count)]

    def build(k):
        pts = torch.tensor(W.batch_problem(k, sizes[k]), device="cuda")
        return IFMM(pts, "imq", 0.01, 1.0, 0, 3, 1e-6, precision=32, leaf_max=64, stream=streams[k])

    t = time.perf_counter()
    with ThreadPoolExecutor(args.threads) as ex:
        hs = list(ex.map(build, range(count)))
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    warm = hs[: min(8, count)]
    factorize_batch(warm, args.threads)
    torch.cuda.synchronize()
    times = []
    for _ in range(args.steps):
        t = time.perf_counter()
        factorize_batch(hs, args.threads)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
    T = float(np.mean(times))
    # quality on a sample: relative residual of one FP32-factor solve against the FP64 H2 matvec
    worst = 0.0
    for k in range(0, count, max(1, count // 8)):
        b = torch.tensor(W.normal_rhs(sizes[k], 1, 4600 + k), device="cuda")
        x = hs[k].solve(b)
        r = (hs[k].matvec(x) - b).norm() / b.norm()
        worst = max(worst, float(r))
    peak = max(h.stats()["device_bytes_peak"] for h in hs)
    total = sum(h.stats()["device_bytes"] for h in hs)
    for h in hs:
        h.close()
    out = {
        "metric": "IFMM batched factor Mpts/s (uneven problems, FP32 factors)",
        "value": sum(sizes) / T / 1e6, "unit": "Mpts/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": T * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch%d: N log-uniform [1024, 16384], sphere/cube alternating, IMQ c=0.01 + 1.0 I, "
                               "order 3, eps 1e-6, <= 64 points per leaf" % count,
                   "problems": count, "points": sum(sizes), "threads": args.threads},
        "build_s": build_s, "max_relres_sample": worst,
        "device_bytes_resident": total, "device_bytes_peak_per_problem": peak,
    }
    print(json.dumps(out))


def run_solve(args):
    """Solve latency alone on the clustered 2^20-point workload: FP32 factors at eps 1e-5, then
    --latency-reps single-right-hand-side solves (HIP-graph replay), p50 / p99 and the rate over the stored
    factors. For kernel traces of the substitution without the bench's other legs."""
    import numpy as np
    import torch

    import workloads as W
    from paper_1508_01835_amd import IFMM

    wl = W.cluster3d(args.n_per_cluster, args.depth_cluster)
    pts = torch.tensor(wl.points, device="cuda")
    b = torch.tensor(np.ascontiguousarray(wl.rhs[:, 0]), device="cuda")
    g = IFMM(pts, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, 1e-5, precision=32)
    g.factorize()
    lat = []
    for _ in range(args.latency_reps + 3):
        torch.cuda.synchronize()
        t = time.perf_counter()
        g.solve(b)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat[3:])
    fb = g.stats()["factor_bytes"]
    g.close()
    p50 = float(np.percentile(lat, 50))
    print(json.dumps({"metric": "IFMM solve latency (1 RHS, FP32 factors)", "value": p50, "unit": "ms",
                      "p99": float(np.percentile(lat, 99)), "reps": int(lat.size), "factor_bytes": int(fb),
                      "hbm_GBs_at_p50": fb / (p50 * 1e-3) / 1e9, "higher_is_better": False,
                      "config": {"workload": "cluster3d_%d: FP32 factors at eps 1e-5, depth %d, order 4"
                                             % (wl.n, wl.depth)}}))


def run_calib():
    """Counter calibration: three device copies of 512 MiB (FP64 ones), so that rocprofv3's FETCH_SIZE and
    WRITE_SIZE per dispatch can be compared with the bytes known to move (run under --pmc)."""
    import torch
    a = torch.ones(64 << 20, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"metric": "counter calibration copy", "value": a.numel() * 8, "unit": "B per copy",
                      "copies": 3}))


def run_serve(args):
    """Serving loop: Poisson arrivals, 25% factorize (+ one solve) with N log-uniform in [8192, 524288]
    (uniform cube or 8 Gaussian clusters, half each), 75% solves of 1..64 right-hand sides on a resident
    factor; IMQ c = 0.01 + 1.0 I, Chebyshev order 3, eps 1e-5, FP32 factors (FP64 ones at eps <= shift /
    (20 sigma_0) where the FP32 factors fail a 40-iteration GMRES probe), FP64 GMRES to 1e-10."""
    import torch

    from paper_1508_01835_amd.serve import Server, synthetic_requests

    warm = synthetic_requests(3, rate=100.0, n_lo=2048, n_hi=2048, seed=5000)
    Server(hbm_budget_bytes=args.serve_budget).run(warm)
    torch.cuda.synchronize()
    reqs = synthetic_requests(args.serve_count, rate=args.rate, n_lo=8192, n_hi=524288, seed=5001)
    res = Server(hbm_budget_bytes=args.serve_budget, factor_workers=args.factor_workers, progress=True).run(reqs)
    out = {
        "metric": "IFMM serving p99 request latency (continuous batching, FP32 factors with FP64 fallback + "
                  "FP64 GMRES 1e-10)",
        "value": res["p99_ms"], "unit": "ms", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": res["wall_s"] * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "serve%d: Poisson %.2f req/s, 25%% factorize N log-uniform [8192, 524288] "
                               "(cube / 8 clusters), 75%% solve nrhs 1..64, IMQ c=0.01 + 1.0 I, order 3, "
                               "eps 1e-5, FP32 factors, FP64 where a 40-iteration probe fails"
                               % (args.serve_count, args.rate),
                   "hbm_budget_bytes": args.serve_budget, "factor_workers": args.factor_workers},
        "serve": res,
    }
    print(json.dumps(out))


# the paper's Tables 1-2 (Xeon E5-2650 v2, C++/Eigen): GMRES iterations and total CPU time [s] to 1e-10,
# N = 1e5 uniform in [-1,1]^3, kernel K(0)=1, r/d, d/r; eps 1e-3; rows: none, IFMM n = 1..4
PAPER_TABLES = {
    1e-3: {"none": (78, 509.0), 1: (19, 213.0), 2: (6, 119.0), 3: (3, 118.0), 4: (2, 265.0)},
    1e-2: {"none": (500, 4290.0), 1: (305, 2522.0), 2: (61, 521.0), 3: (24, 301.0), 4: (14, 414.0)},
}
# App. B, Tables 5-6: left preconditioning by order n -> (iterations, preconditioned relative residual,
# relative error of x) as printed
PAPER_LEFT = {
    1e-3: {1: (19, 3.5e-11, 4.5e-11), 2: (6, 9.1e-12, 9.2e-12), 3: (3, 2.8e-11, 2.8e-11), 4: (2, 2.0e-11, 2.0e-11)},
    1e-2: {1: (303, 5.4e-11, 5.2e-8), 2: (62, 9.3e-11, 5.2e-9), 3: (27, 3.8e-11, 2.0e-9), 4: (18, 3.8e-11, 1.6e-9)},
}


def run_paper(args):
    """The paper's own GMRES workload (Sec. 3.2, Tables 1-2): N = 1e5 points uniform in [-1,1]^3, kernel
    K(0)=1, r/d below d, d/r above, d in {1e-3, 1e-2}; IFMM preconditioner of Chebyshev order n = 1..4 and
    eps 1e-3 (FP64), octree depth 3 (about 195 points per leaf, the depth closest to the paper's 100);
    right-preconditioned non-restarted GMRES to 1e-10, at most 500 iterations, and GMRES without a
    preconditioner; with --paper-left also left preconditioning with the same factorization (App. B,
    Tables 5-6; its residual is the preconditioned one). Products use the Chebyshev H2 of order
    --paper-op-order (the paper's black-box FMM accuracy is not stated). x has N(0,1) entries and
    b = A~ x. Time per row = preconditioner build + factorization + GMRES (the operator's own build is
    reported apart)."""
    import torch

    import workloads as W
    from paper_1508_01835_amd import IFMM

    rows = []
    for d in (1e-3, 1e-2):
        wl = W.paper_cube(n=args.paper_n, d=d, order=args.paper_op_order)
        pts = torch.tensor(wl.points, device="cuda")
        t0 = time.perf_counter()
        op = IFMM(pts, wl.kernel, wl.kparam, wl.shift, wl.depth, args.paper_op_order, wl.eps, precision=64)
        torch.cuda.synchronize()
        t_op = time.perf_counter() - t0
        xt = torch.tensor(wl.rhs[:, 0], device="cuda")
        b = op.matvec(xt)
        torch.cuda.synchronize()
        for n in ["none", 1, 2, 3, 4]:
            t0 = time.perf_counter()
            pr = None
            if n != "none":
                pr = IFMM(pts, wl.kernel, wl.kparam, wl.shift, wl.depth, n, wl.eps, precision=64)
                pr.factorize()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, it, rr = op.gmres(b, tol=1e-10, maxit=500, prec=pr, precondition=pr is not None)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            err = float(torch.linalg.norm(x - xt) / torch.linalg.norm(xt))
            row = {"d": d, "precond": n if n == "none" else "ifmm_n%d" % n, "iters": it, "relres": rr,
                   "relerr": err, "seconds": t2 - t0, "construct_s": t1 - t0, "gmres_s": t2 - t1,
                   "op_build_s": t_op, "paper_iters": PAPER_TABLES[d][n][0],
                   "paper_cpu_s": PAPER_TABLES[d][n][1]}
            if pr is not None:
                row["max_rank"] = pr.stats()["max_rank"]
                if args.paper_left:
                    t3 = time.perf_counter()
                    xl, itl, rpl, rtl = op.gmres_left(b, tol=1e-10, maxit=500, prec=pr)
                    torch.cuda.synchronize()
                    errl = float(torch.linalg.norm(xl - xt) / torch.linalg.norm(xt))
                    row["left"] = {"iters": itl, "relres_prec": rpl, "relres_true": rtl, "relerr": errl,
                                   "gmres_s": time.perf_counter() - t3, "paper_iters": PAPER_LEFT[d][n][0],
                                   "paper_relres": PAPER_LEFT[d][n][1], "paper_relerr": PAPER_LEFT[d][n][2]}
                    log("paper d=%g %s left: %d it, prec relres %.2e, true %.2e, err %.2e (paper %d it, err %.1e)"
                        % (d, row["precond"], itl, rpl, rtl, errl, PAPER_LEFT[d][n][0], PAPER_LEFT[d][n][2]))
                pr.close()
            rows.append(row)
            log("paper d=%g %s: %d it, relres %.2e, err %.2e, %.2f s (paper %d it, %.0f s)" %
                (d, row["precond"], it, rr, err, row["seconds"], row["paper_iters"], row["paper_cpu_s"]))
        op.close()
    best = [r for r in rows if r["d"] == 1e-3 and r["precond"] == "ifmm_n3"][0]
    out = {
        "metric": "IFMM-preconditioned GMRES time to 1e-10, paper Table 1 workload (n = 3, d = 1e-3)",
        "value": best["seconds"], "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0,
        "ms_per_step": best["seconds"] * 1e3, "higher_is_better": False, "scaling": "weak",
        "vs_baseline": best["seconds"] / PAPER_TABLES[1e-3][3][1],
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "paper_cube: N=%d uniform [-1,1]^3, K = 1 / r/d / d/r, d in {1e-3, 1e-2}, "
                               "IFMM n=1..4 eps 1e-3 depth 3, GMRES 1e-10 <= 500 it, operator order %d"
                               % (args.paper_n, args.paper_op_order)},
        "paper_rows": rows,
    }
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--depth", type=int, default=5)
    ap.add_argument("--quick", action="store_true",
                    help="timed steps only: no latency, time-to-tolerance or CPU runs (for counter runs)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="end with a 512 MiB device-to-device copy, the reference for HBM byte counters")
    ap.add_argument("--workload", choices=["cluster3d", "uniform3d", "batch", "serve", "paper", "calib", "solve"],
                    default="cluster3d")
    ap.add_argument("--n-per-cluster", type=int, default=131072)
    ap.add_argument("--depth-cluster", type=int, default=7)
    ap.add_argument("--maxit", type=int, default=30, help="GMRES iterations of a timed step at most")
    ap.add_argument("--maxit-ttr", type=int, default=100, help="GMRES iterations of the time-to-1e-10 legs")
    ap.add_argument("--latency-reps", type=int, default=30)
    ap.add_argument("--skip-fp64", action="store_true", help="no FP64 eps 1e-10 leg (it takes minutes at 2^20)")
    ap.add_argument("--skip-probe", action="store_true",
                    help="no leg of FP32 factors with a GMRES probe and FP64 fallback (the serving loop's rule)")
    ap.add_argument("--skip-uniform", action="store_true", help="no FP32 / FP64 comparison on the uniform workload")
    ap.add_argument("--time-budget", type=float, default=100.0,
                    help="seconds of timed steps at most; fewer than --steps are timed when they would not fit")
    ap.add_argument("--paper-n", type=int, default=100000)
    ap.add_argument("--paper-left", action="store_true",
                    help="paper workload: also run left-preconditioned GMRES with each factorization")
    ap.add_argument("--paper-op-order", type=int, default=5)
    ap.add_argument("--serve-count", type=int, default=120)
    ap.add_argument("--rate", type=float, default=1.0)
    ap.add_argument("--factor-workers", type=int, default=2)
    ap.add_argument("--serve-budget", type=int, default=64 << 30)
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--threads", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "paper":
        run_paper(args)
        return
    if args.workload == "serve":
        run_serve(args)
        return
    if args.workload == "calib":
        run_calib()
        return
    if args.workload == "solve":
        run_solve(args)
        return
    if args.workload == "cluster3d":
        run_cluster3d(args)
        return

    import numpy as np
    import torch

    import workloads as W
    from paper_1508_01835_amd import IFMM

    wl = W.uniform3d_65536(n=args.n, depth=args.depth)
    dev = torch.device("cuda:0")
    pts = torch.tensor(wl.points, device=dev)
    B = torch.tensor(np.ascontiguousarray(wl.rhs), device=dev)
    n = wl.n

    def step(precision=64, eps=wl.eps):
        g = IFMM(pts, wl.kernel, wl.kparam, wl.shift, wl.depth, wl.order, eps, precision=precision)
        g.factorize()
        X, it, rr = g.gmres(B, tol=1e-10, maxit=200)
        return g, it, rr

    single = [f for f in range(len(FAMILIES)) if FAMILIES[f] in KERNEL_OF_FAMILY]
    warm_stats = None
    os.environ["IFMM_KTIMING"] = "1"
    for _ in range(args.warmup):
        g, it, rr = step()
        warm_stats = g.stats()
        g.close()
    torch.cuda.synchronize()
    if warm_stats is not None:   # time only the dominant single-kernel family in the timed steps
        dom_w = max(single, key=lambda f: warm_stats["kfam_ms"][f])
        os.environ["IFMM_KTIMING"] = "m%x" % (1 << dom_w)
    handles = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        g, it, rr = step()
        handles.append((g, it, rr))
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    os.environ["IFMM_KTIMING"] = "1"
    stats = [h[0].stats() for h in handles]
    iters = max(h[1] for h in handles)
    relres = max(h[2] for h in handles)
    if relres > 1e-10:
        log("GMRES did not reach 1e-10: %.3e" % relres)

    # kernel families over the timed region (sum over the timed handles); the
    # roofline reports the single-kernel family with the most device time, each
    # of its launches timed with its own HIP events on the handle's stream
    fam_ms = [sum(s["kfam_ms"][f] for s in stats) for f in range(len(FAMILIES))]
    fam_fl = [sum(s["kfam_flops"][f] for s in stats) for f in range(len(FAMILIES))]
    fam_nl = [sum(s["kfam_launches"][f] for s in stats) for f in range(len(FAMILIES))]
    dom = max(single, key=lambda f: fam_ms[f])
    name = FAMILIES[dom]
    roof = family_roofline(name, fam_fl[dom], fam_ms[dom], fam_nl[dom], args.steps, 64)
    if warm_stats is not None:   # every family, from the last warm-up step
        breakdown = {FAMILIES[f]: round(warm_stats["kfam_ms"][f], 2) for f in range(len(FAMILIES))
                     if warm_stats["kfam_ms"][f] > 0}
    else:
        breakdown = {FAMILIES[f]: round(fam_ms[f] / args.steps, 2) for f in range(len(FAMILIES)) if fam_ms[f] > 0}

    if args.quick:
        for h in handles:
            h[0].close()
        out = {"metric": "IFMM factor Mpts/s (quick run)", "value": n * args.steps / T / 1e6, "unit": "Mpts/s",
               "ms_per_step": T / args.steps * 1e3, "kernel_ms_per_step": breakdown, "roofline": roof}
        if args.calib_copy:
            src = torch.ones(64 << 20, dtype=torch.float64, device=dev)   # 512 MiB
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
            out["calib_copy_bytes"] = src.numel() * 8
        print(json.dumps(out))
        return
    g0 = handles[0][0]
    st0 = stats[0]
    factor_ms = float(np.mean([s["t_factor_ms"] for s in stats]))
    build_ms = float(np.mean([s["t_build_ms"] for s in stats]))
    # solve latency, single RHS, resident FP64 factors (outside the timed region)
    b1 = B[:, 0].contiguous()
    lat = []
    for _ in range(30):
        torch.cuda.synchronize()
        t = time.perf_counter()
        g0.solve(b1)
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - t) * 1e3)
    lat = np.array(lat[3:])
    for h in handles:
        h[0].close()

    # GMRES time-to-1e-10: FP32 factors (eps 1e-5) vs FP64 factors (eps 1e-6), same GPU
    ttr = {}
    for prec, eps in ((32, 1e-5), (64, 1e-6)):
        torch.cuda.synchronize()
        t = time.perf_counter()
        g, it2, rr2 = step(prec, eps)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t
        sg = g.stats()
        ttr["fp%d" % prec] = {"seconds": sec, "iters": it2, "relres": rr2, "eps": eps,
                              "build_ms": sg["t_build_ms"], "factor_ms": sg["t_factor_ms"],
                              "kernel_ms": {FAMILIES[f]: round(sg["kfam_ms"][f], 1) for f in range(len(FAMILIES))
                                            if sg["kfam_ms"][f] > 0}}
        g.close()

    out = {
        "metric": "IFMM factor Mpts/s, GMRES time-to-1e-10 FP32 vs FP64; p50/p99 solve latency",
        "value": n * args.steps / T / 1e6,
        "unit": "Mpts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": T / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "uniform3d_65536: N=65536 uniform [0,1]^3, IMQ c=0.005 + 1.0 I, depth 5, "
                               "Chebyshev order 3, eps 1e-6, GMRES 16 RHS to 1e-10",
                   "n": n, "depth": wl.depth, "cheb_order": wl.order, "eps": wl.eps, "nrhs": 16},
        "factor_mpts_s": n / (factor_ms * 1e-3) / 1e6,
        "factor_ms": factor_ms,
        "build_ms": build_ms,
        "gmres_iters": iters,
        "gmres_relres": relres,
        "time_to_1e-10_s": ttr,
        "time_to_1e-10_s_uniform3d_65536": ttr_u,
        "solve_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                             "nrhs": 1, "factor_bytes": int(st0["factor_bytes"]),
                             # every stored factor element is read once per solve: factor bytes / p50
                             "hbm_GBs_at_p50": st0["factor_bytes"] / (np.percentile(lat, 50) * 1e-3) / 1e9,
                             "hbm_peak_GBs": PEAKS["hbm_GBs"]},
        "max_rank": st0["max_rank"],
        "kernel_ms_per_step": breakdown,
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
