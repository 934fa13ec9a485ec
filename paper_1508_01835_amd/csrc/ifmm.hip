// C ABI of the IFMM library (include/ifmm.h). Every entry point converts
// failures into status codes; nothing throws across the boundary.
#include <algorithm>
#include <atomic>
#include <map>
#include <mutex>
#include <thread>

#include "gmres.hpp"

using namespace ifmm;

namespace {

thread_local std::string g_last_error;

template <class T>
struct Factors : FactorStoreBase {
  FactorStore<T> F;
  SolvePlan<T> S;
};

template <class F>
int guarded(F&& fn) {
  try {
    fn();
    g_last_error.clear();
    return IFMM_OK;
  } catch (const Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return IFMM_ERR_OOM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return IFMM_ERR_INTERNAL;
  } catch (...) {
    g_last_error = "unknown failure";
    return IFMM_ERR_INTERNAL;
  }
}

// Non-finite detection (IFMM_ERR_NUMERICAL). Word 2 of the handle's device
// info block is set by the vector checks, word 3 by the factor scan; -1 means
// clean. A thread that meets a NaN or an infinity stores its tag: every such
// store writes the same kind of value, so the race between them is harmless.
constexpr int INFO_VEC = 2, INFO_FAC = 3;

__global__ void k_nonfinite_vec(const double* __restrict__ v, int64_t n, int nrhs, int64_t ld, int tag,
                                int* __restrict__ info) {
  const int64_t total = n * nrhs;
  bool bad = false;
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < total; e += (int64_t)gridDim.x * WG) {
    const int64_t t = e % n, c = e / n;
    bad = bad || !isfinite(v[t + c * ld]);
  }
  if (bad) info[INFO_VEC] = tag;
}

struct FiniteSpan {
  const void* p;
  int64_t count;
  int tag;
  int pad;
};

// One workgroup per span (a stored factor block).
template <class T>
__global__ void k_nonfinite_spans(const FiniteSpan* __restrict__ sp, int* __restrict__ info) {
  const FiniteSpan s = sp[blockIdx.x];
  const T* v = static_cast<const T*>(s.p);
  bool bad = false;
  for (int64_t e = threadIdx.x; e < s.count; e += WG) bad = bad || !isfinite((double)v[e]);
  if (bad) atomicMax(info + INFO_FAC, s.tag);   // the finest level holding one (-1: none)
}

// Launch the check of an n x nrhs block (leading dimension ld); the host reads
// the verdict with finite_verdict after its next synchronisation.
void check_finite_vec(Problem& P, const double* v, int64_t n, int nrhs, int64_t ld, int tag) {
  const int64_t total = n * nrhs;
  const unsigned g = (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(total, WG)));
  hipLaunchKernelGGL(k_nonfinite_vec, dim3(g), dim3(WG), 0, P.stream, v, n, nrhs, ld, tag, P.d_info);
  IFMM_LAUNCH_CHECK();
}

void reset_finite(Problem& P) {
  IFMM_HIP(hipMemsetAsync(P.d_info + INFO_VEC, 0xff, sizeof(int) * 2, P.stream));
}

// Reads both words (synchronises); returns the vector tag (-1: clean).
int finite_verdict(Problem& P) {
  std::vector<int> info;
  P.download(info, P.d_info, 4);
  return info[INFO_VEC];
}

// Scan the stored factors for non-finite values; fails with IFMM_ERR_NUMERICAL
// naming the finest level where one sits (where it arose: the elimination
// carries fill upwards only).
template <class T>
void scan_factors(Problem& P, FactorStore<T>& F) {
  // the blocks H = [A; G] and W_x of every elimination (padding between them is never written)
  std::vector<FiniteSpan> sp;
  for (int l = (int)F.cls.size() - 1; l >= 2; --l)
    for (const auto& cf : F.cls[l]) {
      const T* sol = cf.sol.template as<T>();
      for (const auto& e : cf.el) {
        if (e.m == 0) continue;
        sp.push_back({sol + e.h, (int64_t)(e.m + e.f) * e.m, l, 0});
        if (e.f > 0) sp.push_back({sol + e.wx, (int64_t)e.m * e.f, l, 0});
      }
    }
  if (F.ntop > 0) sp.push_back({F.topinv.p, (int64_t)F.ntop * F.ntop, 1, 0});
  if (sp.empty()) return;
  DevBuf d;
  P.upload(d, sp);
  hipLaunchKernelGGL(k_nonfinite_spans<T>, dim3((unsigned)sp.size()), dim3(WG), 0, P.stream,
                     d.as<FiniteSpan>(), P.d_info);
  IFMM_LAUNCH_CHECK();
  std::vector<int> info;
  P.download(info, P.d_info, 4);
  if (info[INFO_FAC] != -1) {
    P.st.error_level = info[INFO_FAC];
    P.st.error_box = -1;
    fail(IFMM_ERR_NUMERICAL, "non-finite value in the factors (level " + std::to_string(info[INFO_FAC]) +
                                 "; 1 = top system)");
  }
}

void* scratch_address(int device);   // allocation-free solve: address of the device's array (noalloc.hpp)

}  // namespace

// Two events without timing, destroyed with the scope.
struct EventPair {
  hipEvent_t a = nullptr, b = nullptr;
  void create() {
    IFMM_HIP(hipEventCreateWithFlags(&a, hipEventDisableTiming));
    IFMM_HIP(hipEventCreateWithFlags(&b, hipEventDisableTiming));
  }
  ~EventPair() {
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
  }
};

struct ifmm_problem {
  Problem P;
  GmresWork G;
};

extern "C" {

void ifmm_default_options(ifmm_options* opt) {
  if (!opt) return;
  opt->precision = 64;
  opt->leaf_max = 64;
  opt->rank_max = 0;
  opt->sigma0_override = 0.0;
  opt->hbm_budget_bytes = 0;
  opt->stream = nullptr;
  opt->dev_alloc = nullptr;
  opt->dev_free = nullptr;
  opt->alloc_ctx = nullptr;
}

const char* ifmm_strerror(int code) {
  switch (code) {
    case IFMM_OK: return "ok";
    case IFMM_ERR_ARG: return "invalid argument";
    case IFMM_ERR_OOM: return "out of device memory or over the HBM budget";
    case IFMM_ERR_SINGULAR: return "singular pivot block";
    case IFMM_ERR_NUMERICAL: return "non-finite value";
    case IFMM_ERR_STATE: return "call not legal in the handle's state";
    case IFMM_ERR_HIP: return "HIP runtime error";
    case IFMM_ERR_INTERNAL: return "internal error";
    default: return "unknown status";
  }
}

const char* ifmm_last_error(void) { return g_last_error.c_str(); }

int ifmm_build(const double* points, int64_t n, int dim, ifmm_kernel k, int depth, int cheb_order, double eps,
               const ifmm_options* opt, ifmm_handle* out) {
  if (out) *out = nullptr;
  ifmm_problem* h = nullptr;
  const int rc = guarded([&] {
    if (!points || !out) fail(IFMM_ERR_ARG, "null pointer");
    if (n < 1 || n > (int64_t)INT32_MAX) fail(IFMM_ERR_ARG, "n out of range");
    if (dim < 1 || dim > 3) fail(IFMM_ERR_ARG, "dim must be 1, 2 or 3");
    if (cheb_order < 1 || cheb_order > MAXN) fail(IFMM_ERR_ARG, "cheb_order must be in [1, 8]");
    if (!(eps >= 0.0) || !std::isfinite(eps)) fail(IFMM_ERR_ARG, "eps must be finite and >= 0");
    if (k.kind < 0 || k.kind > 3) fail(IFMM_ERR_ARG, "unknown kernel kind");
    if ((k.kind == IFMM_K_GAUSS || k.kind == IFMM_K_PAPER) && !(k.param > 0)) fail(IFMM_ERR_ARG, "kernel parameter must be > 0");
    ifmm_options o;
    ifmm_default_options(&o);
    if (opt) o = *opt;
    if (o.precision != 32 && o.precision != 64) fail(IFMM_ERR_ARG, "precision must be 32 or 64");
    if (!o.dev_alloc != !o.dev_free) fail(IFMM_ERR_ARG, "dev_alloc and dev_free must be given together");
    int q = 1;
    for (int a = 0; a < dim; ++a) q *= cheb_order;
    if (q > SW_MAXC) fail(IFMM_ERR_ARG, "cheb_order^dim above 512");
    h = new ifmm_problem();
    Problem& P = h->P;
    P.mem.budget = o.hbm_budget_bytes;
    {
      const char* kt = std::getenv("IFMM_KTIMING");
      P.kt.on = kt && (kt[0] == '1' || kt[0] == 'm');
      if (kt && kt[0] == 'm') P.kt.mask = (uint32_t)std::strtoul(kt + 1, nullptr, 16);
    }
    P.stream = static_cast<hipStream_t>(o.stream);
    P.alloc.alloc = o.dev_alloc;
    P.alloc.free = o.dev_free;
    P.alloc.ctx = o.alloc_ctx;
    StreamScope ss(P.stream);
    AllocScope as(P.alloc);
    IFMM_HIP(hipGetDevice(&P.device));
    scratch_address(P.device);
    P.n = n;
    P.d = dim;
    P.order = cheb_order;
    P.q = q;
    P.precision = o.precision;
    P.eps = eps;
    P.rank_max = o.rank_max;
    P.kf.kind = k.kind;
    P.kf.param = k.param;
    P.kf.shift = k.diag_shift;
    P.cc.n = cheb_order;
    P.cc.d = dim;
    P.cc.q = q;
    for (int a = 0; a < cheb_order; ++a) P.cc.t[a] = std::cos((2.0 * a + 1.0) * M_PI / (2.0 * cheb_order));
    P.info_buf.alloc(sizeof(int) * 4, &P.mem);
    P.d_info = P.info_buf.as<int>();
    IFMM_HIP(hipMemsetAsync(P.d_info, 0xff, sizeof(int) * 4, P.stream));
    const double t0 = now_ms();
    auto phase = [&](const char* what) {
      if (!progress_on()) return;
      P.sync();
      std::fprintf(stderr, "[ifmm] build: %s done, %.1f s, device %.1f GB\n", what, (now_ms() - t0) * 1e-3,
                   P.mem.cur * 1e-9);
      std::fflush(stderr);
    };
    build_tree(P, points, depth, o.leaf_max);
    phase("tree");
    build_r1(P);
    phase("H2 operators");
    build_r2(P, o.sigma0_override);
    if (progress_on())
      std::fprintf(stderr, "[ifmm] build: sigma_0 %.6e in %d Lanczos steps, %.1f s\n", P.sigma0, P.sigma0_iters,
                   P.st.t_sigma0_ms * 1e-3);
    phase("weighted system");
    P.st.t_build_ms = now_ms() - t0;
    *out = h;
  });
  if (rc != IFMM_OK && h) {   // the build may have left work on the stream
    const hipStream_t st = h->P.stream;
    (void)hipStreamSynchronize(st);
    {
      StreamScope ss(DevPool::idle_stream());
      delete h;
    }
    DevPool::inst().idle(st);
  }
  return rc;
}

}  // extern "C"

namespace {

void factorize_handle(ifmm_handle h) {
  {
    if (!h) fail(IFMM_ERR_ARG, "null handle");
    Problem& P = h->P;
    StreamScope ss(P.stream);
    AllocScope as(P.alloc);
    P.arena_reset();
    P.factorized = false;
    P.fac.reset();
    IFMM_HIP(hipMemsetAsync(P.d_info, 0xff, sizeof(int) * 4, P.stream));
    P.st.error_level = P.st.error_box = -1;
    const double t0 = now_ms();
    reset_finite(P);
    if (P.precision == 64) {
      auto f = std::make_unique<Factors<double>>();
      Factorizer<double> z(P, f->F);
      z.run();
      scan_factors(P, f->F);
      solve_plan(P, f->F, f->S);   // built now, so that a solve only launches
      P.fac = std::move(f);
    } else {
      auto f = std::make_unique<Factors<float>>();
      Factorizer<float> z(P, f->F);
      z.run();
      scan_factors(P, f->F);
      solve_plan(P, f->F, f->S);
      P.fac = std::move(f);
    }
    P.st.t_factor_ms = now_ms() - t0;
    P.factorized = true;
    if (HostProf::on()) {
      P.hprof.print("factorize");
      P.hprof.acc.clear();
    }
  }
}

}  // namespace

extern "C" {

int ifmm_factorize(ifmm_handle h) {
  return guarded([&] { factorize_handle(h); });
}

int ifmm_factorize_batch(ifmm_handle* hs, int count, int nthreads, int* status) {
  std::vector<int> rc;
  int first = IFMM_OK;
  std::string first_msg;
  const int vrc = guarded([&] {
    if (count < 0 || (count > 0 && !hs)) fail(IFMM_ERR_ARG, "null handle array or negative count");
    if (nthreads < 1) fail(IFMM_ERR_ARG, "nthreads must be >= 1");
    for (int i = 0; i < count; ++i) {
      if (!hs[i]) fail(IFMM_ERR_ARG, "null handle in the batch");
      for (int j = 0; j < i; ++j)
        if (hs[j] == hs[i]) fail(IFMM_ERR_ARG, "a handle appears twice in the batch");
    }
    // largest problems first, so that the last ones to finish are small
    std::vector<int> order(count);
    for (int i = 0; i < count; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return hs[a]->P.n > hs[b]->P.n; });
    rc.assign(count, IFMM_OK);
    std::vector<std::string> msg(count);
    std::atomic<int> next{0};
    auto worker = [&] {
      for (;;) {
        const int t = next.fetch_add(1);
        if (t >= count) break;
        const int i = order[t];
        rc[i] = guarded([&] { factorize_handle(hs[i]); });
        if (rc[i] != IFMM_OK) msg[i] = g_last_error;
      }
    };
    const int nt = std::max(1, std::min(nthreads, count));
    std::vector<std::thread> pool;
    for (int w = 1; w < nt; ++w) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    for (int i = 0; i < count; ++i)
      if (rc[i] != IFMM_OK) { first = rc[i]; first_msg = msg[i]; break; }
  });
  if (vrc != IFMM_OK) return vrc;
  if (status)
    for (int i = 0; i < count; ++i) status[i] = rc[i];
  if (first != IFMM_OK) g_last_error = first_msg;
  return first;
}

static void solve_any(Problem& P, const double* b, double* x, int nrhs, int64_t ld) {
  if (P.precision == 64) {
    auto* f = static_cast<Factors<double>*>(P.fac.get());
    solve_impl<double>(P, f->F, f->S, b, x, nrhs, ld);
  } else {
    auto* f = static_cast<Factors<float>*>(P.fac.get());
    solve_impl<float>(P, f->F, f->S, b, x, nrhs, ld);
  }
}

int ifmm_solve(ifmm_handle h, const double* b, double* x, int nrhs, int64_t ld) {
  return guarded([&] {
    if (!h || !b || !x) fail(IFMM_ERR_ARG, "null pointer");
    Problem& P = h->P;
    StreamScope ss(P.stream);
    AllocScope as(P.alloc);
    if (!P.factorized) fail(IFMM_ERR_STATE, "ifmm_solve needs a factorized handle");
    if (nrhs < 1 || ld < P.n) fail(IFMM_ERR_ARG, "nrhs must be >= 1 and ld >= n");
    const double t0 = now_ms();
    reset_finite(P);
    check_finite_vec(P, b, P.n, nrhs, ld, 1);
    solve_any(P, b, x, nrhs, ld);
    check_finite_vec(P, x, P.n, nrhs, ld, 2);
    const int bad = finite_verdict(P);   // synchronises
    P.st.t_last_solve_ms = now_ms() - t0;
    if (bad == 1) fail(IFMM_ERR_NUMERICAL, "b holds a non-finite value");
    if (bad != -1) fail(IFMM_ERR_NUMERICAL, "the solve produced a non-finite value");
  });
}

int ifmm_query_ranks(ifmm_handle h, int level, int* out, int count) {
  return guarded([&] {
    if (!h || !out) fail(IFMM_ERR_ARG, "null pointer");
    Problem& P = h->P;
    if (!P.factorized) fail(IFMM_ERR_STATE, "ifmm_query_ranks needs a factorized handle");
    if (level < 2 || level > P.L) fail(IFMM_ERR_ARG, "level must be in [2, depth]");
    if (count != P.T.lev[level].nb) fail(IFMM_ERR_ARG, "count must equal the occupied boxes of the level");
    const std::vector<int64_t>& y = P.precision == 64
                                        ? static_cast<Factors<double>*>(P.fac.get())->F.sl[level].yoff
                                        : static_cast<Factors<float>*>(P.fac.get())->F.sl[level].yoff;
    for (int i = 0; i < count; ++i) out[i] = (int)(y[i + 1] - y[i]);
  });
}

static void matvec_any(Problem& P, const double* x, double* y, int nrhs, int64_t ld) {
  const int64_t n = P.n;
  P.mv_x.reserve(sizeof(double) * n * nrhs, &P.mem);
  P.mv_y.reserve(sizeof(double) * n * nrhs, &P.mem);
  dim3 g((unsigned)std::max<int64_t>(1, ceil_div(n * nrhs, WG)));
  hipLaunchKernelGGL(k_perm_gather, g, dim3(WG), 0, P.stream, x, ld, P.perm.as<int>(), n, nrhs,
                     P.mv_x.as<double>(), n);
  IFMM_LAUNCH_CHECK();
  P.kset(KF_MATVEC, 0, 0);
  P.kbegin();
  matvec_tree(P, P.mv_x.as<double>(), P.mv_y.as<double>(), nrhs);
  P.kend();
  P.kset(-1);
  hipLaunchKernelGGL(k_perm_scatter, g, dim3(WG), 0, P.stream, (const double*)P.mv_y.as<double>(), n,
                     P.perm.as<int>(), n, nrhs, y, ld);
  IFMM_LAUNCH_CHECK();
}

int ifmm_matvec(ifmm_handle h, const double* x, double* y, int nrhs, int64_t ld) {
  return guarded([&] {
    if (!h || !x || !y) fail(IFMM_ERR_ARG, "null pointer");
    Problem& P = h->P;
    StreamScope ss(P.stream);
    AllocScope as(P.alloc);
    if (nrhs < 1 || ld < P.n) fail(IFMM_ERR_ARG, "nrhs must be >= 1 and ld >= n");
    if (x == y) fail(IFMM_ERR_ARG, "x and y must not alias");
    const double t0 = now_ms();
    matvec_any(P, x, y, nrhs, ld);
    P.sync();
    P.st.t_last_matvec_ms = now_ms() - t0;
  });
}

static int gmres_entry(ifmm_handle op, ifmm_handle prec, const double* b, double* x, int nrhs, int64_t ld,
                       double tol, int maxit, int* iters_out, double* relres_out, double* true_relres_out, bool left) {
  return guarded([&] {
    if (!op || !b || !x) fail(IFMM_ERR_ARG, "null pointer");
    Problem& A = op->P;
    StreamScope ss(A.stream);
    AllocScope as(A.alloc);
    if (prec) {
      if (A.n != prec->P.n) fail(IFMM_ERR_ARG, "op and prec have different sizes");
      if (!prec->P.factorized) fail(IFMM_ERR_STATE, "the preconditioner handle is not factorized");
    }
    if (nrhs < 1 || ld < A.n) fail(IFMM_ERR_ARG, "nrhs must be >= 1 and ld >= n");
    if (maxit < 1 || maxit > 1000) fail(IFMM_ERR_ARG, "maxit must be in [1, 1000]");
    if (!(tol > 0)) fail(IFMM_ERR_ARG, "tol must be > 0");
    {   // x is written before b is read for the last time (exit residual): the two must not overlap
      const char* b0 = reinterpret_cast<const char*>(b);
      const char* x0 = reinterpret_cast<const char*>(x);
      const size_t span = sizeof(double) * (size_t)(ld * (nrhs - 1) + A.n);
      if (b0 < x0 + span && x0 < b0 + span) fail(IFMM_ERR_ARG, "x and b must not overlap");
    }
    reset_finite(A);
    check_finite_vec(A, b, A.n, nrhs, ld, 1);
    if (finite_verdict(A) != -1) fail(IFMM_ERR_NUMERICAL, "b holds a non-finite value");
    // op and prec may live on different streams: every preconditioner solve
    // waits for the work of op's stream that wrote its input, and op's stream
    // waits for the solve before reading its output (device-side, by events)
    EventPair ev;
    if (prec && prec->P.stream != A.stream) ev.create();
    if (prec && prec->P.stream != A.stream) prec->P.sync();
    auto applyA_k = [&](const double* in, double* out, int k) { matvec_any(A, in, out, k, A.n); };
    auto applyM_k = [&](const double* in, double* out, int k) {
      if (!prec) {   // no preconditioner: z = v
        IFMM_HIP(hipMemcpyAsync(out, in, sizeof(double) * (size_t)A.n * k, hipMemcpyDeviceToDevice, A.stream));
        return;
      }
      Problem& M = prec->P;
      if (M.stream != A.stream) {
        IFMM_HIP(hipEventRecord(ev.a, A.stream));
        IFMM_HIP(hipStreamWaitEvent(M.stream, ev.a, 0));
      }
      {
        StreamScope ms(M.stream);   // buffers the solve takes belong to the preconditioner handle
        AllocScope ma(M.alloc);
        solve_any(M, in, out, k, M.n);
      }
      if (M.stream != A.stream) {
        IFMM_HIP(hipEventRecord(ev.b, M.stream));
        IFMM_HIP(hipStreamWaitEvent(A.stream, ev.b, 0));
      }
    };
    auto applyA = [&](const double* in, double* out) { applyA_k(in, out, nrhs); };
    auto applyM = [&](const double* in, double* out) { applyM_k(in, out, nrhs); };
    auto applyA1 = [&](const double* in, double* out) { applyA_k(in, out, 1); };
    auto applyM1 = [&](const double* in, double* out) { applyM_k(in, out, 1); };
    GmresResult r;
    try {
      r = gmres_run(A, op->G, applyA, applyM, b, x, nrhs, ld, tol, maxit, left);
      if (!left) gmres_restart_columns(A, op->G, applyA1, applyM1, b, x, nrhs, ld, tol, maxit, r);
    } catch (...) {
      (void)hipStreamSynchronize(A.stream);
      if (prec) (void)hipStreamSynchronize(prec->P.stream);
      op->G.release();
      throw;
    }
    A.sync();
    if (prec && prec->P.stream != A.stream) prec->P.sync();
    op->G.release();   // the Krylov storage is not kept between calls
    A.st.gmres_iters = r.iters;
    A.st.gmres_relres = r.relres;
    A.st.gmres_restarts = r.restarts;
    if (iters_out) *iters_out = r.iters;
    if (relres_out) *relres_out = r.relres;
    if (true_relres_out) *true_relres_out = r.true_relres;
  });
}

int ifmm_gmres(ifmm_handle op, ifmm_handle prec, const double* b, double* x, int nrhs, int64_t ld, double tol,
               int maxit, int* iters_out, double* relres_out) {
  return gmres_entry(op, prec, b, x, nrhs, ld, tol, maxit, iters_out, relres_out, nullptr, false);
}

int ifmm_gmres_left(ifmm_handle op, ifmm_handle prec, const double* b, double* x, int nrhs, int64_t ld, double tol,
                    int maxit, int* iters_out, double* relres_out, double* true_relres_out) {
  return gmres_entry(op, prec, b, x, nrhs, ld, tol, maxit, iters_out, relres_out, true_relres_out, true);
}

int ifmm_query(ifmm_handle h, ifmm_stats* s) {
  return guarded([&] {
    if (!h || !s) fail(IFMM_ERR_ARG, "null pointer");
    Problem& P = h->P;
    P.st.n = P.n;
    P.st.dim = P.d;
    P.st.depth = P.L;
    P.st.cheb_order = P.order;
    P.st.precision = P.precision;
    P.st.eps = P.eps;
    P.st.sigma0 = P.sigma0;
    P.st.tau = P.tau;
    P.st.levels = P.L - 1;
    for (int l = 0; l <= P.L && l < 32; ++l) P.st.boxes[l] = l < (int)P.T.lev.size() ? P.T.lev[l].nb : 0;
    P.st.device_bytes = P.mem.cur;
    P.st.device_bytes_peak = P.mem.peak;
    P.sync();
    P.kt.collect();
    for (int f = 0; f < KF_COUNT && f < 24; ++f) {
      P.st.kfam_ms[f] = P.kt.ms[f];
      P.st.kfam_flops[f] = P.kt.flops[f];
      P.st.kfam_bytes[f] = P.kt.bytes[f];
      P.st.kfam_launches[f] = P.kt.launches[f];
    }
    *s = P.st;
  });
}

int ifmm_destroy(ifmm_handle h) {
  return guarded([&] {
    if (!h) return;
    const hipStream_t st = h->P.stream;
    (void)hipStreamSynchronize(st);
    {
      StreamScope ss(DevPool::idle_stream());   // the stream is idle: the blocks may serve any stream
      delete h;
    }
    DevPool::inst().idle(st);
    if (trace_on())
      std::fprintf(stderr, "[ifmm-trace] hipMalloc %lld calls %.1f ms, hipFree %.1f ms (process totals)\n",
                   (long long)AllocClock::calls.load(), AllocClock::ns_malloc.load() * 1e-6,
                   AllocClock::ns_free.load() * 1e-6);
  });
}

}  // extern "C"

#include "noalloc.hpp"
