// Non-restarted GMRES in float64 (Sec. 3.2): products with the H2 matvec, the
// IFMM factorization as preconditioner, classical Gram-Schmidt with one
// re-orthogonalisation, x0 = 0, residuals recomputed at exit.
//  - right preconditioning (the paper's default): GMRES on A P^-1 y = b with
//    flexible storage of the preconditioned directions Z_k = P^-1 v_k, x = Z y;
//    the monitored residual is the true one, ||b - A x|| / ||b||;
//  - left preconditioning (App. B): GMRES on P^-1 A x = P^-1 b, x = V y; the
//    monitored residual is ||P^-1 (b - A x)|| / ||P^-1 b||.
// Every column of the right-hand side block is an independent GMRES run; all
// columns share each matvec and each preconditioner solve.
#pragma once

#include <functional>

#include "solve.hpp"

namespace ifmm {

constexpr int DOT_CHUNK = WG * 64;

// part[(pair) * nch + chunk] = partial of sum_t A[j, c, t] * B[c, t], pair = j * nrhs + c
__global__ void k_dots(const double* __restrict__ A, const double* __restrict__ B, int64_t n, int nrhs, int npairs,
                       int nch, double* __restrict__ part) {
  const int pair = blockIdx.x;
  const int ch = blockIdx.y;
  if (pair >= npairs) return;
  const int c = pair % nrhs;
  const double* a = A + (int64_t)pair * n;
  const double* b = B + (int64_t)c * n;
  __shared__ double sh[WG / WAVE];
  double s = 0;
  const int64_t e0 = (int64_t)ch * DOT_CHUNK;
  const int64_t e1 = e0 + DOT_CHUNK < n ? e0 + DOT_CHUNK : n;
  for (int64_t t = e0 + threadIdx.x; t < e1; t += WG) s += a[t] * b[t];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[(int64_t)pair * nch + ch] = s;
}

__global__ void k_reduce_parts(const double* __restrict__ part, int npairs, int nch, double* __restrict__ out) {
  const int p = blockIdx.x * WG + threadIdx.x;
  if (p >= npairs) return;
  double s = 0;
  for (int c = 0; c < nch; ++c) s += part[(int64_t)p * nch + c];
  out[p] = s;
}

// w[c] -= sum_{j < k1} V[j, c] h[j, c]
__global__ void k_sub_comb(const double* __restrict__ V, const double* __restrict__ h, int k1, int64_t n, int nrhs,
                           double* __restrict__ w) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t t = e % n;
  const int c = (int)(e / n);
  double s = 0;
  for (int j = 0; j < k1; ++j) s += V[((int64_t)j * nrhs + c) * n + t] * h[j * nrhs + c];
  w[(int64_t)c * n + t] -= s;
}

// dst[c] = src[c] * a[c]
__global__ void k_colscale(const double* __restrict__ src, const double* __restrict__ a, int64_t n, int nrhs,
                           double* __restrict__ dst) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n * nrhs) return;
  dst[e] = src[e] * a[e / n];
}

// x[c] = sum_{j < kc} Z[j, c] y[c, j]   (x with leading dimension ld)
__global__ void k_combine(const double* __restrict__ Z, const double* __restrict__ y, const int* __restrict__ kc,
                          int maxk, int64_t n, int nrhs, double* __restrict__ x, int64_t ld) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t t = e % n;
  const int c = (int)(e / n);
  double s = 0;
  for (int j = 0; j < kc[c]; ++j) s += Z[((int64_t)j * nrhs + c) * n + t] * y[(int64_t)c * maxk + j];
  x[t + (int64_t)c * ld] = s;
}

// x += d (n entries)
__global__ void k_add(double* __restrict__ x, const double* __restrict__ d, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e < n) x[e] += d[e];
}

// r -= w (both n x nrhs, leading dimension n)
__global__ void k_sub(double* __restrict__ r, const double* __restrict__ w, int64_t nv) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e < nv) r[e] -= w[e];
}

__global__ void k_copy_ld(const double* __restrict__ src, int64_t lds, int64_t n, int nrhs, double* __restrict__ dst,
                          int64_t ldd, double a) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t t = e % n;
  const int c = (int)(e / n);
  dst[t + (int64_t)c * ldd] = a * src[t + (int64_t)c * lds];
}

struct GmresResult {
  int iters = 0;
  double relres = 0;        // monitored residual at exit (max over columns)
  double true_relres = 0;   // ||b - A x|| / ||b|| at exit (max over columns)
  std::vector<int> iters_col;       // per column
  std::vector<double> true_col;     // per column ||b - A x|| / ||b||
  std::vector<double> bnorm;        // per column ||b||
  int restarts = 0;                 // column restarts from the true residual
};

struct GmresWork {
  DevBuf V, Z, w, part, dots, hbuf, scal, y, kc, r;
  void release() {
    for (DevBuf* b : {&V, &Z, &w, &part, &dots, &hbuf, &scal, &y, &kc, &r}) b->release();
  }
};

// Grow b to hold at least `need` bytes, keeping its first `used` bytes
// (stream-ordered copy); capacity doubles, up to `cap` bytes.
inline void grow_keep(Problem& P, DevBuf& b, size_t need, size_t used, size_t cap) {
  if (need <= b.bytes) return;
  DevBuf nb;
  nb.alloc(std::min(cap, std::max(need, 2 * b.bytes)), &P.mem);
  if (used > 0) IFMM_HIP(hipMemcpyAsync(nb.p, b.p, used, hipMemcpyDeviceToDevice, P.stream));
  b = std::move(nb);
}

// apply_A(x, y): y = A x (both n x nrhs, ld n); apply_M(x, y): y = M^-1 x.
// left selects left preconditioning (no Z storage).
inline GmresResult gmres_run(Problem& P, GmresWork& G, const std::function<void(const double*, double*)>& apply_A,
                             const std::function<void(const double*, double*)>& apply_M, const double* b, double* x,
                             int nrhs, int64_t ld, double tol, int maxit, bool left = false) {
  const int64_t n = P.n;
  const int64_t nv = n * nrhs;
  // Krylov storage grows with the iterations (a few vectors first), so a call
  // that converges early never holds maxit + 1 vectors
  const size_t vb = sizeof(double) * (size_t)nv;
  grow_keep(P, G.V, vb * (size_t)std::min(maxit + 1, 8), 0, vb * (size_t)(maxit + 1));
  if (!left) grow_keep(P, G.Z, vb * (size_t)std::min(maxit, 8), 0, vb * (size_t)maxit);
  G.w.reserve(sizeof(double) * nv, &P.mem);
  G.r.reserve(sizeof(double) * nv, &P.mem);
  const int nch = (int)std::max<int64_t>(1, ceil_div(n, DOT_CHUNK));
  G.part.reserve(sizeof(double) * (int64_t)(maxit + 1) * nrhs * nch, &P.mem);
  G.dots.reserve(sizeof(double) * (int64_t)(maxit + 1) * nrhs, &P.mem);
  G.scal.reserve(sizeof(double) * nrhs, &P.mem);
  double* V = G.V.as<double>();
  double* Z = G.Z.as<double>();
  double* w = G.w.as<double>();
  dim3 gv((unsigned)std::max<int64_t>(1, ceil_div(nv, WG)));
  auto dots = [&](const double* A, int npairs, const double* B, std::vector<double>& out) {
    hipLaunchKernelGGL(k_dots, dim3(npairs, nch), dim3(WG), 0, P.stream, A, B, n, nrhs, npairs, nch,
                       G.part.as<double>());
    hipLaunchKernelGGL(k_reduce_parts, dim3((unsigned)ceil_div(npairs, WG)), dim3(WG), 0, P.stream,
                       (const double*)G.part.as<double>(), npairs, nch, G.dots.as<double>());
    IFMM_LAUNCH_CHECK();
    P.download(out, G.dots.p, (size_t)npairs);
  };
  auto setscal = [&](const std::vector<double>& s) {
    void* h = P.stage.get(sizeof(double) * nrhs);
    std::memcpy(h, s.data(), sizeof(double) * nrhs);
    IFMM_HIP(hipMemcpyAsync(G.scal.p, h, sizeof(double) * nrhs, hipMemcpyHostToDevice, P.stream));
    P.sync();
  };
  // v0 = r0 / ||r0|| with r0 = b (right) or P^-1 b (left)
  std::vector<double> beta, bnorm;
  if (left) {
    hipLaunchKernelGGL(k_copy_ld, gv, dim3(WG), 0, P.stream, b, ld, n, nrhs, G.r.as<double>(), n, 1.0);
    IFMM_LAUNCH_CHECK();
    dots(G.r.as<double>(), nrhs, G.r.as<double>(), bnorm);
    apply_M(G.r.as<double>(), w);
  } else {
    hipLaunchKernelGGL(k_copy_ld, gv, dim3(WG), 0, P.stream, b, ld, n, nrhs, w, n, 1.0);
    IFMM_LAUNCH_CHECK();
  }
  dots(w, nrhs, w, beta);
  for (auto& x : beta) x = std::sqrt(x);
  if (!left) bnorm = beta;
  else
    for (auto& x : bnorm) x = std::sqrt(x);
  std::vector<double> inv(nrhs);
  for (int c = 0; c < nrhs; ++c) inv[c] = beta[c] > 0 ? 1.0 / beta[c] : 0.0;
  setscal(inv);
  hipLaunchKernelGGL(k_colscale, gv, dim3(WG), 0, P.stream, (const double*)w, G.scal.as<double>(), n, nrhs, V);
  IFMM_LAUNCH_CHECK();
  std::vector<std::vector<double>> H(nrhs, std::vector<double>((size_t)(maxit + 1) * maxit, 0.0));
  std::vector<std::vector<double>> cs(nrhs, std::vector<double>(maxit, 0.0)), sn = cs;
  std::vector<std::vector<double>> g(nrhs, std::vector<double>(maxit + 1, 0.0));
  std::vector<int> kdone(nrhs, 0);
  std::vector<char> active(nrhs, 1);
  for (int c = 0; c < nrhs; ++c) {
    g[c][0] = beta[c];
    if (beta[c] == 0) active[c] = 0;
  }
  std::vector<double> hk, h2, nrm;
  int k = 0;
  for (k = 0; k < maxit; ++k) {
    bool any = false;
    for (int c = 0; c < nrhs; ++c) any = any || active[c];
    if (!any) break;
    grow_keep(P, G.V, vb * (size_t)(k + 2), vb * (size_t)(k + 1), vb * (size_t)(maxit + 1));
    V = G.V.as<double>();
    if (!left) {
      grow_keep(P, G.Z, vb * (size_t)(k + 1), vb * (size_t)k, vb * (size_t)maxit);
      Z = G.Z.as<double>();
    }
    double* vk = V + (int64_t)k * nv;
    if (left) {   // w = P^-1 A v_k
      apply_A(vk, G.r.as<double>());
      apply_M(G.r.as<double>(), w);
    } else {      // z_k = P^-1 v_k, w = A z_k
      double* zk = Z + (int64_t)k * nv;
      apply_M(vk, zk);
      apply_A(zk, w);
    }
    // CGS2
    std::vector<double> h((size_t)(k + 2) * nrhs, 0.0);
    for (int pass = 0; pass < 2; ++pass) {
      dots(V, (k + 1) * nrhs, w, hk);
      for (size_t t = 0; t < hk.size(); ++t) h[t] += hk[t];
      G.hbuf.reserve(sizeof(double) * hk.size(), &P.mem);
      void* hh = P.stage.get(sizeof(double) * hk.size());
      std::memcpy(hh, hk.data(), sizeof(double) * hk.size());
      IFMM_HIP(hipMemcpyAsync(G.hbuf.p, hh, sizeof(double) * hk.size(), hipMemcpyHostToDevice, P.stream));
      P.sync();
      hipLaunchKernelGGL(k_sub_comb, gv, dim3(WG), 0, P.stream, (const double*)V, G.hbuf.as<double>(), k + 1, n,
                         nrhs, w);
      IFMM_LAUNCH_CHECK();
    }
    dots(w, nrhs, w, nrm);
    std::vector<double> sc(nrhs, 0.0);
    for (int c = 0; c < nrhs; ++c) {
      const double hn = std::sqrt(nrm[c]);
      h[(size_t)(k + 1) * nrhs + c] = hn;
      sc[c] = (active[c] && hn > 0) ? 1.0 / hn : 0.0;
    }
    setscal(sc);
    hipLaunchKernelGGL(k_colscale, gv, dim3(WG), 0, P.stream, (const double*)w, G.scal.as<double>(), n, nrhs,
                       V + (int64_t)(k + 1) * nv);
    IFMM_LAUNCH_CHECK();
    for (int c = 0; c < nrhs; ++c) {
      if (!active[c]) continue;
      std::vector<double> col(k + 2);
      for (int j = 0; j <= k + 1; ++j) col[j] = h[(size_t)j * nrhs + c];
      for (int j = 0; j < k; ++j) {
        const double t = cs[c][j] * col[j] + sn[c][j] * col[j + 1];
        col[j + 1] = -sn[c][j] * col[j] + cs[c][j] * col[j + 1];
        col[j] = t;
      }
      const double den = std::hypot(col[k], col[k + 1]);
      cs[c][k] = den > 0 ? col[k] / den : 1.0;
      sn[c][k] = den > 0 ? col[k + 1] / den : 0.0;
      col[k] = den;
      col[k + 1] = 0;
      for (int j = 0; j <= k + 1; ++j) H[c][(size_t)j * maxit + k] = col[j];
      g[c][k + 1] = -sn[c][k] * g[c][k];
      g[c][k] = cs[c][k] * g[c][k];
      kdone[c] = k + 1;
      if (std::fabs(g[c][k + 1]) <= tol * beta[c] || den == 0) active[c] = 0;
    }
  }
  // y = H^-1 g per column (upper triangular), x = Z y
  int maxk = 1;
  for (int c = 0; c < nrhs; ++c) maxk = std::max(maxk, kdone[c]);
  std::vector<double> Y((size_t)maxk * nrhs, 0.0);
  for (int c = 0; c < nrhs; ++c) {
    const int kc = kdone[c];
    for (int i = kc - 1; i >= 0; --i) {
      double s = g[c][i];
      for (int j = i + 1; j < kc; ++j) s -= H[c][(size_t)i * maxit + j] * Y[(size_t)c * maxk + j];
      const double dd = H[c][(size_t)i * maxit + i];
      Y[(size_t)c * maxk + i] = dd != 0 ? s / dd : 0.0;
    }
  }
  P.upload(G.y, Y);
  P.upload(G.kc, kdone);
  hipLaunchKernelGGL(k_combine, gv, dim3(WG), 0, P.stream, (const double*)(left ? V : Z), G.y.as<double>(),
                     G.kc.as<int>(), maxk, n, nrhs, x, ld);
  IFMM_LAUNCH_CHECK();
  // true residual r = b - A x
  hipLaunchKernelGGL(k_copy_ld, gv, dim3(WG), 0, P.stream, x, ld, n, nrhs, G.r.as<double>(), n, 1.0);
  IFMM_LAUNCH_CHECK();
  apply_A(G.r.as<double>(), w);
  hipLaunchKernelGGL(k_copy_ld, gv, dim3(WG), 0, P.stream, b, ld, n, nrhs, G.r.as<double>(), n, 1.0);
  hipLaunchKernelGGL(k_sub, gv, dim3(WG), 0, P.stream, G.r.as<double>(), (const double*)w, nv);
  IFMM_LAUNCH_CHECK();
  GmresResult res;
  std::vector<double> rn;
  dots(G.r.as<double>(), nrhs, G.r.as<double>(), rn);
  res.true_col.assign(nrhs, 0.0);
  res.bnorm = bnorm;
  for (int c = 0; c < nrhs; ++c)
    if (bnorm[c] > 0) {
      res.true_col[c] = std::sqrt(rn[c]) / bnorm[c];
      res.true_relres = std::max(res.true_relres, res.true_col[c]);
    }
  if (left) {   // preconditioned residual P^-1 (b - A x)
    apply_M(G.r.as<double>(), w);
    dots(w, nrhs, w, rn);
    for (int c = 0; c < nrhs; ++c)
      if (beta[c] > 0) res.relres = std::max(res.relres, std::sqrt(rn[c]) / beta[c]);
  } else {
    res.relres = res.true_relres;
  }
  res.iters = 0;
  res.iters_col = kdone;
  for (int c = 0; c < nrhs; ++c) res.iters = std::max(res.iters, kdone[c]);
  return res;
}

// Right preconditioning only. A column whose monitored residual met tol while
// its true residual, recomputed at exit, did not (rounding in the Arnoldi
// recurrence and in x = Z y) is restarted from that residual: GMRES on
// A d = b - A x with at most GMRES_RESTART_ITERS of the iterations the column
// has left, then x += d and the true residual again; at most `passes`
// restarts, and none after a restart that took less than 1% off the true
// residual (the residual is then at the rounding floor of the product itself,
// where more iterations only cost time). Columns are refined one at a time
// (one-column runs), so a column's result does not depend on the others.
// On entry G.r holds b - A x (n x nrhs, leading dimension n), as gmres_run
// leaves it; res is updated.
constexpr int GMRES_RESTART_ITERS = 10;
inline void gmres_restart_columns(Problem& P, GmresWork& G, const std::function<void(const double*, double*)>& A1,
                                  const std::function<void(const double*, double*)>& M1, const double* b, double* x,
                                  int nrhs, int64_t ld, double tol, int maxit, GmresResult& res, int passes = 3) {
  const int64_t n = P.n;
  std::vector<char> stalled(nrhs, 0);
  auto needs = [&](int c) { return !stalled[c] && res.true_col[c] > tol && res.iters_col[c] < maxit; };
  bool any = false;
  for (int c = 0; c < nrhs; ++c) any = any || needs(c);
  if (!any) return;
  DevBuf R, D, part, dot;   // residual columns (one-column runs overwrite G.r), correction, norm partials
  R.alloc(sizeof(double) * (size_t)(n * nrhs), &P.mem);
  D.alloc(sizeof(double) * (size_t)n, &P.mem);
  const int nch = (int)std::max<int64_t>(1, ceil_div(n, DOT_CHUNK));
  part.alloc(sizeof(double) * (size_t)nch, &P.mem);
  dot.alloc(sizeof(double), &P.mem);
  IFMM_HIP(hipMemcpyAsync(R.p, G.r.p, sizeof(double) * (size_t)(n * nrhs), hipMemcpyDeviceToDevice, P.stream));
  const dim3 g1((unsigned)std::max<int64_t>(1, ceil_div(n, WG)));
  for (int pass = 0; pass < passes; ++pass) {
    bool ran = false;
    for (int c = 0; c < nrhs; ++c) {
      if (!needs(c)) continue;
      ran = true;
      ++res.restarts;
      double* rc = R.as<double>() + (int64_t)c * n;
      double* xc = x + (int64_t)c * ld;
      const double before = res.true_col[c];
      const GmresResult in = gmres_run(P, G, A1, M1, rc, D.as<double>(), 1, n, tol / before,
                                       std::min(maxit - res.iters_col[c], GMRES_RESTART_ITERS));
      res.iters_col[c] += std::max(1, in.iters);
      hipLaunchKernelGGL(k_add, g1, dim3(WG), 0, P.stream, xc, (const double*)D.as<double>(), n);
      IFMM_LAUNCH_CHECK();
      // r_c = b_c - A x_c, ||r_c|| / ||b_c||
      A1(xc, D.as<double>());
      hipLaunchKernelGGL(k_copy_ld, g1, dim3(WG), 0, P.stream, b + (int64_t)c * ld, ld, n, 1, rc, n, 1.0);
      hipLaunchKernelGGL(k_sub, g1, dim3(WG), 0, P.stream, rc, (const double*)D.as<double>(), n);
      hipLaunchKernelGGL(k_dots, dim3(1, nch), dim3(WG), 0, P.stream, (const double*)rc, (const double*)rc, n, 1, 1,
                         nch, part.as<double>());
      hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(WG), 0, P.stream, (const double*)part.as<double>(), 1, nch,
                         dot.as<double>());
      IFMM_LAUNCH_CHECK();
      std::vector<double> rn;
      P.download(rn, dot.p, 1);
      res.true_col[c] = res.bnorm[c] > 0 ? std::sqrt(rn[0]) / res.bnorm[c] : 0.0;
      if (res.true_col[c] > 0.99 * before) stalled[c] = 1;
    }
    if (!ran) break;
  }
  res.iters = 0;
  res.true_relres = 0;
  for (int c = 0; c < nrhs; ++c) {
    res.iters = std::max(res.iters, res.iters_col[c]);
    res.true_relres = std::max(res.true_relres, res.true_col[c]);
  }
  res.relres = res.true_relres;
}

}  // namespace ifmm
