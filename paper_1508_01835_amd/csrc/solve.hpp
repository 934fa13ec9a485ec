// Substitution with the stored factors (Alg. 1, solve for y^(2) and
// substitute back down the tree): forward over the eliminations in their
// order, c_P = E_PP^-1 b_P and b_F -= E_FP c_P; the dense top solve; backward
// in reverse order, x_P = c_P - W x_F. Memory bound: every factor block is
// read once per call for all right-hand sides together.
#pragma once

#include "factor.hpp"

namespace ifmm {

struct SolveDesc {
  const void* lu;
  const int* piv;
  const void* w;
  const void* efp;
  int m, r, p, f, nF, F0;
  int64_t xoff;    // offset of x~_i in the level's vector
  int64_t coff;    // offset of c_P in the c store, in units of nrhs
};

struct SolveNode {
  int type, dim, off, pad;
  int64_t voff;    // offset in the level's x~ vector (type 0) or in the y vector (type 1)
};

// c_P = [b(x~_i); 0]
template <class T>
__global__ void k_fwd_init(const SolveDesc* __restrict__ ds, const T* __restrict__ X, int64_t ldx, int nrhs,
                           T* __restrict__ C) {
  const SolveDesc d = ds[blockIdx.x];
  T* c = C + d.coff * nrhs;
  for (int t = threadIdx.x; t < d.p * nrhs; t += WG) {
    const int i = t % d.p, rr = t / d.p;
    c[t] = i < d.m ? X[d.xoff + i + (int64_t)rr * ldx] : (T)0;
  }
}

// b_F -= E_FP c_P, one block per (elimination, node of F).
template <class T>
__global__ void k_fwd_update(const SolveDesc* __restrict__ ds, const SolveNode* __restrict__ ns,
                             T* __restrict__ X, int64_t ldx, T* __restrict__ Y, int64_t ldy, int nrhs,
                             const T* __restrict__ C) {
  const SolveDesc d = ds[blockIdx.x];
  if ((int)blockIdx.y >= d.nF) return;
  const SolveNode n = ns[d.F0 + blockIdx.y];
  const T* efp = static_cast<const T*>(d.efp);
  const T* c = C + d.coff * nrhs;
  T* dst = n.type == 0 ? X + n.voff : Y + n.voff;
  const int64_t ld = n.type == 0 ? ldx : ldy;
  for (int t = threadIdx.x; t < n.dim * nrhs; t += WG) {
    const int i = t % n.dim, rr = t / n.dim;
    T s = 0;
    for (int k = 0; k < d.p; ++k) s += efp[(n.off + i) + (int64_t)k * d.f] * c[k + (int64_t)rr * d.p];
    dst[i + (int64_t)rr * ld] -= s;
  }
}

// x~_i = (c_P - W x_F)[0:m]
template <class T>
__global__ void k_bwd(const SolveDesc* __restrict__ ds, const SolveNode* __restrict__ ns, T* __restrict__ X,
                      int64_t ldx, const T* __restrict__ Y, int64_t ldy, int nrhs, const T* __restrict__ C) {
  const SolveDesc d = ds[blockIdx.x];
  const T* w = static_cast<const T*>(d.w);
  const T* c = C + d.coff * nrhs;
  for (int t = threadIdx.x; t < d.m * nrhs; t += WG) {
    const int i = t % d.m, rr = t / d.m;
    T s = c[i + (int64_t)rr * d.p];
    for (int a = 0; a < d.nF; ++a) {
      const SolveNode n = ns[d.F0 + a];
      const T* src = n.type == 0 ? X + n.voff + (int64_t)rr * ldx : Y + n.voff + (int64_t)rr * ldy;
      for (int u = 0; u < n.dim; ++u) s -= w[i + (int64_t)(n.off + u) * d.p] * src[u];
    }
    X[d.xoff + i + (int64_t)rr * ldx] = s;
  }
}

template <class Ts, class Td>
__global__ void k_perm_convert(const Ts* __restrict__ src, int64_t lds, const int* __restrict__ perm, int64_t n,
                               int nrhs, Td* __restrict__ dst, int64_t ldd, int to_tree) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t t = e % n;
  const int r = (int)(e / n);
  if (to_tree) dst[t + r * ldd] = (Td)src[(int64_t)perm[t] + r * lds];
  else dst[(int64_t)perm[t] + r * ldd] = (Td)src[t + r * lds];
}

template <class T>
struct SolvePlan {
  // per level, per class: device descriptors
  struct Cls {
    DevBuf d, nodes;
    std::vector<SolveDesc> h;
    int n = 0, maxF = 0;
  };
  std::vector<std::vector<Cls>> cls;
  std::vector<int64_t> M;        // vector size per level (level 1 = the top vector)
  int64_t cstore = 0;
  double factor_elems = 0;       // elements of the factors one solve reads
  bool built = false;
};

template <class T>
inline SolvePlan<T>& solve_plan(Problem& P, FactorStore<T>& F, SolvePlan<T>& S) {
  if (S.built) return S;
  const int L = P.L;
  S.cls.clear();
  S.cls.resize(L + 1);
  S.M.assign(L + 1, 0);
  int64_t co = 0;
  for (int l = L; l >= 2; --l) {
    const SolveLevel<T>& sl = F.sl[l];
    S.M[l] = sl.M;
    S.M[l - 1] = sl.Mup;
    S.cls[l].resize(F.cls[l].size());
    for (size_t c = 0; c < F.cls[l].size(); ++c) {
      const ClassFactors<T>& cf = F.cls[l][c];
      auto& sc = S.cls[l][c];
      if (cf.el.empty()) continue;
      std::vector<SolveNode> nodes;
      for (const auto& e : cf.el) {
        SolveDesc d{};
        d.lu = cf.fac.template as<T>() + e.lu;
        d.piv = cf.piv.template as<int>() + e.piv;
        d.w = cf.fac.template as<T>() + e.w;
        d.efp = cf.fac.template as<T>() + e.efp;
        d.m = e.m; d.r = e.r; d.p = e.p; d.f = e.f; d.nF = e.nF;
        d.F0 = (int)nodes.size();
        d.xoff = sl.xoff[e.box];
        d.coff = co;
        co += e.p;
        S.factor_elems += (double)e.p * e.p + 2.0 * e.p * e.f;
        for (int a = 0; a < e.nF; ++a) {
          const FNode& n = cf.F[e.F0 + a];
          SolveNode sn{};
          sn.type = n.type;
          sn.dim = n.dim;
          sn.off = n.off;
          sn.voff = n.type == 0 ? sl.xoff[n.box] : sl.yoff[n.box];
          nodes.push_back(sn);
        }
        sc.maxF = std::max(sc.maxF, e.nF);
        sc.h.push_back(d);
      }
      sc.n = (int)sc.h.size();
      P.upload(sc.d, sc.h);
      P.upload(sc.nodes, nodes);
    }
  }
  S.cstore = co;
  S.built = true;
  return S;
}

// x = IFMM^-1 b, b and x in caller order (float64), nrhs columns.
template <class T>
inline void solve_impl(Problem& P, FactorStore<T>& F, SolvePlan<T>& S, const double* b, double* x, int nrhs,
                       int64_t ld) {
  const int L = P.L;
  solve_plan(P, F, S);
  {
    const double fe = S.factor_elems + (double)F.ntop * F.ntop;
    P.kset(KF_SOLVE, 2.0 * fe * nrhs, fe * sizeof(T));
  }
  // vectors: level L..1
  std::vector<int64_t> base(L + 1, 0);
  int64_t tot = 0;
  for (int l = L; l >= 1; --l) {
    base[l] = tot;
    tot += S.M[l] * nrhs;
  }
  F.sx.reserve(sizeof(T) * std::max<int64_t>(tot, 1), &P.mem);
  F.sc.reserve(sizeof(T) * std::max<int64_t>(S.cstore * nrhs, 1), &P.mem);
  T* X = F.sx.template as<T>();
  T* C = F.sc.template as<T>();
  IFMM_HIP(hipMemsetAsync(X, 0, sizeof(T) * std::max<int64_t>(tot, 1), P.stream));
  dim3 g((unsigned)std::max<int64_t>(1, ceil_div(P.n * nrhs, WG)));
  hipLaunchKernelGGL((k_perm_convert<double, T>), g, dim3(WG), 0, P.stream, b, ld, P.perm.template as<int>(), P.n, nrhs,
                     X + base[L], P.n, 1);
  IFMM_LAUNCH_CHECK();
  DevBuf scr;
  for (int l = L; l >= 2; --l) {
    T* Xl = X + base[l];
    T* Yl = X + base[l - 1];
    for (auto& sc : S.cls[l]) {
      if (!sc.n) continue;
      P.kbegin();
      hipLaunchKernelGGL(k_fwd_init<T>, dim3(sc.n), dim3(WG), 0, P.stream, sc.d.template as<SolveDesc>(), (const T*)Xl,
                         S.M[l], nrhs, C);
      IFMM_LAUNCH_CHECK();
      P.kend();
      std::vector<TrsJob> jobs;
      for (const auto& d : sc.h)
        if (d.p > 0) jobs.push_back({d.lu, d.piv, C + d.coff * nrhs, d.p, d.p, nrhs, d.p});
      lu_solve_blocked<T>(P, jobs, F.lus);
      P.kbegin();
      hipLaunchKernelGGL(k_fwd_update<T>, dim3(sc.n, std::max(sc.maxF, 1)), dim3(WG), 0, P.stream,
                         sc.d.template as<SolveDesc>(), sc.nodes.template as<SolveNode>(), Xl, S.M[l], Yl, S.M[l - 1], nrhs,
                         (const T*)C);
      IFMM_LAUNCH_CHECK();
      P.kend();
    }
  }
  if (F.ntop > 0) {
    std::vector<TrsJob> jobs(1);
    jobs[0] = {F.top.template as<T>(), F.toppiv.template as<int>(), X + base[1], F.ntop, F.ntop, nrhs, (int)S.M[1]};
    lu_solve_blocked<T>(P, jobs, F.lus);
  }
  for (int l = 2; l <= L; ++l) {
    T* Xl = X + base[l];
    T* Yl = X + base[l - 1];
    for (int c = (int)S.cls[l].size() - 1; c >= 0; --c) {
      auto& sc = S.cls[l][c];
      if (!sc.n) continue;
      P.kbegin();
      hipLaunchKernelGGL(k_bwd<T>, dim3(sc.n), dim3(WG), 0, P.stream, sc.d.template as<SolveDesc>(),
                         sc.nodes.template as<SolveNode>(), Xl, S.M[l], (const T*)Yl, S.M[l - 1], nrhs, (const T*)C);
      IFMM_LAUNCH_CHECK();
      P.kend();
    }
  }
  hipLaunchKernelGGL((k_perm_convert<T, double>), g, dim3(WG), 0, P.stream, (const T*)(X + base[L]), P.n,
                     P.perm.template as<int>(), P.n, nrhs, x, ld, 0);
  IFMM_LAUNCH_CHECK();
  P.kset(-1);
}

}  // namespace ifmm
