// Level-by-level factorization of E (Alg. 1 and 2, Alg. 3), templated on the
// arithmetic of the factors (float or double).
//
// One level lives in a device pool holding every edge of the graph of E at
// that level: S (x~-x~), U, V, the weights, K (y-y), XY / YX (x~-y fill of
// eliminated neighbours) and the transfers to the parent. Boxes are eliminated
// one colour class (independent set) at a time; each class is a fixed
// sequence of batched launches, planned on the host with exact sizes (one
// device-to-host read of the ranks per class).
#pragma once

#include <thread>

#include "blocked.hpp"
#include "build.hpp"
#include "factor_kernels.hpp"

namespace ifmm {

constexpr double RT_GEMM_WORK = 64.0 * 64 * 64;   // r_j / t_j by batched GEMMs above this kq r m_j
constexpr double CLASS_BYTES = 6.0e9;   // transient bytes of one batch of a colour class (the class is split above)
constexpr int CAP_MAX = 4096;   // largest rank capacity of a box (the basis-change kernels stage r rows in LDS)

// Capacity of y_i (rows of its K edges, columns of U_i / V_i) for a rank k,
// at most the box's x~ size: room for some growth, so that a recompression
// that adds a few directions does not re-lay out the box's edges.
inline int cap_for_rank(int k, int m) { return std::min(m, k + std::max(4, k / 4)); }

template <class T>
struct LevelPool {
  int l = 0, nb = 0, c7 = 0, c3 = 0;
  std::vector<int> m, cap, r, rpar;
  std::vector<int64_t> Kt, St, XYt, YXt, Uo, Vo, SUo, SVo, PUo, PVo;
  std::vector<int> B7;
  // per box, the offset codes of its existing edges K(j, q) (row) and K(q, j)
  // (column), CSR; built on first use, the edge tables of a level are fixed
  std::vector<int> erow_start, erow, ecol_start, ecol;
  DevBuf derow_start, derow, decol_start, decol;
  int64_t size = 0;       // elements of the pool in use (slots are appended; a grown box leaves its old slots)
  int64_t capacity = 0;   // elements allocated
  DevBuf pool;
  DevBuf dm, dcap, dr, drnew, dKt, dB7, dSt, dXYt, dYXt, dUo, dVo, dSUo, dSVo, dPUo, dPVo, drpar, dparent;
  T* P() const { return pool.template as<T>(); }
  LevelView view(const Problem& pb) const {
    LevelView v;
    v.nb = nb; v.d = pb.d; v.c7 = c7; v.c3 = c3; v.haspar = l > 2 ? 1 : 0;
    v.coords = pb.ldev[l].coords.template as<int>();
    v.m = dm.template as<int>(); v.cap = dcap.template as<int>(); v.r = dr.template as<int>(); v.rnew = drnew.template as<int>();
    v.Kt = dKt.template as<int64_t>(); v.B7 = dB7.template as<int>(); v.St = dSt.template as<int64_t>();
    v.XYt = dXYt.template as<int64_t>(); v.YXt = dYXt.template as<int64_t>();
    v.Uo = dUo.template as<int64_t>(); v.Vo = dVo.template as<int64_t>(); v.SUo = dSUo.template as<int64_t>(); v.SVo = dSVo.template as<int64_t>();
    v.PUo = l > 2 ? dPUo.template as<int64_t>() : nullptr; v.PVo = l > 2 ? dPVo.template as<int64_t>() : nullptr;
    v.rpar = l > 2 ? drpar.template as<int>() : nullptr;
    v.parent = l > 2 ? pb.ldev[l].parent.template as<int>() : nullptr;
    return v;
  }
};

// Stored factors of one colour class (read once per solve). With b_P =
// [b(x~_i); 0] (the z rows of the right-hand side stay zero), the
// substitution of one elimination needs only
//   A = (E_PP^-1)[0:m, 0:m], G = E_FP (E_PP^-1)[:, 0:m], W_x = (E_PP^-1 E_PF)[0:m, :]
// forward: c = A b(x~_i), b_F -= G b(x~_i); backward: x~_i = c - W_x x_F.
// H = [A; G] and W_x live in sol; the LU, E_PF and E_FP blocks are transient.
template <class T>
struct ClassFactors {
  DevBuf sol;                  // H and W_x of every elimination
  std::vector<ElimDesc> el;    // h / wx offsets relative to sol
  std::vector<FNode> F;
};

template <class T>
struct SolveLevel {
  std::vector<std::vector<ElimDesc>> el;   // per class, with solve offsets in w/efp fields
  std::vector<std::vector<FNode>> F;
  std::vector<int64_t> xoff;               // x~ offsets at this level (prefix of m)
  std::vector<int64_t> yoff;               // y offsets (prefix of final r) = x~ offsets one level up
  int64_t M = 0, Mup = 0;                  // sizes of the level's x~ vector and y vector
};

template <class T>
struct FactorStore : FactorStoreBase {
  std::vector<std::vector<ClassFactors<T>>> cls;   // by level, by class
  std::vector<SolveLevel<T>> sl;                   // by level
  DevBuf topinv;                                   // inverse of the y^(2) system
  int ntop = 0;
  DevBuf arena, pivs;                              // transient blocks of the class being eliminated
  // scratch reused across calls
  DevBuf work, d1, d2, d3, d4, d5;
  DevBuf rtmp;                                     // redirect: U^T D products of x~-x~ pairs
  DevBuf qcw;                                      // step-wise pivoted QR: norms, pivots, state
  LuScratch lus;
  QrScratch qrs;
};

// --------------------------------------------------------------- fill kernels
template <class T>
__global__ void k_p2p_blocks(const double* __restrict__ pts, const int64_t* __restrict__ leaf_start,
                             const int* __restrict__ nb_start, const int* __restrict__ nbr,
                             const int* __restrict__ coords, int nb, int d, int c3, KernelFn kf,
                             const int64_t* __restrict__ St, T* __restrict__ pool) {
  const int t = blockIdx.x;
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nb_start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int i = lo, j = nbr[t];
  const int64_t si = leaf_start[i], mi = leaf_start[i + 1] - si;
  const int64_t sj = leaf_start[j], mj = leaf_start[j + 1] - sj;
  const int64_t off = St[(int64_t)i * c3 + code3(coords, d, i, j)];
  for (int64_t e = threadIdx.x; e < mi * mj; e += WG) {
    const int64_t a = e % mi, b = e / mi;
    double r2 = 0;
    for (int k = 0; k < d; ++k) {
      const double df = pts[(si + a) * d + k] - pts[(sj + b) * d + k];
      r2 += df * df;
    }
    double v = kappa(kf, sqrt(r2));
    if (si + a == sj + b) v += kf.shift;
    pool[off + a + b * mi] = (T)v;
  }
}

// K(i, j) from the initial operators for every interaction-list pair (ld cap_i).
template <class T>
__global__ void k_kinit(const int* __restrict__ in_start, const int* __restrict__ inter,
                        const int* __restrict__ coords, int nb, int d, int c7, const double* __restrict__ K0,
                        const int64_t* __restrict__ k0off, const int* __restrict__ k0,
                        const int* __restrict__ cap, const int64_t* __restrict__ Kt, T* __restrict__ pool) {
  const int t = blockIdx.x;
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (in_start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int i = lo, j = inter[t];
  const int ki = k0[i], kj = k0[j];
  const int64_t off = Kt[(int64_t)i * c7 + code7(coords, d, i, j)];
  const double* src = K0 + k0off[t];
  const int ld = cap[i];
  for (int e = threadIdx.x; e < ki * kj; e += WG) {
    const int a = e % ki, b = e / ki;
    pool[off + a + (int64_t)b * ld] = (T)src[a + (int64_t)b * ki];
  }
}

// Merge: S(p, q) = [K(c, c')] over the children of p and q (eq. K_merge);
// one block per (p, neighbour q).
template <class T>
__global__ void k_merge_S(const int* __restrict__ nb_start, const int* __restrict__ nbr,
                          const int* __restrict__ pcoords, int nbp, int d, const int* __restrict__ ch_start,
                          const int* __restrict__ ccoords, const int* __restrict__ choff,
                          const int* __restrict__ rc, const int* __restrict__ capc, const int64_t* __restrict__ Ktc,
                          int c7, const T* __restrict__ cpool, const int* __restrict__ mp,
                          const int64_t* __restrict__ Stp, int c3, T* __restrict__ ppool) {
  const int t = blockIdx.x;
  int lo = 0, hi = nbp - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nb_start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int p = lo, qb = nbr[t];
  const int64_t off = Stp[(int64_t)p * c3 + code3(pcoords, d, p, qb)];
  const int ld = mp[p];
  for (int c = ch_start[p]; c < ch_start[p + 1]; ++c)
    for (int c2 = ch_start[qb]; c2 < ch_start[qb + 1]; ++c2) {
      const int code = code7(ccoords, d, c, c2);
      const int64_t ko = code >= 0 ? Ktc[(int64_t)c * c7 + code] : -1;
      const int r1 = rc[c], r2 = rc[c2];
      for (int e = threadIdx.x; e < r1 * r2; e += WG) {
        const int a = e % r1, b = e / r1;
        const T v = ko >= 0 ? cpool[ko + a + (int64_t)b * capc[c]] : (T)0;
        ppool[off + (choff[c] + a) + (int64_t)(choff[c2] + b) * ld] = v;
      }
    }
}

// Merge: U_p = stack PU(c), V_p = stack PV(c) (eqs. U_merge, V_merge).
template <class T>
__global__ void k_merge_UV(const int* __restrict__ ch_start, int nbp, const int* __restrict__ choff,
                           const int* __restrict__ rc, const int* __restrict__ capc,
                           const int64_t* __restrict__ PUc, const int64_t* __restrict__ PVc,
                           const T* __restrict__ cpool, const int* __restrict__ mp, const int* __restrict__ rp,
                           const int64_t* __restrict__ Up, const int64_t* __restrict__ Vp, T* __restrict__ ppool) {
  const int p = blockIdx.x;
  if (p >= nbp) return;
  const int ld = mp[p], cols = rp[p];
  for (int c = ch_start[p]; c < ch_start[p + 1]; ++c) {
    const int r1 = rc[c];
    for (int e = threadIdx.x; e < r1 * cols; e += WG) {
      const int a = e % r1, b = e / r1;
      ppool[Up[p] + (choff[c] + a) + (int64_t)b * ld] = cpool[PUc[c] + a + (int64_t)b * capc[c]];
      ppool[Vp[p] + (choff[c] + a) + (int64_t)b * ld] = cpool[PVc[c] + a + (int64_t)b * capc[c]];
    }
  }
}

// Top: dense system of y^(2) from the level-2 K edges (all pairs are edges).
template <class T>
__global__ void k_top_gather(int nb, const int* __restrict__ coords, int d, int c7, const int* __restrict__ r,
                             const int* __restrict__ cap, const int64_t* __restrict__ Kt,
                             const int64_t* __restrict__ off, int n, const T* __restrict__ pool,
                             T* __restrict__ D) {
  const int t = blockIdx.x;
  const int i = t % nb, j = t / nb;
  const int code = code7(coords, d, i, j);
  const int64_t ko = code >= 0 ? Kt[(int64_t)i * c7 + code] : -1;
  const int ri = r[i], rj = r[j];
  for (int e = threadIdx.x; e < ri * rj; e += WG) {
    const int a = e % ri, b = e / ri;
    D[(off[i] + a) + (off[j] + b) * (int64_t)n] = ko >= 0 ? pool[ko + a + (int64_t)b * cap[i]] : (T)0;
  }
}

// table[upd[2t]] = upd[2t + 1] for every pair t (offset-table updates of grown boxes).
__global__ void k_scatter_offsets(const int64_t* __restrict__ upd, int64_t n, int64_t* __restrict__ table) {
  const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (t < n) table[upd[2 * t]] = upd[2 * t + 1];
}

// ---------------------------------------------------------------- host logic
template <class T>
struct Factorizer {
  Problem& P;
  FactorStore<T>& F;
  double flops_lu = 0, flops_schur = 0, flops_comp = 0, flops_other = 0;
  int64_t factor_elems = 0;
  Factorizer(Problem& p, FactorStore<T>& f) : P(p), F(f) {}

  // Allocate and lay out the pool of level l.
  void layout(LevelPool<T>& L, int l, const std::vector<int>& m, const std::vector<int>& r0) {
    const HLevel& lv = P.T.lev[l];
    const int d = P.d;
    L.l = l;
    L.nb = lv.nb;
    L.c7 = 1;
    L.c3 = 1;
    for (int k = 0; k < d; ++k) { L.c7 *= 7; L.c3 *= 3; }
    L.m = m;
    L.r = r0;
    L.cap.resize(lv.nb);
    for (int i = 0; i < lv.nb; ++i) {
      // sized for the present rank (grown by grow_boxes when a recompression needs more)
      int c = cap_for_rank(r0[i], m[i]);
      if (P.rank_max > 0) c = std::min(c, P.rank_max);
      L.cap[i] = std::max(c, r0[i]);
      if (L.cap[i] > CAP_MAX)
        fail(IFMM_ERR_ARG, "a basis at level " + std::to_string(l) + " needs " + std::to_string(L.cap[i]) +
                               " columns (limit " + std::to_string(CAP_MAX) + ")");
    }
    L.rpar.assign(lv.nb, 0);
    if (l > 2)
      for (int i = 0; i < lv.nb; ++i) L.rpar[i] = P.r2[l - 1].k[lv.parent[i]];
    L.Kt.assign((size_t)lv.nb * L.c7, -1);
    L.B7.assign((size_t)lv.nb * L.c7, -1);
    L.St.assign((size_t)lv.nb * L.c3, -1);
    L.XYt.assign((size_t)lv.nb * L.c3, -1);
    L.YXt.assign((size_t)lv.nb * L.c3, -1);
    L.Uo.resize(lv.nb); L.Vo.resize(lv.nb); L.SUo.resize(lv.nb); L.SVo.resize(lv.nb);
    L.PUo.assign(lv.nb, 0); L.PVo.assign(lv.nb, 0);
    int64_t o = 0;
    auto take = [&](int64_t n) { const int64_t a = o; o += (n + 1) & ~int64_t(1); return a; };
    for (int i = 0; i < lv.nb; ++i) {
      for (int t = lv.nb_start[i]; t < lv.nb_start[i + 1]; ++t) {
        const int j = lv.nbr[t];
        L.St[(size_t)i * L.c3 + offset3(lv, i, j)] = take((int64_t)m[i] * m[j]);
        if (lv.colour[j] < lv.colour[i]) {   // x~_i - y_j fill (j eliminated first)
          L.XYt[(size_t)i * L.c3 + offset3(lv, i, j)] = take((int64_t)m[i] * L.cap[j]);
          L.YXt[(size_t)j * L.c3 + offset3(lv, j, i)] = take((int64_t)L.cap[j] * m[i]);
        }
      }
      L.Uo[i] = take((int64_t)m[i] * L.cap[i]);
      L.Vo[i] = take((int64_t)m[i] * L.cap[i]);
      L.SUo[i] = take(L.cap[i]);
      L.SVo[i] = take(L.cap[i]);
      if (l > 2) {
        L.PUo[i] = take((int64_t)L.cap[i] * L.rpar[i]);
        L.PVo[i] = take((int64_t)L.cap[i] * L.rpar[i]);
      }
      auto addK = [&](int j) {
        const int c = offset7(lv, d, i, j);
        L.Kt[(size_t)i * L.c7 + c] = take((int64_t)L.cap[i] * L.cap[j]);
        L.B7[(size_t)i * L.c7 + c] = j;
      };
      for (int t = lv.nb_start[i]; t < lv.nb_start[i + 1]; ++t) addK(lv.nbr[t]);
      for (int t = lv.in_start[i]; t < lv.in_start[i + 1]; ++t) addK(lv.inter[t]);
    }
    L.size = o;
    L.capacity = std::max<int64_t>(o + o / 8, 2);   // some room for boxes that grow
    L.pool.alloc(sizeof(T) * L.capacity, &P.mem);
    IFMM_HIP(hipMemsetAsync(L.pool.p, 0, sizeof(T) * L.capacity, P.stream));
    P.upload(L.dm, L.m); P.upload(L.dcap, L.cap); P.upload(L.dr, L.r); P.upload(L.drnew, L.r);
    P.upload(L.dKt, L.Kt); P.upload(L.dB7, L.B7); P.upload(L.dSt, L.St); P.upload(L.dXYt, L.XYt);
    P.upload(L.dYXt, L.YXt); P.upload(L.dUo, L.Uo); P.upload(L.dVo, L.Vo); P.upload(L.dSUo, L.SUo);
    P.upload(L.dSVo, L.SVo); P.upload(L.dPUo, L.PUo); P.upload(L.dPVo, L.PVo); P.upload(L.drpar, L.rpar);
  }

  // Give the boxes of `want` (box, new capacity) larger y capacities: new
  // slots for U, V, the weights, the parent transfers and every K edge in
  // which they take part (copied, leading dimensions adjusted), and for the
  // x~-y fill blocks XY / YX of their y (zero: a box that grows is not yet
  // eliminated). Old slots stay unused until the level is released. The pool
  // is reallocated (and copied) when the new slots do not fit.
  void grow_boxes(LevelPool<T>& L, const std::vector<std::pair<int, int>>& want) {
    if (want.empty()) return;
    const HLevel& lv = P.T.lev[L.l];
    std::vector<int> nc = L.cap;
    std::vector<char> g(L.nb, 0);
    for (const auto& w : want) {
      if (w.second > CAP_MAX)
        fail(IFMM_ERR_ARG, "a basis at level " + std::to_string(L.l) + " needs " + std::to_string(w.second) +
                               " columns (limit " + std::to_string(CAP_MAX) + ")");
      if (w.second > nc[w.first]) { nc[w.first] = w.second; g[w.first] = 1; }
    }
    int64_t o = L.size;
    auto take = [&](int64_t n) { const int64_t a = o; o += (n + 1) & ~int64_t(1); return a; };
    struct Mv { int64_t src, dst; int lds, ldd, rows, cols; };
    std::vector<Mv> mv;
    std::vector<std::pair<int64_t, int64_t>> upd7, updxy, updyx;   // (table index, new offset)
    std::vector<int64_t> edges;                                    // row box * c7 + code of every K edge to move
    for (int j = 0; j < L.nb; ++j) {
      if (!g[j]) continue;
      const int co = L.cap[j], cn = nc[j], mj = L.m[j];
      int64_t a = take((int64_t)mj * cn);
      mv.push_back({L.Uo[j], a, mj, mj, mj, co}); L.Uo[j] = a;
      a = take((int64_t)mj * cn);
      mv.push_back({L.Vo[j], a, mj, mj, mj, co}); L.Vo[j] = a;
      a = take(cn); mv.push_back({L.SUo[j], a, co, cn, co, 1}); L.SUo[j] = a;
      a = take(cn); mv.push_back({L.SVo[j], a, co, cn, co, 1}); L.SVo[j] = a;
      if (L.l > 2 && L.rpar[j] > 0) {
        a = take((int64_t)cn * L.rpar[j]); mv.push_back({L.PUo[j], a, co, cn, co, L.rpar[j]}); L.PUo[j] = a;
        a = take((int64_t)cn * L.rpar[j]); mv.push_back({L.PVo[j], a, co, cn, co, L.rpar[j]}); L.PVo[j] = a;
      }
      for (int code = 0; code < L.c7; ++code) {
        const int q = L.B7[(size_t)j * L.c7 + code];
        if (q < 0) continue;
        if (L.Kt[(size_t)j * L.c7 + code] >= 0) edges.push_back((int64_t)j * L.c7 + code);
        const int back = L.c7 - 1 - code;
        if (L.Kt[(size_t)q * L.c7 + back] >= 0) edges.push_back((int64_t)q * L.c7 + back);
      }
      for (int t = lv.nb_start[j]; t < lv.nb_start[j + 1]; ++t) {
        const int q = lv.nbr[t];
        if (q == j) continue;
        const size_t ixy = (size_t)q * L.c3 + offset3(lv, q, j), iyx = (size_t)j * L.c3 + offset3(lv, j, q);
        if (L.XYt[ixy] >= 0) { a = take((int64_t)L.m[q] * cn); mv.push_back({-1, a, 0, L.m[q], L.m[q], cn}); L.XYt[ixy] = a; updxy.push_back({(int64_t)ixy, a}); }
        if (L.YXt[iyx] >= 0) { a = take((int64_t)cn * L.m[q]); mv.push_back({-1, a, 0, cn, cn, L.m[q]}); L.YXt[iyx] = a; updyx.push_back({(int64_t)iyx, a}); }
      }
    }
    std::sort(edges.begin(), edges.end());
    edges.erase(std::unique(edges.begin(), edges.end()), edges.end());
    for (int64_t e : edges) {
      const int a = (int)(e / L.c7), code = (int)(e % L.c7);
      const int b = L.B7[(size_t)e];
      const int64_t d = take((int64_t)nc[a] * nc[b]);
      mv.push_back({L.Kt[(size_t)e], d, L.cap[a], nc[a], L.cap[a], L.cap[b]});
      L.Kt[(size_t)e] = d;
      upd7.push_back({e, d});
      (void)code;
    }
    // room for the new slots (the pool is copied when it moves), then zero them
    const int64_t used = L.size;
    if (o > L.capacity) {
      DevBuf np;
      const int64_t ncap = o + o / 4;
      np.alloc(sizeof(T) * ncap, &P.mem);
      IFMM_HIP(hipMemcpyAsync(np.p, L.pool.p, sizeof(T) * used, hipMemcpyDeviceToDevice, P.stream));
      L.pool = std::move(np);
      L.capacity = ncap;
    }
    IFMM_HIP(hipMemsetAsync(L.P() + used, 0, sizeof(T) * (o - used), P.stream));
    L.size = o;
    CopyBatch<T, T> cb;
    for (const auto& x : mv)
      if (x.src >= 0) cb.add(L.P() + x.src, x.lds, L.P() + x.dst, x.ldd, x.rows, x.cols);
    run_copy(P, cb, F.d4);
    L.cap = nc;
    // device tables: per-box arrays whole, the offset tables by scatter
    P.upload(L.dcap, L.cap); P.upload(L.dUo, L.Uo); P.upload(L.dVo, L.Vo); P.upload(L.dSUo, L.SUo);
    P.upload(L.dSVo, L.SVo); P.upload(L.dPUo, L.PUo); P.upload(L.dPVo, L.PVo);
    scatter_offsets(L.dKt, upd7);
    scatter_offsets(L.dXYt, updxy);
    scatter_offsets(L.dYXt, updyx);
    ++grow_events;
  }
  int64_t grow_events = 0;

  void scatter_offsets(DevBuf& table, const std::vector<std::pair<int64_t, int64_t>>& upd) {
    if (upd.empty()) return;
    DevBuf d;
    P.upload(d, upd);
    hipLaunchKernelGGL(k_scatter_offsets, dim3((unsigned)ceil_div((int64_t)upd.size(), WG)), dim3(WG), 0, P.stream,
                       d.template as<const int64_t>(), (int64_t)upd.size(), table.template as<int64_t>());
    IFMM_LAUNCH_CHECK();
    P.sync();   // d is released on return
  }

  // adjacency of two offsets in {-1, 0, 1}^d (codes as offset3): |o_a - o_b| <= 1 per axis
  std::vector<uint8_t> adj3_;
  int c3_ = 0;
  void build_adj3() {
    if (!adj3_.empty()) return;
    c3_ = 1;
    for (int k = 0; k < P.d; ++k) c3_ *= 3;
    adj3_.assign((size_t)c3_ * c3_, 0);
    for (int a = 0; a < c3_; ++a)
      for (int b = 0; b < c3_; ++b) {
        bool ok = true;
        for (int k = 0, x = a, y = b; k < P.d; ++k, x /= 3, y /= 3) {
          const int dd = x % 3 - y % 3;
          if (dd > 1 || dd < -1) ok = false;
        }
        adj3_[(size_t)a * c3_ + b] = ok ? 1 : 0;
      }
  }

  int offset3(const HLevel& lv, int i, int j) const {
    int code = 0, mul = 1;
    for (int k = 0; k < P.d; ++k) {
      code += (lv.coords[(size_t)j * P.d + k] - lv.coords[(size_t)i * P.d + k] + 1) * mul;
      mul *= 3;
    }
    return code;
  }

  // Initial K, PU, PV, SU, SV of level l from the R2 operators.
  void fill_from_r2(LevelPool<T>& L) {
    const int l = L.l;
    const HLevel& lv = P.T.lev[l];
    R2Level& z = P.r2[l];
    DevBuf dk = up(P, z.k), dko = up(P, z.k_off);
    if (!lv.inter.empty()) {
      hipLaunchKernelGGL(k_kinit<T>, dim3((unsigned)lv.inter.size()), dim3(WG), 0, P.stream,
                         P.ldev[l].in_start.template as<int>(), P.ldev[l].inter.template as<int>(), P.ldev[l].coords.template as<int>(), lv.nb,
                         P.d, L.c7, z.K.template as<double>(), dko.template as<int64_t>(), dk.template as<int>(), L.dcap.template as<int>(),
                         L.dKt.template as<int64_t>(), L.P());
      IFMM_LAUNCH_CHECK();
    }
    CopyBatch<double, T> cb;
    for (int i = 0; i < lv.nb; ++i) {
      cb.add(z.SU.template as<double>() + z.s_off[i], 1, L.P() + L.SUo[i], 1, z.k[i], 1);
      cb.add(z.SV.template as<double>() + z.s_off[i], 1, L.P() + L.SVo[i], 1, z.k[i], 1);
      if (l > 2) {
        const int kp = L.rpar[i];
        cb.add(z.PU.template as<double>() + z.p_off[i], z.k[i], L.P() + L.PUo[i], L.cap[i], z.k[i], kp);
        cb.add(z.PV.template as<double>() + z.p_off[i], z.k[i], L.P() + L.PVo[i], L.cap[i], z.k[i], kp);
      }
    }
    run_copy(P, cb, F.d1);
    P.sync();
  }

  void setup_leaf(LevelPool<T>& L) {
    const int l = P.L;
    const HLevel& lv = P.T.lev[l];
    std::vector<int> m(lv.nb);
    for (int i = 0; i < lv.nb; ++i) m[i] = (int)(P.T.leaf_start[i + 1] - P.T.leaf_start[i]);
    layout(L, l, m, P.r2[l].k);
    if (!lv.nbr.empty()) {
      hipLaunchKernelGGL(k_p2p_blocks<T>, dim3((unsigned)lv.nbr.size()), dim3(WG), 0, P.stream, P.pts.template as<double>(),
                         P.leaf_start.template as<int64_t>(), P.ldev[l].nb_start.template as<int>(), P.ldev[l].nbr.template as<int>(),
                         P.ldev[l].coords.template as<int>(), lv.nb, P.d, L.c3, P.kf, L.dSt.template as<int64_t>(), L.P());
      IFMM_LAUNCH_CHECK();
    }
    R2Level& z = P.r2[l];
    CopyBatch<double, T> cb;
    for (int i = 0; i < lv.nb; ++i) {
      cb.add(z.U.template as<double>() + z.u_off[i], m[i], L.P() + L.Uo[i], m[i], m[i], z.k[i]);
      cb.add(z.V.template as<double>() + z.u_off[i], m[i], L.P() + L.Vo[i], m[i], m[i], z.k[i]);
    }
    run_copy(P, cb, F.d1);
    fill_from_r2(L);
  }

  // ---------------------------------------------------------- recompression
  // Row and column edge lists of every box of the level (edges exist or not
  // for the whole level), built once per level on host threads and uploaded.
  // The first batch of a level builds them while its eliminations run.
  void ensure_edge_tables(LevelPool<T>& L) {
    if (L.erow_start.empty()) {
      // boxes split over host threads, chunks concatenated in order
      const int nt = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
      std::vector<std::vector<int>> rch(nt), cch(nt), rcnt(nt), ccnt(nt);
      std::vector<std::thread> th;
      const int per = (L.nb + nt - 1) / nt;
      for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
          const int j0 = t * per, j1 = std::min(L.nb, j0 + per);
          for (int j = j0; j < j1; ++j) {
            int nr = 0, nc = 0;
            for (int code = 0; code < L.c7; ++code) {
              const int q = L.B7[(size_t)j * L.c7 + code];
              if (q < 0) continue;
              if (L.Kt[(size_t)j * L.c7 + code] >= 0) { rch[t].push_back(code); ++nr; }
              if (L.Kt[(size_t)q * L.c7 + (L.c7 - 1 - code)] >= 0) { cch[t].push_back(code); ++nc; }
            }
            rcnt[t].push_back(nr);
            ccnt[t].push_back(nc);
          }
        });
      for (auto& x : th) x.join();
      L.erow_start.assign(L.nb + 1, 0);
      L.ecol_start.assign(L.nb + 1, 0);
      int j = 0;
      for (int t = 0; t < nt; ++t) {
        L.erow.insert(L.erow.end(), rch[t].begin(), rch[t].end());
        L.ecol.insert(L.ecol.end(), cch[t].begin(), cch[t].end());
        for (size_t k = 0; k < rcnt[t].size(); ++k, ++j) {
          L.erow_start[j + 1] = L.erow_start[j] + rcnt[t][k];
          L.ecol_start[j + 1] = L.ecol_start[j] + ccnt[t][k];
        }
      }
      P.upload(L.derow_start, L.erow_start);
      P.upload(L.derow, L.erow);
      P.upload(L.decol_start, L.ecol_start);
      P.upload(L.decol, L.ecol);
    }
  }

  // Plans workspace for the recompressions cs (ncols and box filled in) and
  // runs: gather, QR of MU^T / MV^T, transpose, Jacobi SVD, rank, r_j / t_j,
  // row and column transforms of every edge of the affected boxes, commit.
  void recompress(LevelPool<T>& L, std::vector<CompDesc>& cs, const std::vector<ElimDesc>& el,
                  const ElimDesc* d_el, const FNode* d_F, int64_t wbase) {
    if (cs.empty()) return;
    int64_t o = wbase;
    auto take = [&](int64_t n) { const int64_t a = o; o += (n + 1) & ~int64_t(1); return a; };
    for (auto& c : cs) {
      const int mj = L.m[c.box];
      c.kq = std::min(c.ncols, mj);
      c.mu = take((int64_t)c.ncols * mj);
      c.mv = take((int64_t)c.ncols * mj);
      c.ru = take((int64_t)c.kq * mj);
      c.rv = take((int64_t)c.kq * mj);
      c.uu = take((int64_t)mj * c.kq);
      c.vv = take((int64_t)mj * c.kq);
      c.su = take(c.kq);
      c.sv = take(c.kq);
      c.ldt = std::max(c.kq, 1);   // r_j, t_j: (new rank <= kq) x (old rank), leading dimension kq
      c.tr = take((int64_t)c.ldt * std::max(L.r[c.box], 1));
      c.tt = take((int64_t)c.ldt * std::max(L.r[c.box], 1));
      c.pu = take(mj + 2);
      c.pv = take(mj + 2);
      flops_comp += 2.0 * 2.0 * c.ncols * mj * mj + 2.0 * 12.0 * (double)mj * c.kq * c.kq;
    }
    if ((size_t)o * sizeof(T) > F.work.bytes) {
      P.sync();
      DevBuf nw;
      nw.alloc((size_t)o * sizeof(T) + ((size_t)o * sizeof(T)) / 4, &P.mem);
      if (debug_on()) IFMM_HIP(hipMemsetAsync(nw.p, 0, nw.bytes, P.stream));
      if (wbase > 0)
        IFMM_HIP(hipMemcpyAsync(nw.p, F.work.p, sizeof(T) * wbase, hipMemcpyDeviceToDevice, P.stream));
      F.work = std::move(nw);
    }
    T* W = F.work.template as<T>();
    const CompDesc* dc = P.put(F.d3, cs);
    LevelView v = L.view(P);   // taken again after grow_boxes, whose uploads may move the tables
    int mmax = 1;
    for (const auto& c : cs) mmax = std::max(mmax, L.m[c.box]);
    hipLaunchKernelGGL(k_comp_gather<T>, dim3((unsigned)cs.size(), (unsigned)ceil_div(mmax, COMP_ROWS)), dim3(WG), 0,
                       P.stream, dc, d_el, d_F, v, (const T*)L.P(), W);
    IFMM_LAUNCH_CHECK();
    std::vector<QrDesc> qd;
    std::vector<QrcpDesc> pd;
    std::vector<SvdDesc> sd;
    for (const auto& c : cs) {
      const int mj = L.m[c.box];
      for (int side = 0; side < 2; ++side) {
        QrDesc q;
        q.A = W + (side ? c.mv : c.mu);
        q.R = W + (side ? c.rv : c.ru);
        q.Q = nullptr;
        q.M = c.ncols; q.N = mj; q.lda = c.ncols; q.ldr = c.kq; q.ldq = 1; q.pad = 0;
        qd.push_back(q);
        // truncated pivoted QR of R; Y = R'^T (m_j x k) into the MU / MV storage
        int* perm = reinterpret_cast<int*>(W + (side ? c.pv : c.pu));
        QrcpDesc r;
        r.R = W + (side ? c.rv : c.ru);
        r.Y = W + (side ? c.mv : c.mu);
        r.perm = perm;
        r.kout = perm + mj;
        r.m = c.kq; r.n = mj; r.ldr = c.kq; r.ldy = mj;
        r.over = P.d_info + 1;
        pd.push_back(r);
        SvdDesc s{};
        s.B = W + (side ? c.mv : c.mu);
        s.U = W + (side ? c.vv : c.uu);
        s.S = W + (side ? c.sv : c.su);
        s.nlive = perm + mj;
        s.perm = perm;
        s.M = mj; s.N = c.kq; s.ldb = mj; s.ldu = mj;
        sd.push_back(s);
      }
    }
    chk(L, "comp_gather", nullptr, o);
    double fq = 0, bq = 0;
    for (const auto& c : cs) {
      const double mj = L.m[c.box], n = c.ncols, k = c.kq;
      fq += 2.0 * (2.0 * n * mj * mj - 2.0 / 3.0 * mj * mj * mj);   // Householder R of MU^T and MV^T
      bq += 2.0 * sizeof(T) * (n * mj + k * mj);
    }
    P.kset(KF_QR, fq, bq);
    {
      std::vector<QrJob> qj;
      qj.reserve(qd.size());
      for (const auto& q : qd) qj.push_back({q.A, q.R, q.M, q.N, q.lda, q.ldr});
      qr_blocked<T>(P, qj, F.qrs);
    }
    chk(L, "comp_qr", nullptr, o);
    auto nan_report = [&](const char* what, bool y) {
      if (!trace_on()) return;
      for (const auto& c : cs) {
        const int mj = L.m[c.box];
        for (int side = 0; side < 2; ++side) {
          std::vector<T> h;
          const int64_t off = y ? (side ? c.mv : c.mu) : (side ? c.rv : c.ru);
          P.download(h, W + off, (size_t)mj * c.kq);
          size_t bad = 0;
          double mx = 0;
          for (auto x : h) { if (!std::isfinite((double)x)) ++bad; else mx = std::max(mx, std::fabs((double)x)); }
          if (bad)
            std::fprintf(stderr, "[ifmm-trace] nan %s level=%d box=%d side=%d mj=%d kq=%d ncols=%d bad=%zu max=%.3e\n",
                         what, P.trace_level, c.box, side, mj, c.kq, c.ncols, bad, mx);
        }
      }
    };
    nan_report("after_qr", false);
    P.kset(-1);
    run_qrcp<T>(P, pd, F.d4, F.qcw, 1e-7 * P.tau);
    chk(L, "comp_qrcp", nullptr, o);
    nan_report("after_qrcp", true);
    P.kset(KF_SVD, 0, 0);   // flops are attributed to the SVD kernels themselves
    run_svd<T>(P, sd, F.d4, 1e-6 * P.tau);
    P.kset(-1);
    chk(L, "comp_svd", nullptr, o);
    P.kset(KF_XFORM);
    P.kbegin();
    hipLaunchKernelGGL(k_comp_rank<T>, dim3((unsigned)ceil_div((int64_t)cs.size(), WG)), dim3(WG), 0, P.stream, dc,
                       (int)cs.size(), v, (const T*)W, P.tau, P.rank_max);
    IFMM_LAUNCH_CHECK();
    // large boxes: r_j and t_j as batched products on the matrix cores, which
    // needs the new ranks on the host
    double rt_work = 0;
    for (const auto& c : cs) rt_work = std::max(rt_work, (double)c.kq * L.r[c.box] * L.m[c.box]);
    const bool rt_gemm = rt_work > RT_GEMM_WORK;
    std::vector<int> rn;
    {   // boxes whose new rank exceeds their capacity get larger slots first
      bool may = false;
      for (const auto& c : cs) may = may || c.kq > L.cap[c.box];
      if (may || rt_gemm) P.download(rn, L.drnew.p, (size_t)L.nb);
      if (may) {
        std::vector<std::pair<int, int>> want;
        for (const auto& c : cs)
          if (rn[c.box] > L.cap[c.box]) want.push_back({c.box, cap_for_rank(rn[c.box], L.m[c.box])});
        grow_boxes(L, want);
        v = L.view(P);
      }
    }
    if (trace_on()) {   // boxes whose common rank exceeds the resolved directions of one side
      std::vector<int> rn;
      P.download(rn, L.drnew.p, (size_t)L.nb);
      for (const auto& c : cs) {
        const int mj = L.m[c.box], k = rn[c.box];
        std::vector<T> su, sv;
        std::vector<int> pu, pv;
        P.download(su, W + c.su, (size_t)c.kq);
        P.download(sv, W + c.sv, (size_t)c.kq);
        P.download(pu, reinterpret_cast<int*>(W + c.pu) + mj, 1);
        P.download(pv, reinterpret_cast<int*>(W + c.pv) + mj, 1);
        int ku = 0, kv = 0, gu = 0, gv = 0;
        for (int a = 0; a < c.kq; ++a) {
          ku += su[a] > P.tau; kv += sv[a] > P.tau;
          gu += su[a] > 2e-6 * P.tau; gv += sv[a] > 2e-6 * P.tau;
        }
        if (k > gu || k > gv || ku != kv)
          std::fprintf(stderr,
                       "[ifmm-trace] rank level=%d box=%d elim=%d mj=%d ncols=%d kq=%d k=%d ku=%d kv=%d gu=%d gv=%d "
                       "liveu=%d livev=%d su[k-1]/tau=%.3e sv[k-1]/tau=%.3e\n",
                       P.trace_level, c.box, c.elim, mj, c.ncols, c.kq, k, ku, kv, gu, gv, pu[0], pv[0],
                       k > 0 ? (double)su[k - 1] / P.tau : 0.0, k > 0 ? (double)sv[k - 1] / P.tau : 0.0);
      }
    }
    {   // work vectors of the orthonormal completion in LDS: m_j + k values
      int64_t need = 1;
      for (const auto& c : cs) need = std::max<int64_t>(need, (int64_t)L.m[c.box] + c.kq);
      const size_t lds = sizeof(T) * (size_t)need;
      if (lds > COMPLETE_LDS_MAX) fail(IFMM_ERR_ARG, "a recompressed box is too large for the completion kernel");
      static const bool attr = [] {
        IFMM_HIP(hipFuncSetAttribute((const void*)k_comp_complete<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)COMPLETE_LDS_MAX));
        return true;
      }();
      (void)attr;
      hipLaunchKernelGGL(k_comp_complete<T>, dim3((unsigned)cs.size(), 2), dim3(WG), lds, P.stream, dc, v, W,
                         2e-6 * P.tau);
      IFMM_LAUNCH_CHECK();
    }
    if (rt_gemm) {   // r_j = Uhat^T U_j, t_j = Vhat^T V_j: (k x m_j)(m_j x r), leading dimension ldt
      GemmBatch g;
      for (const auto& c : cs) {
        const int j = c.box, k = rn[j], r = L.r[j], mj = L.m[j];
        if (k == 0 || r == 0 || mj == 0) continue;
        g.add(W + c.uu, mj, 1, L.P() + L.Uo[j], mj, 0, W + c.tr, c.ldt, k, r, mj, 1.0, 0.0);
        g.add(W + c.vv, mj, 1, L.P() + L.Vo[j], mj, 0, W + c.tt, c.ldt, k, r, mj, 1.0, 0.0);
      }
      P.kend();   // run_gemm times its launch as a range of its own (same family)
      run_gemm<T>(P, g, F.d5);
      P.kbegin();
    } else {
      hipLaunchKernelGGL(k_comp_rt<T>, dim3((unsigned)cs.size()), dim3(WG), 0, P.stream, dc, v, (const T*)L.P(), W);
      IFMM_LAUNCH_CHECK();
    }
    chk(L, "comp_rt", nullptr, o);
    P.kend();
    // one task per existing edge (the host holds the edge tables); flops of the
    // basis changes 2 k r cols per edge, with the new rank k bounded by the old
    // rank r (the new ranks are still on the device)
    ensure_edge_tables(L);
    // per recompression the first workgroup of its edges; flops estimated as
    // 2 r_j^2 (edges of j) rbar with the level's mean rank rbar (exact counts
    // would need a pass over every edge on the host)
    const int extra = L.l > 2 ? 2 : 0;
    std::vector<int> prow(cs.size() + 1, 0), pcol(cs.size() + 1, 0);
    double rbar = 0;
    for (int x : L.r) rbar += x;
    rbar = L.nb ? rbar / L.nb : 0.0;
    double frow = 0, fcol = 0;
    for (size_t ci = 0; ci < cs.size(); ++ci) {
      const int j = cs[ci].box;
      const int nr = L.erow_start[j + 1] - L.erow_start[j], nc = L.ecol_start[j + 1] - L.ecol_start[j];
      prow[ci + 1] = prow[ci] + nr + extra;
      pcol[ci + 1] = pcol[ci] + nc;
      const double r = L.r[j];
      frow += 2.0 * r * r * (nr * rbar + (extra ? 2.0 * L.rpar[j] : 0.0));
      fcol += 2.0 * r * r * nc * rbar;
    }
    std::vector<int> pre(prow.begin(), prow.end() - 1);
    pre.insert(pre.end(), pcol.begin(), pcol.end() - 1);
    const int* dpre = P.put(F.d5, pre);
    XfTasks xr{dpre, (int)cs.size(), extra, L.derow_start.template as<int>(), L.derow.template as<int>()};
    XfTasks xc{dpre + cs.size(), (int)cs.size(), 0, L.decol_start.template as<int>(), L.decol.template as<int>()};
    // small ranks (fine levels): one wavefront per edge, many edges resident per CU;
    // every capacity of the level within XF_BOX_R: one workgroup per recompressed box
    int rmax = 0;
    for (const auto& c : cs) rmax = std::max(rmax, L.r[c.box]);
    const bool small = rmax <= XF_SMALL_R;
    int capmax = 0;
    int64_t staged = 0;   // largest rank x parent-rank block a per-box workgroup stages
    for (int x : L.cap) capmax = std::max(capmax, x);
    for (const auto& c : cs) staged = std::max<int64_t>(staged, (int64_t)L.cap[c.box] * L.rpar[c.box]);
    const bool perbox = capmax <= XF_BOX_R && staged <= (int64_t)XF_BOX_R * XF_BOX_R;
    if (prow.back() > 0) {
      P.kone_begin(KF_ROW_XFORM, frow);
      if (perbox)
        hipLaunchKernelGGL(k_row_xform_box<T>, dim3((unsigned)cs.size()), dim3(256), 0, P.stream, dc, xr, v, L.P(),
                           (const T*)W);
      else if (small)
        hipLaunchKernelGGL((k_row_xform<T, 64, 8192>), dim3((unsigned)prow.back()), dim3(64), 0, P.stream, dc, xr, v,
                           L.P(), (const T*)W);
      else
        hipLaunchKernelGGL((k_row_xform<T, WG, XF_LDS>), dim3((unsigned)prow.back()), dim3(WG), 0, P.stream, dc, xr,
                           v, L.P(), (const T*)W);
      IFMM_LAUNCH_CHECK();
      P.kone_end();
    }
    chk(L, "row_xform", nullptr, o);
    if (pcol.back() > 0) {
      P.kone_begin(KF_COL_XFORM, fcol);
      if (perbox)
        hipLaunchKernelGGL(k_col_xform_box<T>, dim3((unsigned)cs.size()), dim3(256), 0, P.stream, dc, xc, v, L.P(),
                           (const T*)W);
      else if (small)
        hipLaunchKernelGGL((k_col_xform<T, 64, 8192>), dim3((unsigned)pcol.back()), dim3(64), 0, P.stream, dc, xc, v,
                           L.P(), (const T*)W);
      else
        hipLaunchKernelGGL((k_col_xform<T, WG, XF_LDS>), dim3((unsigned)pcol.back()), dim3(WG), 0, P.stream, dc, xc,
                           v, L.P(), (const T*)W);
      IFMM_LAUNCH_CHECK();
      P.kone_end();
    }
    P.kbegin();
    hipLaunchKernelGGL(k_comp_commit<T>, dim3((unsigned)cs.size()), dim3(WG), 0, P.stream, dc, v, L.P(),
                       (const T*)W);
    IFMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_commit_ranks, dim3((unsigned)ceil_div((int64_t)cs.size(), WG)), dim3(WG), 0, P.stream, dc,
                       (int)cs.size(), v);
    IFMM_LAUNCH_CHECK();
    P.kend();
    P.kset(-1);
    (void)el;
  }

  // Diagnostics: count non-finite values after a step (IFMM_DEBUG only).
  int dbg_level = 0, dbg_class = 0;
  bool dbg_reported = false;
  void chk(LevelPool<T>& L, const char* what, const DevBuf* fac, int64_t wused) {
    if (!debug_on() || dbg_reported) return;
    std::vector<T> h;
    size_t np = 0, nw = 0, nf = 0;
    P.download(h, L.pool.p, (size_t)L.size);
    for (auto x : h) np += std::isfinite((double)x) ? 0 : 1;
    if (wused > 0) {
      P.download(h, F.work.p, (size_t)wused);
      for (auto x : h) nw += std::isfinite((double)x) ? 0 : 1;
    }
    if (fac) {
      P.download(h, fac->p, fac->bytes / sizeof(T));
      for (auto x : h) nf += std::isfinite((double)x) ? 0 : 1;
    }
    if (np || nw || nf) {
      std::fprintf(stderr, "[ifmm] NON-FINITE after %s (level %d class %d): pool %zu work %zu factors %zu\n", what,
                   dbg_level, dbg_class, np, nw, nf);
      dbg_reported = true;
    }
  }

  // Diagnostics: smallest |pivot| of the class and non-finite values in the pool.
  void debug_class(LevelPool<T>& L, ClassFactors<T>& cf, int c) {
    std::vector<T> fac, pool;
    P.download(fac, F.arena.p, F.arena.bytes / sizeof(T));
    P.download(pool, L.pool.p, (size_t)L.size);
    double pmin = INFINITY;
    int bmin = -1;
    size_t nf = 0;
    for (const auto& e : cf.el)
      for (int k = 0; k < e.p; ++k) {
        const double v = std::fabs((double)fac[e.lu + k + (int64_t)k * e.p]);
        if (!(v >= pmin)) { pmin = v; bmin = e.box; }
      }
    for (auto x : pool) nf += std::isfinite((double)x) ? 0 : 1;
    std::fprintf(stderr, "[ifmm] level %d class %d: %zu eliminations, min |pivot| %.3e (box %d), non-finite in pool %zu\n",
                 L.l, c, cf.el.size(), pmin, bmin, nf);
  }

  // H = [A; G] and W_x of every elimination of a class (see ClassFactors),
  // from X = E_PP^-1[:, 0:m] (the first m columns of the inverse): G = E_FP X,
  // A = X[0:m, :], W_x = W[0:m, :].
  void solve_blocks(const std::vector<ElimDesc>& el, T* fac, T* sol) {
    CopyBatch<T, T> cp;
    GemmBatch gg;
    double fl = 0;
    for (const auto& e : el) {
      if (e.m == 0 || e.p == 0) continue;
      if (e.f > 0) {
        gg.add(fac + e.efp, e.f, 0, fac + e.xi, e.p, 0, sol + e.h + e.m, e.m + e.f, e.f, e.m, e.p, 1.0, 0.0);
        cp.add(fac + e.w, e.p, sol + e.wx, e.m, e.m, e.f, 0);
      }
      cp.add(fac + e.xi, e.p, sol + e.h, e.m + e.f, e.m, e.m, 0);
      fl += 2.0 * e.f * (double)e.p * e.m;
    }
    P.kset(KF_SCHUR, fl, 0);
    run_gemm<T>(P, gg, F.d5);
    P.kset(-1);
    run_copy(P, cp, F.d4);
  }

  // Redirect the compressed well-separated fill through K (eq. K_kj_update,
  // Alg. 3): for every ordered pair (a, b) of F of an elimination whose boxes
  // are not adjacent (and not both y), K(a, b) += op_a(D(a, b)) op_b with
  // op = Uhat^T on an x~ row side and Vhat on an x~ column side, as batched
  // products: x~-x~ pairs through T = Uhat_a^T D(a, b), then K += T Vhat_b; an
  // x~-y or y-x~ pair in one product. The new ranks are read once per class.
  void redirect(LevelPool<T>& L, const std::vector<ElimDesc>& el, const std::vector<FNode>& Fs,
                const HLevel& lv) {
    P.download(L.r, L.dr.p, (size_t)L.nb);
    T* Wk = F.work.template as<T>();
    T* pool = L.P();
    GemmBatch g1, g2;
    struct Pend { const T* D; int ldD, ma, mb, ka, kb; int64_t dst, ua, vb; int ld; };
    std::vector<Pend> xx;
    int64_t tmp = 0;
    double fl = 0;
    for (const auto& e : el) {
      for (int ia = 0; ia < e.nF; ++ia) {
        const FNode& A = Fs[e.F0 + ia];
        for (int ib = 0; ib < e.nF; ++ib) {
          const FNode& B = Fs[e.F0 + ib];
          if (A.type == 1 && B.type == 1) continue;
          if (adjacent(lv, P.d, A.box, B.box)) continue;
          const int code = offset7(lv, P.d, A.box, B.box);
          if (code < 0) continue;
          const int64_t dst = L.Kt[(size_t)A.box * L.c7 + code];
          if (dst < 0) continue;
          const int ka = A.type == 0 ? L.r[A.box] : A.dim;
          const int kb = B.type == 0 ? L.r[B.box] : B.dim;
          if (ka == 0 || kb == 0 || A.dim == 0 || B.dim == 0) continue;
          const T* D = Wk + e.dlt + A.off + (int64_t)B.off * e.f;
          const int ld = L.cap[A.box];
          if (A.type == 0 && B.type == 0) {
            xx.push_back({D, e.f, A.dim, B.dim, ka, kb, dst, L.Uo[A.box], L.Vo[B.box], ld});
            tmp += ((int64_t)ka * B.dim + 1) & ~int64_t(1);
            fl += 2.0 * ka * A.dim * B.dim + 2.0 * ka * B.dim * kb;
          } else if (A.type == 0) {   // Uhat_a^T D
            g1.add(pool + L.Uo[A.box], A.dim, 1, D, e.f, 0, pool + dst, ld, ka, kb, A.dim, 1.0, 1.0);
            fl += 2.0 * ka * A.dim * kb;
          } else {                    // D Vhat_b
            g1.add(D, e.f, 0, pool + L.Vo[B.box], B.dim, 0, pool + dst, ld, ka, kb, B.dim, 1.0, 1.0);
            fl += 2.0 * ka * B.dim * kb;
          }
        }
      }
    }
    if (!xx.empty()) {
      if ((size_t)tmp * sizeof(T) > F.rtmp.bytes) P.sync();
      F.rtmp.reserve(sizeof(T) * (size_t)std::max<int64_t>(tmp, 2), &P.mem);
      T* Tb = F.rtmp.template as<T>();
      int64_t o = 0;
      for (const auto& x : xx) {
        g1.add(pool + x.ua, x.ma, 1, x.D, x.ldD, 0, Tb + o, x.ka, x.ka, x.mb, x.ma, 1.0, 0.0);
        g2.add(Tb + o, x.ka, 0, pool + x.vb, x.mb, 0, pool + x.dst, x.ld, x.ka, x.kb, x.mb, 1.0, 1.0);
        o += ((int64_t)x.ka * x.mb + 1) & ~int64_t(1);
      }
    }
    P.kset(KF_XFORM, fl, 0);
    run_gemm<T>(P, g1, F.d5);
    run_gemm<T>(P, g2, F.d5);
    P.kset(-1);
  }

  // ----------------------------------------------------------- one level
  void eliminate_level(LevelPool<T>& L) {
    build_adj3();
    const int l = L.l;
    const HLevel& lv = P.T.lev[l];
    const int d = P.d;
    F.cls[l].clear();
    for (int c = 0; c < lv.ncolour; ++c) {
      if (lv.classes[c].empty()) continue;
      {
        HostScope hs(P.hprof, "class: wait + read ranks");
        P.download(L.r, L.dr.p, (size_t)lv.nb);
      }
      // A class whose transient blocks (pivot blocks, couplings, Schur fill
      // f x f, recompression matrices) would exceed CLASS_BYTES is taken in
      // several batches, one after the other. The boxes of a class are an
      // independent set, so the split leaves every elimination's F unchanged.
      std::vector<std::vector<int>> batches(1);
      {
        double acc = 0;
        for (int i : lv.classes[c]) {
          const double est = elim_bytes(L, lv, i);
          if (acc > 0 && acc + est > (double)CLASS_BYTES) { batches.emplace_back(); acc = 0; }
          batches.back().push_back(i);
          acc += est;
        }
      }
      for (size_t bt = 0; bt < batches.size(); ++bt) {
        eliminate_batch(L, batches[bt], c, bt > 0);
        if (progress_level() >= 2) {
          double est = 0;
          for (int i : batches[bt]) est += elim_bytes(L, lv, i);
          P.sync();
          std::fprintf(stderr, "[ifmm]     level %d class %d batch %zu: %zu boxes, estimate %.2f GB, device %.2f GB "
                       "(peak %.2f GB)\n", l, c, bt, batches[bt].size(), est * 1e-9, P.mem.cur * 1e-9,
                       P.mem.peak * 1e-9);
          std::fflush(stderr);
        }
      }
      if (progress_on() && l <= 4) {
        P.sync();
        std::fprintf(stderr, "[ifmm]   level %d class %d: %zu boxes done, device %.1f GB\n", l, c,
                     lv.classes[c].size(), P.mem.cur * 1e-9);
        std::fflush(stderr);
      }
    }
    P.download(L.r, L.dr.p, (size_t)lv.nb);
  }

  // Host estimate of the transient bytes of eliminating box i now: the class
  // arena (2 p^2 + 3 p f), the Schur fill (f^2), the solve blocks ((m + f) m +
  // m f) and the recompression matrices of its neighbours (about 6 (r_j + f) m_j).
  double elim_bytes(const LevelPool<T>& L, const HLevel& lv, int i) const {
    const double m = L.m[i], p = m + L.r[i];
    double f = L.r[i], rec = 0;
    for (int t = lv.nb_start[i]; t < lv.nb_start[i + 1]; ++t) {
      const int j = lv.nbr[t];
      if (j != i) f += std::max(L.m[j], L.cap[j]);
    }
    for (int t = lv.nb_start[i]; t < lv.nb_start[i + 1]; ++t) {
      const int j = lv.nbr[t];
      if (j != i) rec += 6.0 * (L.r[j] + f) * L.m[j];
    }
    return sizeof(T) * (2 * p * p + 3 * p * f + f * f + (m + f) * m + m * f + rec);
  }

  // Eliminate the boxes of one batch of colour class c (all of it, or a part
  // when the class is split); `again`: a later batch of the same class, whose
  // ranks must be read back first.
  void eliminate_batch(LevelPool<T>& L, const std::vector<int>& boxes, int c, bool again) {
    const int l = L.l;
    const HLevel& lv = P.T.lev[l];
    const int d = P.d;
    {
      if (again) {
        HostScope hs(P.hprof, "class: wait + read ranks");
        P.download(L.r, L.dr.p, (size_t)lv.nb);
      }
      // ranks are exact on the host at the start of every batch; the stream is
      // idle, so the descriptors of the previous batch can be recycled
      P.arena_reset();
      HostScope hs_plan(P.hprof, "class: plan");
      F.cls[l].emplace_back();
      ClassFactors<T>& cf = F.cls[l].back();
      std::vector<ElimDesc>& el = cf.el;
      std::vector<FNode>& Fs = cf.F;
      el.clear();
      Fs.clear();
      int64_t fo = 0, po = 0, wo = 0, so = 0;
      int maxF = 0;
      std::vector<CompDesc> cs;
      // Each box is planned on its own (its F nodes in order, the recompressions
      // its elimination triggers), on host threads for large batches; offsets
      // into the class buffers are then assigned in box order, so the plan is
      // the same whatever the thread count.
      const int nbx = (int)boxes.size();
      std::vector<ElimDesc> eb(nbx);
      std::vector<std::vector<FNode>> fb(nbx);
      std::vector<std::vector<CompDesc>> cb(nbx);
      auto plan_box = [&](int x, std::vector<int>& fcode) {
        const int i = boxes[x];
        ElimDesc& e = eb[x];
        std::vector<FNode>& nodes = fb[x];
        e = ElimDesc{};
        e.box = i;
        e.m = L.m[i];
        e.r = L.r[i];
        e.p = e.m + e.r;
        fcode.clear();
        int f = 0;
        auto push = [&](int type, int b) {
          fcode.push_back(offset3(lv, i, b));
          FNode n{};
          n.type = type;
          n.box = b;
          n.dim = type == 0 ? L.m[b] : L.r[b];
          n.off = f;
          if (type == 0) {
            n.src_row = L.St[(size_t)i * L.c3 + offset3(lv, i, b)];
            n.ld_row = L.m[i];
            n.src_col = L.St[(size_t)b * L.c3 + offset3(lv, b, i)];
            n.ld_col = L.m[b];
          } else if (b != i) {
            n.src_row = L.XYt[(size_t)i * L.c3 + offset3(lv, i, b)];
            n.ld_row = L.m[i];
            n.src_col = L.YXt[(size_t)b * L.c3 + offset3(lv, b, i)];
            n.ld_col = L.cap[b];
          } else {
            n.src_row = -1; n.src_col = -1; n.ld_row = 1; n.ld_col = 1;
          }
          f += n.dim;
          nodes.push_back(n);
        };
        for (int t = lv.nb_start[i]; t < lv.nb_start[i + 1]; ++t) {
          const int j = lv.nbr[t];
          if (j != i && lv.colour[j] > c) push(0, j);
        }
        for (int t = lv.nb_start[i]; t < lv.nb_start[i + 1]; ++t) {
          const int j = lv.nbr[t];
          if (j != i && lv.colour[j] < c) push(1, j);
        }
        push(1, i);
        e.nF = (int)nodes.size();
        e.f = f;
        e.S = L.St[(size_t)i * L.c3 + offset3(lv, i, i)];
        e.U = L.Uo[i];
        e.V = L.Vo[i];
        // recompressions triggered by this elimination
        for (int a = 0; a < e.nF; ++a) {
          const FNode& X = nodes[a];
          if (X.type != 0) continue;
          int nc = L.r[X.box];
          bool any = false;
          // both are neighbours of i: adjacent iff their offsets from i differ by at most one
          const uint8_t* adj = &adj3_[(size_t)fcode[a] * c3_];
          for (int b = 0; b < e.nF; ++b) {
            if (!adj[fcode[b]]) { nc += nodes[b].dim; any = true; }
          }
          if (!any) continue;
          CompDesc cd{};
          cd.box = X.box;
          cd.elim = x;
          cd.a = a;
          cd.ncols = nc;
          cb[x].push_back(cd);
        }
      };
      {
        const int nt = nbx >= 512 ? (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())) : 1;
        auto part = [&](int t) {
          std::vector<int> fcode;   // offset code (3^d) of each F node of the box relative to it
          for (int x = t; x < nbx; x += nt) plan_box(x, fcode);
        };
        if (nt == 1) {
          part(0);
        } else {
          std::vector<std::thread> th;
          for (int t = 0; t < nt; ++t) th.emplace_back(part, t);
          for (auto& h : th) h.join();
        }
      }
      for (int x = 0; x < nbx; ++x) {
        ElimDesc e = eb[x];
        e.F0 = (int)Fs.size();
        Fs.insert(Fs.end(), fb[x].begin(), fb[x].end());
        maxF = std::max(maxF, e.nF);
        e.lu = fo; fo += ((int64_t)e.p * e.p + 1) & ~int64_t(1);
        e.w = fo; fo += ((int64_t)e.p * e.f + 1) & ~int64_t(1);
        e.epf = fo; fo += ((int64_t)e.p * e.f + 1) & ~int64_t(1);
        e.efp = fo; fo += ((int64_t)e.f * e.p + 1) & ~int64_t(1);
        e.xi = fo; fo += ((int64_t)e.p * e.p + 1) & ~int64_t(1);
        e.h = so; so += ((int64_t)(e.m + e.f) * e.m + 1) & ~int64_t(1);
        e.wx = so; so += ((int64_t)e.m * e.f + 1) & ~int64_t(1);
        e.piv = po; po += e.p;
        e.dlt = wo; wo += ((int64_t)e.f * e.f + 1) & ~int64_t(1);
        cs.insert(cs.end(), cb[x].begin(), cb[x].end());
        flops_lu += 2.0 / 3.0 * e.p * (double)e.p * e.p + 2.0 * e.p * (double)e.p * e.f;
        flops_schur += 2.0 * e.f * (double)e.f * e.p;
        flops_other += 2.0 * e.p * (double)e.p * e.p + 2.0 * e.f * (double)e.p * e.m;
        factor_elems += (int64_t)(e.m + e.f) * e.m + (int64_t)e.m * e.f;
        el.push_back(e);
      }
      hs_plan.stop();
      HostScope hs_launch(P.hprof, "class: allocate + launch");
      if ((size_t)fo * sizeof(T) > F.arena.bytes || (size_t)po * sizeof(int) > F.pivs.bytes ||
          (size_t)wo * sizeof(T) > F.work.bytes)
        P.sync();   // kernels of the previous class may still use the buffers being replaced
      F.arena.reserve(sizeof(T) * std::max<int64_t>(fo, 2), &P.mem);
      F.pivs.reserve(sizeof(int) * std::max<int64_t>(po, 1), &P.mem);
      cf.sol.alloc(sizeof(T) * std::max<int64_t>(so, 2), &P.mem);
      if ((size_t)wo * sizeof(T) > F.work.bytes)
        F.work.alloc((size_t)wo * sizeof(T) + (size_t)wo * sizeof(T) / 4 + 64, &P.mem);
      T* fac = F.arena.template as<T>();
      int* piv = F.pivs.template as<int>();
      T* sol = cf.sol.template as<T>();
      T* W = F.work.template as<T>();
      if (debug_on()) {   // so that the non-finite checks see only computed values
        IFMM_HIP(hipMemsetAsync(F.arena.p, 0, F.arena.bytes, P.stream));
        IFMM_HIP(hipMemsetAsync(F.work.p, 0, F.work.bytes, P.stream));
      }
      const ElimDesc* del = P.put(F.d1, el);
      const FNode* dF = P.put(F.d2, Fs);
      // gather pivot blocks and couplings
      hipLaunchKernelGGL(k_gather<T>, dim3((unsigned)el.size(), maxF + 1), dim3(WG), 0, P.stream, del, dF,
                         (const T*)L.P(), fac);
      IFMM_LAUNCH_CHECK();
      // LU with partial pivoting of every pivot block, E_PP^-1 by the LU solve of
      // the identity, then W = E_PP^-1 E_PF as one product (instead of a
      // triangular solve with |F| right-hand sides)
      std::vector<LuJob> lu;
      std::vector<TrsJob> ls;
      CopyBatch<T, T> eye;
      GemmBatch gb, gw;
      for (const auto& e : el) {
        if (e.p > 0) {
          lu.push_back({fac + e.lu, piv + e.piv, e.p, e.p, l * 1000000 + e.box});
          eye.add(nullptr, e.p, fac + e.xi, e.p, e.p, e.p, 2, 1.0);
          ls.push_back({fac + e.lu, piv + e.piv, fac + e.xi, e.p, e.p, e.p, e.p});
          if (e.f > 0)
            gw.add(fac + e.xi, e.p, 0, fac + e.epf, e.p, 0, fac + e.w, e.p, e.p, e.f, e.p, 1.0, 0.0);
        }
        // Schur fill D = -E_FP W (f x f, inner p)
        gb.add(fac + e.efp, std::max(e.f, 1), 0, fac + e.w, std::max(e.p, 1), 0, W + e.dlt, std::max(e.f, 1), e.f,
               e.f, e.p, -1.0, 0.0);
        if (e.p == 0 && e.f > 0)
          IFMM_HIP(hipMemsetAsync(W + e.dlt, 0, sizeof(T) * (size_t)e.f * e.f, P.stream));
      }
      if (debug_on() && l == P.L && c == 0) {
        for (size_t b = 0; b < el.size() && b < 3; ++b) {
          const ElimDesc& e = el[b];
          std::fprintf(stderr, "[ifmm] elim box %d m %d r %d p %d f %d nF %d\n", e.box, e.m, e.r, e.p, e.f, e.nF);
          dbg_dump<T>(P, "EPP", fac + e.lu, (size_t)e.p * e.p, 12);
          dbg_dump<T>(P, "U_i", L.P() + e.U, (size_t)e.m * e.r, 8);
          dbg_dump<T>(P, "S_ii", L.P() + e.S, (size_t)e.m * e.m, 8);
        }
      }
      dbg_level = l;
      dbg_class = c;
      chk(L, "gather", &F.arena, 0);
      double flu = 0, ftr = 0, fsc = 0, bsc = 0;
      for (const auto& e : el) {
        const double p = e.p, f = e.f;
        flu += 2.0 / 3.0 * p * p * p;
        ftr += 2.0 * p * p * p + 2.0 * p * p * f;
        fsc += 2.0 * f * f * p;
        bsc += sizeof(T) * (2.0 * f * p + f * f);   // read E_FP and W once, write D once
      }
      P.kset(KF_LU, flu, 0);
      lu_blocked<T>(P, lu, F.lus);
      chk(L, "lu", &F.arena, 0);
      run_copy(P, eye, F.d4);
      P.kset(KF_TRSM, ftr, 0);
      lu_solve_blocked<T>(P, ls, F.lus);
      run_gemm<T>(P, gw, F.d5);
      chk(L, "lu_solve", &F.arena, 0);
      P.kset(KF_SCHUR, fsc, bsc);
      run_gemm<T>(P, gb, F.d5);
      P.kset(-1);
      chk(L, "schur", nullptr, wo);
      solve_blocks(el, fac, sol);
      chk(L, "solve_blocks", &F.arena, 0);
      LevelView v = L.view(P);
      // near fill: added to existing edges
      hipLaunchKernelGGL(k_near_scatter<T>, dim3((unsigned)el.size(), maxF * maxF), dim3(WG), 0, P.stream, del, dF,
                         v, (const T*)W, L.P());
      IFMM_LAUNCH_CHECK();
      // well-separated fill: recompress the bases of the affected boxes, then redirect
      IFMM_HIP(hipMemcpyAsync(L.drnew.p, L.dr.p, sizeof(int) * lv.nb, hipMemcpyDeviceToDevice, P.stream));
      chk(L, "near_scatter", nullptr, wo);
      ensure_edge_tables(L);   // host work of the level's first batch while its eliminations run
      hs_launch.stop();
      {
        HostScope hs(P.hprof, "class: recompress");
        recompress(L, cs, el, del, dF, wo);
      }
      HostScope hs_red(P.hprof, "class: redirect");
      chk(L, "recompress", nullptr, 0);
      v = L.view(P);   // recompress may have grown boxes, which moves the level's tables
      {   // coarse levels (large ranks): batched products; fine levels: one workgroup per pair on the device
        int rmax = 0, mmax = 0;
        for (int x : L.cap) rmax = std::max(rmax, x);
        for (int x : L.m) mmax = std::max(mmax, x);
        if (rmax > XF_SMALL_R || mmax > REDIRECT_MAXM || force_streamed()) {
          redirect(L, el, Fs, lv);
        } else {
          P.kset(KF_XFORM);
          P.kbegin();
          hipLaunchKernelGGL(k_redirect<T>, dim3((unsigned)el.size(), maxF * maxF), dim3(WG), 0, P.stream, del, dF, v,
                             (const T*)F.work.template as<T>(), L.P());
          IFMM_LAUNCH_CHECK();
          P.kend();
          P.kset(-1);
        }
      }
      if (debug_on()) debug_class(L, cf, c);
    }
  }

  // ---------------------------------------------------- merge into l - 1
  void merge(LevelPool<T>& C, LevelPool<T>& Pp) {
    P.arena_reset();
    const int l = C.l, lp = l - 1;
    const HLevel& lv = P.T.lev[lp];
    std::vector<int> m(lv.nb, 0), choff(C.nb, 0);
    for (int p = 0; p < lv.nb; ++p) {
      int o = 0;
      for (int c = lv.ch_start[p]; c < lv.ch_start[p + 1]; ++c) { choff[c] = o; o += C.r[c]; }
      m[p] = o;
    }
    layout(Pp, lp, m, P.r2[lp].k);
    DevBuf dch = up(P, choff);
    if (!lv.nbr.empty()) {
      hipLaunchKernelGGL(k_merge_S<T>, dim3((unsigned)lv.nbr.size()), dim3(WG), 0, P.stream,
                         P.ldev[lp].nb_start.template as<int>(), P.ldev[lp].nbr.template as<int>(), P.ldev[lp].coords.template as<int>(), lv.nb,
                         P.d, P.ldev[lp].ch_start.template as<int>(), P.ldev[l].coords.template as<int>(), dch.template as<int>(),
                         C.dr.template as<int>(), C.dcap.template as<int>(), C.dKt.template as<int64_t>(), C.c7, (const T*)C.P(),
                         Pp.dm.template as<int>(), Pp.dSt.template as<int64_t>(), Pp.c3, Pp.P());
      IFMM_LAUNCH_CHECK();
    }
    hipLaunchKernelGGL(k_merge_UV<T>, dim3(lv.nb), dim3(WG), 0, P.stream, P.ldev[lp].ch_start.template as<int>(), lv.nb,
                       dch.template as<int>(), C.dr.template as<int>(), C.dcap.template as<int>(), C.dPUo.template as<int64_t>(), C.dPVo.template as<int64_t>(),
                       (const T*)C.P(), Pp.dm.template as<int>(), Pp.dr.template as<int>(), Pp.dUo.template as<int64_t>(), Pp.dVo.template as<int64_t>(),
                       Pp.P());
    IFMM_LAUNCH_CHECK();
    fill_from_r2(Pp);
    // recompress the merged bases [U_p Sigma_U] and [V_p Sigma_V] at tau
    std::vector<CompDesc> cs;
    for (int p = 0; p < lv.nb; ++p) {
      CompDesc cd{};
      cd.box = p;
      cd.elim = -1;
      cd.a = 0;
      cd.ncols = Pp.r[p];
      if (cd.ncols > 0 && Pp.m[p] > 0) cs.push_back(cd);
      else if (Pp.r[p] > 0) fail(IFMM_ERR_INTERNAL, "merged box with basis but no unknowns");
    }
    IFMM_HIP(hipMemcpyAsync(Pp.drnew.p, Pp.dr.p, sizeof(int) * lv.nb, hipMemcpyDeviceToDevice, P.stream));
    recompress(Pp, cs, {}, nullptr, nullptr, 0);
    P.download(Pp.r, Pp.dr.p, (size_t)lv.nb);
  }

  void top(LevelPool<T>& L) {
    P.arena_reset();
    const HLevel& lv = P.T.lev[2];
    std::vector<int64_t> off(lv.nb + 1, 0);
    for (int i = 0; i < lv.nb; ++i) off[i + 1] = off[i] + L.r[i];
    const int n = (int)off[lv.nb];
    F.ntop = n;
    F.topinv.alloc(sizeof(T) * std::max<int64_t>((int64_t)n * n, 1), &P.mem);
    if (n == 0) return;
    DevBuf top, toppiv;
    top.alloc(sizeof(T) * (size_t)n * n, &P.mem);
    toppiv.alloc(sizeof(int) * (size_t)n, &P.mem);
    DevBuf doff = up(P, off);
    hipLaunchKernelGGL(k_top_gather<T>, dim3((unsigned)(lv.nb * lv.nb)), dim3(WG), 0, P.stream, lv.nb,
                       P.ldev[2].coords.template as<int>(), P.d, L.c7, L.dr.template as<int>(), L.dcap.template as<int>(), L.dKt.template as<int64_t>(),
                       doff.template as<int64_t>(), n, (const T*)L.P(), top.template as<T>());
    IFMM_LAUNCH_CHECK();
    std::vector<LuJob> lu(1);
    lu[0] = {top.template as<T>(), toppiv.template as<int>(), n, n, 999999999};
    P.kset(KF_LU, 2.0 / 3.0 * (double)n * n * n, 0);
    lu_blocked<T>(P, lu, F.lus);
    // the explicit inverse turns the top substitution into one matrix-vector product
    CopyBatch<T, T> id;
    id.add(nullptr, n, F.topinv.template as<T>(), n, n, n, 2, 1.0);
    run_copy(P, id, F.d4);
    std::vector<TrsJob> inv(1);
    inv[0] = {top.template as<T>(), toppiv.template as<int>(), F.topinv.template as<T>(), n, n, n, n};
    P.kset(KF_TRSM, 2.0 * (double)n * n * n, 0);
    lu_solve_blocked<T>(P, inv, F.lus);
    P.kset(-1);
    P.sync();   // top and toppiv are released on return
    flops_lu += 2.0 / 3.0 * (double)n * n * n;
    flops_other += 2.0 * (double)n * n * n;
    factor_elems += (int64_t)n * n;
  }

  // Solve plan of a finished level: x~ offsets, y offsets (one level up).
  void plan_solve(const LevelPool<T>& L) {
    const int l = L.l;
    const HLevel& lv = P.T.lev[l];
    SolveLevel<T>& s = F.sl[l];
    s.xoff.assign(lv.nb + 1, 0);
    s.yoff.assign(lv.nb + 1, 0);
    for (int i = 0; i < lv.nb; ++i) {
      s.xoff[i + 1] = s.xoff[i] + L.m[i];
      s.yoff[i + 1] = s.yoff[i] + L.r[i];
    }
    s.M = s.xoff[lv.nb];
    s.Mup = s.yoff[lv.nb];
  }

  void run() {
    const int Lv = P.L;
    F.cls.clear();
    F.cls.resize(Lv + 1);
    F.sl.assign(Lv + 1, SolveLevel<T>());
    auto cur = std::make_unique<LevelPool<T>>();
    const double t0 = now_ms();
    {
      HostScope hs(P.hprof, "setup leaf level");
      setup_leaf(*cur);
    }
    if (progress_on()) {
      P.sync();
      std::fprintf(stderr, "[ifmm] leaf level set up: pool %.2f GB, device %.2f GB (peak %.2f GB)\n",
                   cur->capacity * sizeof(T) * 1e-9, P.mem.cur * 1e-9, P.mem.peak * 1e-9);
      std::fflush(stderr);
    }
    for (int l = Lv; l >= 2; --l) {
      P.trace_level = l;
      eliminate_level(*cur);
      HostScope hs_ps(P.hprof, "plan solve");
      plan_solve(*cur);
      hs_ps.stop();
      P.st.max_rank[l] = 0;
      double sum = 0;
      for (int x : cur->r) { P.st.max_rank[l] = std::max(P.st.max_rank[l], x); sum += x; }
      P.st.mean_rank[l] = cur->nb ? sum / cur->nb : 0.0;
      if (progress_on()) {
        int mmax = 0;
        for (int x : cur->m) mmax = std::max(mmax, x);
        std::fprintf(stderr,
                     "[ifmm] level %d eliminated: %d boxes in %zu batches, largest x~ %d, max rank %d, mean %.1f, "
                     "grown boxes %lld, %.1f s, device %.1f GB (peak %.1f GB)\n",
                     l, cur->nb, F.cls[l].size(), mmax, P.st.max_rank[l], P.st.mean_rank[l], (long long)grow_events,
                     (now_ms() - t0) * 1e-3, P.mem.cur * 1e-9, P.mem.peak * 1e-9);
        std::fflush(stderr);
      }
      if (l > 2) {
        HostScope hs(P.hprof, "merge");
        auto nxt = std::make_unique<LevelPool<T>>();
        merge(*cur, *nxt);
        HostScope hs_free(P.hprof, "free child level");
        cur = std::move(nxt);
      } else {
        HostScope hs(P.hprof, "top");
        top(*cur);
      }
    }
    {
      HostScope hs(P.hprof, "final wait");
      P.sync();
    }
    std::vector<int> info;
    P.download(info, P.d_info, 2);
    if (info[1] != -1)
      fail(IFMM_ERR_ARG, "a recompression kept more than " + std::to_string(SVD_MAXK) +
                             " directions (the largest rank the SVD kernels take)");
    if (info[0] != -1) {
      P.st.error_level = info[0] == 999999999 ? 1 : info[0] / 1000000;
      P.st.error_box = info[0] == 999999999 ? -1 : info[0] % 1000000;
      fail(IFMM_ERR_SINGULAR, "zero pivot in the elimination (level " + std::to_string(P.st.error_level) +
                                  ", box " + std::to_string(P.st.error_box) + ")");
    }
    P.st.factor_flops = flops_lu + flops_schur + flops_comp + flops_other;
    P.st.schur_flops = flops_schur;
    P.st.factor_bytes = factor_elems * (int64_t)sizeof(T);
  }
};

}  // namespace ifmm
