// Build: tree (GPU keys + sort, host lists), R1 operators, R2 initial operators
// with sigma_0, and the H2 product. Alg. 1, lines constructing the octree and
// initialising the operators of every level; Sec. 3 opening; Sec. 2.4.
#pragma once

#include "r2init.hpp"

namespace ifmm {

template <class T>
inline DevBuf up(Problem& P, const std::vector<T>& v) {
  DevBuf b;
  P.upload(b, v);
  return b;
}

inline void grid1(int64_t n, dim3& g) { g = dim3((unsigned)std::max<int64_t>(1, ceil_div(n, WG))); }

// ----------------------------------------------------------------- tree
inline void build_tree(Problem& P, const double* d_points, int depth, int leaf_max) {
  const int64_t n = P.n;
  const int d = P.d;
  // bounding box
  const int nblk = (int)std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(n, WG)));
  DevBuf part;
  part.alloc(sizeof(double) * nblk * 2 * d, &P.mem);
  hipLaunchKernelGGL(k_bbox_partial, dim3(nblk), dim3(WG), 0, P.stream, d_points, n, d, part.as<double>());
  IFMM_LAUNCH_CHECK();
  std::vector<double> hp;
  P.download(hp, part.p, (size_t)nblk * 2 * d);
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
    for (int b = 0; b < nblk; ++b) {
      const double a = hp[(size_t)b * 2 * d + k], c = hp[(size_t)b * 2 * d + d + k];
      if (std::isnan(a) || std::isnan(c)) fail(IFMM_ERR_ARG, "non-finite point coordinates");
      lo[k] = std::min(lo[k], a);
      hi[k] = std::max(hi[k], c);
    }
    if (!std::isfinite(lo[k]) || !std::isfinite(hi[k])) fail(IFMM_ERR_ARG, "non-finite point coordinates");
  }
  double side = 0;
  for (int k = 0; k < d; ++k) side = std::max(side, hi[k] - lo[k]);
  side = side * (1.0 + 1e-12);
  if (side == 0.0) side = 1.0;
  HTree& T = P.T;
  T.n = n;
  T.d = d;
  T.side = side;
  for (int k = 0; k < 3; ++k) T.origin[k] = 0;
  for (int k = 0; k < d; ++k) T.origin[k] = 0.5 * (lo[k] + hi[k]) - 0.5 * side;
  T.inv = 1.0 / side;

  DevBuf keys_in, keys_out, idx_in, idx_out, cnt;
  keys_in.alloc(sizeof(uint64_t) * n, &P.mem);
  keys_out.alloc(sizeof(uint64_t) * n, &P.mem);
  idx_in.alloc(sizeof(int) * n, &P.mem);
  idx_out.alloc(sizeof(int) * n, &P.mem);
  cnt.alloc(sizeof(int) * (size_t)RS_BINS * (size_t)ceil_div(n, RS_TILE), &P.mem);
  dim3 g;
  grid1(n, g);
  auto sort_at = [&](int L) {   // Morton keys of level L, then a stable sort on their L d bits
    hipLaunchKernelGGL(k_point_keys, g, dim3(WG), 0, P.stream, d_points, n, d, T.origin[0], T.origin[1],
                       T.origin[2], T.inv, L, keys_in.as<uint64_t>(), idx_in.as<int>());
    IFMM_LAUNCH_CHECK();
    radix_sort_pairs(P.stream, keys_in.as<uint64_t>(), idx_in.as<int>(), keys_out.as<uint64_t>(), idx_out.as<int>(),
                     n, L * d, cnt.as<int>());
  };
  const int Lmax = d == 3 ? 20 : d == 2 ? 30 : 60;
  int L = depth;
  std::vector<uint64_t> hk;
  if (L <= 0) {
    const int Ltry = std::min(Lmax, 16);
    sort_at(Ltry);
    P.download(hk, keys_out.p, (size_t)n);
    L = -1;
    for (int cand = 2; cand <= Ltry && L < 0; ++cand) {
      const int sh = d * (Ltry - cand);
      int64_t run = 0, best = 0;
      for (int64_t i = 0; i < n; ++i) {
        run = (i > 0 && (hk[i] >> sh) == (hk[i - 1] >> sh)) ? run + 1 : 1;
        best = std::max(best, run);
      }
      if (best <= leaf_max) L = cand;
    }
    if (L < 0) L = Ltry;
  }
  if (L < 2 || L > Lmax) fail(IFMM_ERR_ARG, "depth must be in [2, " + std::to_string(Lmax) + "]");
  P.L = T.L = L;
  sort_at(L);
  P.download(hk, keys_out.p, (size_t)n);
  std::vector<int> hperm;
  P.download(hperm, idx_out.p, (size_t)n);
  T.perm.assign(hperm.begin(), hperm.end());
  plan_tree(T, hk);
  P.perm = std::move(idx_out);
  P.pts.alloc(sizeof(double) * n * d, &P.mem);
  hipLaunchKernelGGL(k_gather_points, g, dim3(WG), 0, P.stream, d_points, P.perm.as<int>(), n, d,
                     P.pts.as<double>());
  IFMM_LAUNCH_CHECK();
  P.upload(P.leaf_start, T.leaf_start);
  // device copies of the level tables
  P.ldev.clear();
  P.ldev.resize(L + 1);
  for (int l = 2; l <= L; ++l) {
    const HLevel& lv = T.lev[l];
    LevelDev& ld = P.ldev[l];
    ld.nb = lv.nb;
    P.upload(ld.coords, lv.coords);
    P.upload(ld.nb_start, lv.nb_start);
    P.upload(ld.nbr, lv.nbr);
    P.upload(ld.in_start, lv.in_start);
    P.upload(ld.inter, lv.inter);
    ld.npairs = (int64_t)lv.inter.size();
    if (l > 2) P.upload(ld.parent, lv.parent);
    if (l < L) P.upload(ld.ch_start, lv.ch_start);
    std::vector<int> cb(lv.nb);
    for (int i = 0; i < lv.nb; ++i) {
      int b = 0;
      for (int k = 0; k < d; ++k) b |= (lv.coords[(size_t)i * d + k] & 1) << k;
      cb[i] = b;
    }
    P.upload(ld.cbits, cb);
    // position of pair (j, i) in j's list, for every pair (i, j): the lists
    // are symmetric and sorted, so visiting i in increasing order meets the
    // entries of j's list in order (one cursor per box)
    std::vector<int> rev(lv.inter.size());
    std::vector<int> cur(lv.in_start.begin(), lv.in_start.end() - 1);
    for (int i = 0; i < lv.nb; ++i)
      for (int t = lv.in_start[i]; t < lv.in_start[i + 1]; ++t) {
        const int j = lv.inter[t];
        const int f = cur[j]++;
        IFMM_CHECK(f < lv.in_start[j + 1] && lv.inter[f] == i, "interaction lists not symmetric");
        rev[t] = f;
      }
    P.upload(ld.in_rev, rev);
  }
}

// ------------------------------------------------------------------- R1
inline void build_m2l_tiles(Problem& P);
inline void build_near_cache(Problem& P);

inline void build_r1(Problem& P) {
  const int d = P.d, q = P.q, L = P.L;
  const HTree& T = P.T;
  P.ubar.alloc(sizeof(double) * P.n * q, &P.mem);
  hipLaunchKernelGGL(k_leaf_ubar, dim3(T.lev[L].nb), dim3(WG), 0, P.stream, P.pts.as<double>(),
                     P.leaf_start.as<int64_t>(), P.ldev[L].coords.as<int>(), T.lev[L].nb, P.cc, T.origin[0],
                     T.origin[1], T.origin[2], T.box_size(L), P.ubar.as<double>());
  IFMM_LAUNCH_CHECK();
  // transfers, one per child position: T_b[m, m'] = l_{m'}(child node m in parent coordinates)
  std::vector<double> tt((size_t)(1 << d) * q * q);
  for (int b = 0; b < (1 << d); ++b)
    for (int m = 0; m < q; ++m) {
      double x[3];
      node_ref(P.cc, m, x);
      for (int k = 0; k < d; ++k) x[k] = 0.5 * x[k] + 0.5 * (((b >> k) & 1) ? 1.0 : -1.0);
      for (int mp = 0; mp < q; ++mp) tt[(size_t)b * q * q + m + (size_t)mp * q] = lagrange_nd(P.cc, mp, x);
    }
  P.upload(P.Ttab, tt);
  int c7 = 1;
  for (int k = 0; k < d; ++k) c7 *= 7;
  P.m2l.clear();
  P.m2l.resize(L + 1);
  for (int l = 2; l <= L; ++l) {
    P.m2l[l].alloc(sizeof(double) * c7 * q * q, &P.mem);
    hipLaunchKernelGGL(k_m2l_table, dim3(c7), dim3(WG), 0, P.stream, P.cc, P.kf, T.box_size(l),
                       P.m2l[l].as<double>());
    IFMM_LAUNCH_CHECK();
  }
  if (q > 32 && q <= M2L_QP) build_m2l_tiles(P);
  build_near_cache(P);
}

// Leaf near-field blocks, stored once when they fit NEAR_CACHE_MAX bytes and
// the leaves are small enough for the wavefront product (IFMM_NEAR_CACHE=0:
// never): every product with A~ or E then reads them instead of evaluating
// the kernel again.
constexpr int64_t NEAR_CACHE_MAX = (int64_t)16 << 30;

inline void build_near_cache(Problem& P) {
  const HTree& T = P.T;
  const int L = P.L, nb = T.lev[L].nb;
  const char* env = std::getenv("IFMM_NEAR_CACHE");
  if ((env && env[0] == '0') || P.n > (int64_t)WAVE * nb) return;
  const HLevel& lv = T.lev[L];
  for (int i = 0; i < nb; ++i)   // the product holds a box's neighbours one per lane
    if (lv.nb_start[i + 1] - lv.nb_start[i] > WAVE) return;
  std::vector<int64_t> off(nb);
  std::vector<int> col(lv.nbr.size());
  int64_t tot = 0;
  for (int i = 0; i < nb; ++i) {
    const int64_t m = T.leaf_start[i + 1] - T.leaf_start[i];
    int c = 0;
    for (int t = lv.nb_start[i]; t < lv.nb_start[i + 1]; ++t) {
      col[t] = c;
      const int j = lv.nbr[t];
      c += (int)(T.leaf_start[j + 1] - T.leaf_start[j]);
    }
    off[i] = tot;
    tot += m * c;
  }
  if (tot * (int64_t)sizeof(double) > NEAR_CACHE_MAX) return;
  P.upload(P.nfoff, off);
  P.upload(P.nfcol, col);
  P.nf.alloc(sizeof(double) * std::max<int64_t>(tot, 1), &P.mem);
  hipLaunchKernelGGL(k_near_fill, dim3((unsigned)ceil_div(nb, WG / WAVE)), dim3(WG), 0, P.stream, P.pts.as<double>(),
                     P.leaf_start.as<int64_t>(), P.ldev[L].nb_start.as<int>(), P.ldev[L].nbr.as<int>(), nb, P.d,
                     P.kf, P.nfoff.as<int64_t>(), P.nfcol.as<int>(), P.nf.as<double>());
  IFMM_LAUNCH_CHECK();
}

// Tables of the offset-tiled M2L and K_pre: for a box with child position b
// (bit k = coordinate k mod 2), the children of its parent's neighbours lie at
// offsets in [-2 - b_k, 3 - b_k] per axis; those outside [-1, 1]^d form its
// interaction offsets, listed in increasing 7^d code. bo holds, per box and
// offset, the position of that pair in the interaction-list CSR (-1: none).
inline void build_m2l_tiles(Problem& P) {
  const int d = P.d, L = P.L;
  const int nb2 = 1 << d;
  int c7 = 1, p6 = 1, p3 = 1;
  for (int k = 0; k < d; ++k) { c7 *= 7; p6 *= 6; p3 *= 3; }
  const int nofs = p6 - p3;
  P.m2l_nofs = nofs;
  std::vector<int> ocode, kof((size_t)nb2 * c7, -1);
  for (int b = 0; b < nb2; ++b) {
    int k = 0;
    for (int code = 0; code < c7; ++code) {
      bool in = true, near = true;
      for (int a = 0, x = code; a < d; ++a, x /= 7) {
        const int o = x % 7 - 3, bb = (b >> a) & 1;
        if (o < -2 - bb || o > 3 - bb) in = false;
        if (o < -1 || o > 1) near = false;
      }
      if (!in || near) continue;
      ocode.push_back(code);
      kof[(size_t)b * c7 + code] = k++;
    }
    if (k != nofs) fail(IFMM_ERR_INTERNAL, "interaction offsets of a child position");
  }
  P.upload(P.m2l_ocode, ocode);
  const HTree& T = P.T;
  for (int l = 2; l <= L; ++l) {
    const HLevel& lv = T.lev[l];
    LevelDev& ld = P.ldev[l];
    std::vector<int> cb(lv.nb), tord;
    for (int i = 0; i < lv.nb; ++i) {
      int b = 0;
      for (int a = 0; a < d; ++a) b |= (lv.coords[(size_t)i * d + a] & 1) << a;
      cb[i] = b;
    }
    ld.m2l_gstart.assign(nb2 + 1, 0);
    for (int b = 0; b < nb2; ++b) {
      ld.m2l_gstart[b] = (int)tord.size();
      for (int i = 0; i < lv.nb; ++i)
        if (cb[i] == b) tord.push_back(i);
    }
    ld.m2l_gstart[nb2] = (int)tord.size();
    std::vector<int> bo((size_t)lv.nb * nofs, -1);
    for (int i = 0; i < lv.nb; ++i)
      for (int t = lv.in_start[i]; t < lv.in_start[i + 1]; ++t) {
        const int j = lv.inter[t];
        int code = 0, mul = 1;
        for (int a = 0; a < d; ++a) {
          code += (lv.coords[(size_t)j * d + a] - lv.coords[(size_t)i * d + a] + 3) * mul;
          mul *= 7;
        }
        const int k = kof[(size_t)cb[i] * c7 + code];
        if (k < 0) fail(IFMM_ERR_INTERNAL, "an interaction pair outside its child position's offsets");
        bo[(size_t)i * nofs + k] = t;
      }
    P.upload(ld.m2l_tord, tord);
    ld.m2l_tord_h = tord;
    P.upload(ld.m2l_bo, bo);
  }
}

// Leaf output (L2P + P2P): a wavefront per box when the leaves are small (at
// most 64 points on average), a workgroup per box otherwise.
inline void launch_l2p_p2p(Problem& P, int nrhs, const double* ubar, const double* g, const double* x, int64_t ldx,
                           double* y, int64_t ldy, int with_far) {
  const HTree& T = P.T;
  const int L = P.L, nb = T.lev[L].nb;
  if (P.n <= (int64_t)WAVE * nb)
    hipLaunchKernelGGL(k_l2p_p2p_w, dim3((unsigned)ceil_div(nb, WG / WAVE)), dim3(WG), 0, P.stream,
                       P.pts.as<double>(), P.leaf_start.as<int64_t>(), P.ldev[L].nb_start.as<int>(),
                       P.ldev[L].nbr.as<int>(), nb, P.d, P.q, nrhs, P.kf, ubar, g, x, ldx, y, ldy, with_far,
                       P.nf.p ? P.nf.as<double>() : nullptr, P.nfoff.as<int64_t>(), P.nfcol.as<int>());
  else
    hipLaunchKernelGGL(k_l2p_p2p, dim3(nb), dim3(WG), 0, P.stream, P.pts.as<double>(), P.leaf_start.as<int64_t>(),
                       P.ldev[L].nb_start.as<int>(), P.ldev[L].nbr.as<int>(), nb, P.d, P.q, nrhs, P.kf, ubar, g, x,
                       ldx, y, ldy, with_far);
}

// g = M2L(w) at level l by offset tiles (the level has them, q and nrhs <= 64).
inline void launch_m2l_tile(Problem& P, int l, int nrhs, const double* w, double* g) {
  const int q = P.q, ng = 1 << P.d;
  const int tpw = M2L_QP / nrhs;   // targets per workgroup
  const auto& gs = P.ldev[l].m2l_gstart;
  M2LGroups gr{};
  int nwg = 0;
  for (int b = 0; b <= ng; ++b) {
    gr.start[b] = gs[b];
    gr.wg0[b] = nwg;
    if (b < ng) nwg += (int)ceil_div(gs[b + 1] - gs[b], tpw);
  }
  if (nwg > 0)
    hipLaunchKernelGGL(k_m2l_tile, dim3((unsigned)nwg), dim3(256), 0, P.stream, P.ldev[l].m2l_tord.as<int>(),
                       P.ldev[l].m2l_bo.as<int>(), P.ldev[l].inter.as<int>(), P.m2l_nofs, P.m2l_ocode.as<int>(), gr,
                       ng, tpw, q, nrhs, P.m2l[l].as<double>(), w, g);
  IFMM_LAUNCH_CHECK();
}

// y = A~ x (tree order in and out), nrhs columns; x, y device, leading dim n.
inline void matvec_tree(Problem& P, const double* x, double* y, int nrhs) {
  const int q = P.q, L = P.L, d = P.d;
  const HTree& T = P.T;
  if ((int)P.mv_w.size() != L + 1 || P.mv_nrhs < nrhs) {
    P.mv_w.clear();
    P.mv_g.clear();
    P.mv_w.resize(L + 1);
    P.mv_g.resize(L + 1);
    for (int l = 2; l <= L; ++l) {
      P.mv_w[l].alloc(sizeof(double) * T.lev[l].nb * q * nrhs, &P.mem);
      P.mv_g[l].alloc(sizeof(double) * T.lev[l].nb * q * nrhs, &P.mem);
    }
    P.mv_nrhs = nrhs;
  }
  hipLaunchKernelGGL(k_p2m, dim3(T.lev[L].nb), dim3(WG), 0, P.stream, P.ubar.as<double>(),
                     P.leaf_start.as<int64_t>(), T.lev[L].nb, q, x, P.n, nrhs, P.mv_w[L].as<double>());
  IFMM_LAUNCH_CHECK();
  for (int l = L - 1; l >= 2; --l) {
    hipLaunchKernelGGL(k_m2m, dim3(T.lev[l].nb), dim3(WG), 0, P.stream, P.ldev[l].ch_start.as<int>(),
                       P.ldev[l + 1].cbits.as<int>(), T.lev[l].nb, q, nrhs, P.Ttab.as<double>(),
                       P.mv_w[l + 1].as<double>(), P.mv_w[l].as<double>());
    IFMM_LAUNCH_CHECK();
  }
  for (int l = 2; l <= L; ++l) {
    const int* ist = P.ldev[l].in_start.as<int>();
    const int* itr = P.ldev[l].inter.as<int>();
    const int* crd = P.ldev[l].coords.as<int>();
    const int nbl = T.lev[l].nb;
    const double* tb = P.m2l[l].as<double>();
    // matrix cores for q <= 64 (orders up to 4 in 3D; offset tiles above q = 32), the vector kernel above that
    if (q <= 16)
      hipLaunchKernelGGL(k_m2l_mfma<1>, dim3(nbl), dim3(256), 0, P.stream, ist, itr, crd, nbl, d, q, nrhs, tb,
                         P.mv_w[l].as<double>(), P.mv_g[l].as<double>());
    else if (q <= 32)
      hipLaunchKernelGGL(k_m2l_mfma<2>, dim3(nbl), dim3(256), 0, P.stream, ist, itr, crd, nbl, d, q, nrhs, tb,
                         P.mv_w[l].as<double>(), P.mv_g[l].as<double>());
    else if (q <= M2L_QP && nrhs <= M2L_QP && !P.ldev[l].m2l_gstart.empty())
      launch_m2l_tile(P, l, nrhs, P.mv_w[l].as<double>(), P.mv_g[l].as<double>());
    else if (q <= 64)
      hipLaunchKernelGGL(k_m2l_mfma<4>, dim3(nbl), dim3(256), 0, P.stream, ist, itr, crd, nbl, d, q, nrhs, tb,
                         P.mv_w[l].as<double>(), P.mv_g[l].as<double>());
    else
      hipLaunchKernelGGL(k_m2l, dim3(nbl), dim3(WG), 0, P.stream, ist, itr, crd, nbl, d, q, nrhs, tb,
                         P.mv_w[l].as<double>(), P.mv_g[l].as<double>());
    IFMM_LAUNCH_CHECK();
  }
  for (int l = 3; l <= L; ++l) {
    hipLaunchKernelGGL(k_l2l, dim3(T.lev[l].nb), dim3(WG), 0, P.stream, P.ldev[l].parent.as<int>(),
                       P.ldev[l].cbits.as<int>(), T.lev[l].nb, q, nrhs, P.Ttab.as<double>(),
                       P.mv_g[l - 1].as<double>(), P.mv_g[l].as<double>());
    IFMM_LAUNCH_CHECK();
  }
  launch_l2p_p2p(P, nrhs, P.ubar.as<double>(), P.mv_g[L].as<double>(), x, P.n, y, P.n, 1);
  IFMM_LAUNCH_CHECK();
}

// ------------------------------------------------------------------- R2
struct R2Pre {                       // pre-rotation orthonormal operators (float64)
  std::vector<std::vector<int>> r;             // by level
  std::vector<std::vector<int64_t>> roff;      // R factor offsets (r_i x q)
  std::vector<std::vector<int64_t>> ppoff;     // by level l > 2: PU_pre(i) offsets
  std::vector<std::vector<int>> pld;           // its leading dimension
  std::vector<std::vector<int64_t>> kpoff;     // per pair offsets of K_pre
  std::vector<DevBuf> R, Kpre, dr, droff, dppoff, dpld, dkpoff;
  DevBuf Q;                                    // leaf bases, ubar layout
  DevBuf Pst;                                  // stacked Q of the transfer QRs (all levels)
};

__global__ void k_fill_valid(double* __restrict__ v, int nb, int q, const int* __restrict__ r, double a) {
  const int i = blockIdx.x;
  if (i >= nb) return;
  for (int m = threadIdx.x; m < q; m += WG) v[(int64_t)i * q + m] = m < r[i] ? a : 0.0;
}

inline double norm2(Problem& P, const double* v, int64_t n, DevBuf& part) {
  const int nb = (int)std::min<int64_t>(512, std::max<int64_t>(1, ceil_div(n, WG)));
  part.reserve(sizeof(double) * nb, &P.mem);
  hipLaunchKernelGGL(k_sumsq_partial, dim3(nb), dim3(WG), 0, P.stream, v, n, part.as<double>());
  IFMM_LAUNCH_CHECK();
  std::vector<double> h;
  P.download(h, part.p, (size_t)nb);
  double s = 0;
  for (double x : h) s += x;
  return std::sqrt(s);
}

constexpr int64_t WEIGHT_CHUNK = (int64_t)1 << 29;   // doubles of far-field block rows formed at a time (4 GiB)

inline double dot(Problem& P, const double* a, const double* b, int64_t n, DevBuf& part) {
  const int nb = (int)std::min<int64_t>(512, std::max<int64_t>(1, ceil_div(n, WG)));
  part.reserve(sizeof(double) * nb, &P.mem);
  hipLaunchKernelGGL(k_dot_partial, dim3(nb), dim3(WG), 0, P.stream, a, b, n, part.as<double>());
  IFMM_LAUNCH_CHECK();
  std::vector<double> h;
  P.download(h, part.p, (size_t)nb);
  double s = 0;
  for (double x : h) s += x;
  return s;
}

// Number of eigenvalues below x of the symmetric tridiagonal (diagonal a,
// off-diagonal b) by the Sturm sequence of its LDL^T pivots.
inline int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int c = 0;
  double d = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double off = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
    d = (a[i] - x) - (i > 0 ? off / d : 0.0);
    if (d == 0.0) d = -1e-300;
    if (d < 0) ++c;
  }
  return c;
}

// max |eigenvalue| of the symmetric tridiagonal: its smallest and largest
// eigenvalues by bisection inside the Gershgorin interval.
inline double tridiag_extreme_abs(const std::vector<double>& a, const std::vector<double>& b) {
  const size_t n = a.size();
  double lo = 0, hi = 0;
  for (size_t i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = i == 0 ? a[i] - r : std::min(lo, a[i] - r);
    hi = i == 0 ? a[i] + r : std::max(hi, a[i] + r);
  }
  auto kth = [&](int k) {   // the k-th smallest eigenvalue (0-based)
    double l = lo, h = hi;
    for (int t = 0; t < 200 && h - l > 1e-15 * std::max(std::fabs(l), std::fabs(h)); ++t) {
      const double m = 0.5 * (l + h);
      if (sturm_count(a, b, m) > k) h = m; else l = m;
    }
    return 0.5 * (l + h);
  };
  return std::max(std::fabs(kth(0)), std::fabs(kth((int)n - 1)));
}

inline void build_r2(Problem& P, double sigma0_override) {
  const int q = P.q, L = P.L;
  const HTree& T = P.T;
  R2Pre R;
  R.r.resize(L + 1);
  R.roff.resize(L + 1);
  R.ppoff.resize(L + 1);
  R.pld.resize(L + 1);
  R.kpoff.resize(L + 1);
  R.R.resize(L + 1);
  R.Kpre.resize(L + 1);
  R.dr.resize(L + 1);
  R.droff.resize(L + 1);
  R.dppoff.resize(L + 1);
  R.dpld.resize(L + 1);
  R.dkpoff.resize(L + 1);
  DevBuf dscr, work;
  QrScratch qrs;
  // ---- leaf QR
  {
    const HLevel& lv = T.lev[L];
    auto& r = R.r[L];
    auto& ro = R.roff[L];
    r.resize(lv.nb);
    ro.resize(lv.nb);
    int64_t tot = 0;
    for (int i = 0; i < lv.nb; ++i) {
      const int64_t m = T.leaf_start[i + 1] - T.leaf_start[i];
      r[i] = (int)std::min<int64_t>(m, q);
      ro[i] = tot;
      tot += (int64_t)r[i] * q;
    }
    R.R[L].alloc(sizeof(double) * tot, &P.mem);
    R.Q.alloc(sizeof(double) * P.n * q, &P.mem);
    IFMM_HIP(hipMemsetAsync(R.Q.p, 0, sizeof(double) * P.n * q, P.stream));
    work.alloc(sizeof(double) * P.n * q, &P.mem);
    IFMM_HIP(hipMemcpyAsync(work.p, P.ubar.p, sizeof(double) * P.n * q, hipMemcpyDeviceToDevice, P.stream));
    std::vector<QrDesc> qd(lv.nb);
    for (int i = 0; i < lv.nb; ++i) {
      const int64_t s = T.leaf_start[i], m = T.leaf_start[i + 1] - s;
      QrDesc& dd = qd[i];
      dd.A = work.as<double>() + s * q;
      dd.R = R.R[L].as<double>() + ro[i];
      dd.Q = R.Q.as<double>() + s * q;
      dd.M = (int)m; dd.N = q; dd.lda = (int)m; dd.ldr = r[i]; dd.ldq = (int)m; dd.pad = 0;
    }
    run_qr<double>(P, qd, dscr);
  }
  // ---- transfers: QR of the stacked R_c T_c, bottom-up
  std::vector<int64_t> pst_off(L + 1, 0);
  int64_t pst_tot = 0;
  std::vector<std::vector<int>> rows(L + 1);
  for (int l = L - 1; l >= 2; --l) {
    const HLevel& lv = T.lev[l];
    rows[l].resize(lv.nb);
    R.r[l].resize(lv.nb);
    for (int p = 0; p < lv.nb; ++p) {
      int s = 0;
      for (int c = lv.ch_start[p]; c < lv.ch_start[p + 1]; ++c) s += R.r[l + 1][c];
      rows[l][p] = s;
      R.r[l][p] = std::min(s, q);
      pst_tot += (int64_t)s * std::min(s, q);
    }
  }
  R.Pst.alloc(sizeof(double) * std::max<int64_t>(pst_tot, 1), &P.mem);
  int64_t pst_cur = 0;
  for (int l = L - 1; l >= 2; --l) {
    const HLevel& lv = T.lev[l];
    const HLevel& lc = T.lev[l + 1];
    auto& r = R.r[l];
    auto& ro = R.roff[l];
    ro.resize(lv.nb);
    int64_t rt = 0, mt = 0;
    std::vector<int64_t> moff(lv.nb);
    for (int p = 0; p < lv.nb; ++p) {
      ro[p] = rt;
      rt += (int64_t)r[p] * q;
      moff[p] = mt;
      mt += (int64_t)rows[l][p] * q;
    }
    R.R[l].alloc(sizeof(double) * std::max<int64_t>(rt, 1), &P.mem);
    work.reserve(sizeof(double) * std::max<int64_t>(mt, 1), &P.mem);
    GemmBatch gb;
    std::vector<int> cb(lc.nb);
    for (int c = 0; c < lc.nb; ++c) {
      int b = 0;
      for (int k = 0; k < P.d; ++k) b |= (lc.coords[(size_t)c * P.d + k] & 1) << k;
      cb[c] = b;
    }
    auto& ppo = R.ppoff[l + 1];
    auto& pl = R.pld[l + 1];
    ppo.assign(lc.nb, 0);
    pl.assign(lc.nb, 1);
    std::vector<QrDesc> qd(lv.nb);
    for (int p = 0; p < lv.nb; ++p) {
      int off = 0;
      const int rowsp = rows[l][p];
      for (int c = lv.ch_start[p]; c < lv.ch_start[p + 1]; ++c) {
        const int rc = R.r[l + 1][c];
        gb.add(R.R[l + 1].as<double>() + R.roff[l + 1][c], rc, 0, P.Ttab.as<double>() + (int64_t)cb[c] * q * q,
               q, 0, work.as<double>() + moff[p] + off, rowsp, rc, q, q, 1.0, 0.0);
        ppo[c] = pst_cur + off;
        pl[c] = rowsp;
        off += rc;
      }
      QrDesc& dd = qd[p];
      dd.A = work.as<double>() + moff[p];
      dd.R = R.R[l].as<double>() + ro[p];
      dd.Q = R.Pst.as<double>() + pst_cur;
      dd.M = rowsp; dd.N = q; dd.lda = rowsp; dd.ldr = r[p]; dd.ldq = rowsp; dd.pad = 0;
      pst_cur += (int64_t)rowsp * r[p];
    }
    run_gemm<double>(P, gb, dscr);
    run_qr<double>(P, qd, dscr);
  }
  // ---- device copies of ranks/offsets, K_pre blocks
  for (int l = 2; l <= L; ++l) {
    const HLevel& lv = T.lev[l];
    R.dr[l] = up(P, R.r[l]);
    R.droff[l] = up(P, R.roff[l]);
    if (l > 2) {
      R.dppoff[l] = up(P, R.ppoff[l]);
      R.dpld[l] = up(P, R.pld[l]);
    }
    auto& ko = R.kpoff[l];
    ko.resize(lv.inter.size());
    int64_t kt = 0;
    for (int i = 0; i < lv.nb; ++i)
      for (int t = lv.in_start[i]; t < lv.in_start[i + 1]; ++t) {
        ko[t] = kt;
        kt += (int64_t)R.r[l][i] * R.r[l][lv.inter[t]];
      }
    R.dkpoff[l] = up(P, ko);
    R.Kpre[l].alloc(sizeof(double) * std::max<int64_t>(kt, 1), &P.mem);
    if (!lv.inter.empty()) {
      int rmx = 0;
      for (int i = 0; i < lv.nb; ++i) rmx = std::max(rmx, R.r[l][i]);
      const int np = (int)lv.inter.size();
      if (!P.ldev[l].m2l_gstart.empty() && !force_streamed()) {   // offset tiles on the matrix cores
        const int nb2 = 1 << P.d;
        std::vector<int> tl;
        std::vector<KpreWg> wg;
        const auto& gs = P.ldev[l].m2l_gstart;
        const auto& tord = P.ldev[l].m2l_tord_h;
        for (int b = 0; b < nb2; ++b)
          for (int rb = 1; rb <= 4; ++rb) {
            const int per = rb == 1 ? 4 : rb == 2 ? 2 : 1;
            const int s0 = (int)tl.size();
            for (int x = gs[b]; x < gs[b + 1]; ++x)
              if ((R.r[l][tord[x]] + 15) / 16 == rb) tl.push_back(tord[x]);
            for (int x = s0; x < (int)tl.size(); x += per)
              wg.push_back({x, std::min(per, (int)tl.size() - x), rb, b});
          }
        DevBuf dtl = up(P, tl), dwg;
        P.upload(dwg, wg);
        double fl = 0;   // R_i K~ (r_i q^2 products) then times R_j^T (r_i q r_j), once per unordered pair
        for (int i = 0; i < lv.nb; ++i)
          for (int t = lv.in_start[i]; t < lv.in_start[i + 1]; ++t)
            if (lv.inter[t] > i) fl += 2.0 * R.r[l][i] * q * (q + R.r[l][lv.inter[t]]);
        P.kone_begin(KF_KPRE, fl);
        hipLaunchKernelGGL(k_kpre_tile, dim3((unsigned)wg.size()), dim3(256), 0, P.stream, dwg.as<KpreWg>(),
                           dtl.as<int>(), P.ldev[l].m2l_bo.as<int>(), P.ldev[l].inter.as<int>(),
                           P.ldev[l].in_rev.as<int>(), P.m2l_nofs,
                           P.m2l_ocode.as<int>(), q, P.m2l[l].as<double>(), R.R[l].as<double>(),
                           R.droff[l].as<int64_t>(), R.dr[l].as<int>(), R.Kpre[l].as<double>(),
                           R.dkpoff[l].as<int64_t>());
        IFMM_LAUNCH_CHECK();
        P.kone_end();
        P.sync();   // the launch tables are freed at the end of this scope
      } else if ((int64_t)rmx * q <= SWW)   // a wavefront per pair
        hipLaunchKernelGGL(k_kpre_w, dim3((unsigned)ceil_div(np, WG / WAVE)), dim3(WG), 0, P.stream,
                           P.ldev[l].in_start.as<int>(), P.ldev[l].inter.as<int>(), P.ldev[l].coords.as<int>(),
                           lv.nb, P.d, q, P.m2l[l].as<double>(), R.R[l].as<double>(), R.droff[l].as<int64_t>(),
                           R.dr[l].as<int>(), R.Kpre[l].as<double>(), R.dkpoff[l].as<int64_t>(), np);
      else
        hipLaunchKernelGGL(k_kpre, dim3((unsigned)np), dim3(WG), 0, P.stream, P.ldev[l].in_start.as<int>(),
                           P.ldev[l].inter.as<int>(), P.ldev[l].coords.as<int>(), lv.nb, P.d, q,
                           P.m2l[l].as<double>(), R.R[l].as<double>(), R.droff[l].as<int64_t>(), R.dr[l].as<int>(),
                           R.Kpre[l].as<double>(), R.dkpoff[l].as<int64_t>());
      IFMM_LAUNCH_CHECK();
    }
  }
  // ---- sigma_0: the largest eigenvalue magnitude of the symmetric E (Lanczos)
  const double t_s0 = now_ms();
  {
    std::vector<int64_t> zo(L + 1), yo(L + 1);
    int64_t tot = P.n;
    for (int l = L; l >= 2; --l) {
      zo[l] = tot;
      tot += (int64_t)T.lev[l].nb * q;
      yo[l] = tot;
      tot += (int64_t)T.lev[l].nb * q;
    }
    DevBuf v, w, part;
    v.alloc(sizeof(double) * tot, &P.mem);
    w.alloc(sizeof(double) * tot, &P.mem);
    // entries of a box beyond its rank are never written by E: keep them zero
    IFMM_HIP(hipMemsetAsync(w.p, 0, sizeof(double) * tot, P.stream));
    DevBuf ew, eg;   // w = R^T y and g = M2L(w) of one level
    {
      int nbmax = 0;
      for (int l = 2; l <= L; ++l) nbmax = std::max(nbmax, T.lev[l].nb);
      ew.alloc(sizeof(double) * (size_t)nbmax * q, &P.mem);
      eg.alloc(sizeof(double) * (size_t)nbmax * q, &P.mem);
    }
    std::vector<int> rmax(L + 1, 0);   // largest rank of each level (kernel choice of the y rows)
    for (int l = 2; l <= L; ++l)
      for (int x : R.r[l]) rmax[l] = std::max(rmax[l], x);
    auto applyE = [&](const double* in, double* out) {
      launch_l2p_p2p(P, 1, R.Q.as<double>(), in + zo[L], in, P.n, out, P.n, 1);
      IFMM_LAUNCH_CHECK();
      for (int l = L; l >= 2; --l) {
        const int nb = T.lev[l].nb;
        const bool leaf = l == L;
        hipLaunchKernelGGL(k_e_zrows, dim3(nb), dim3(WG), 0, P.stream, nb, q, R.dr[l].as<int>(), (int)leaf,
                           P.leaf_start.as<int64_t>(), R.Q.as<double>(), in,
                           leaf ? nullptr : P.ldev[l].ch_start.as<int>(),
                           leaf ? nullptr : R.Pst.as<double>(), leaf ? nullptr : R.dppoff[l + 1].as<int64_t>(),
                           leaf ? nullptr : R.dpld[l + 1].as<int>(), leaf ? nullptr : R.dr[l + 1].as<int>(),
                           leaf ? nullptr : in + yo[l + 1], in + yo[l], out + zo[l]);
        IFMM_LAUNCH_CHECK();
        const bool top = l == 2;
        if (!P.ldev[l].m2l_gstart.empty() && !T.lev[l].inter.empty()) {   // far field through the M2L tables
          hipLaunchKernelGGL(k_e_rty, dim3((unsigned)ceil_div(nb, WG / WAVE)), dim3(WG), 0, P.stream, nb, q,
                             R.dr[l].as<int>(), R.R[l].as<double>(), R.droff[l].as<int64_t>(), in + yo[l],
                             ew.as<double>());
          IFMM_LAUNCH_CHECK();
          launch_m2l_tile(P, l, 1, ew.as<double>(), eg.as<double>());
          hipLaunchKernelGGL(k_e_yrows_g, dim3((unsigned)ceil_div(nb, WG / WAVE)), dim3(WG), 0, P.stream, nb, q,
                             R.dr[l].as<int>(), R.R[l].as<double>(), R.droff[l].as<int64_t>(), eg.as<double>(),
                             in + zo[l], top ? nullptr : P.ldev[l].parent.as<int>(),
                             top ? nullptr : R.Pst.as<double>(), top ? nullptr : R.dppoff[l].as<int64_t>(),
                             top ? nullptr : R.dpld[l].as<int>(), top ? nullptr : R.dr[l - 1].as<int>(),
                             top ? nullptr : in + zo[l - 1], out + yo[l]);
          IFMM_LAUNCH_CHECK();
          continue;
        }
        hipLaunchKernelGGL(rmax[l] <= 32 ? k_e_yrows32 : k_e_yrows, dim3(nb), dim3(WG), 0, P.stream, nb, q,
                           R.dr[l].as<int>(),
                           P.ldev[l].in_start.as<int>(), P.ldev[l].inter.as<int>(), R.Kpre[l].as<double>(),
                           R.dkpoff[l].as<int64_t>(), in + zo[l], in + yo[l],
                           top ? nullptr : P.ldev[l].parent.as<int>(), top ? nullptr : R.Pst.as<double>(),
                           top ? nullptr : R.dppoff[l].as<int64_t>(), top ? nullptr : R.dpld[l].as<int>(),
                           top ? nullptr : R.dr[l - 1].as<int>(), top ? nullptr : in + zo[l - 1],
                           out + yo[l]);
        IFMM_LAUNCH_CHECK();
      }
    };
    if (sigma0_override > 0) {
      P.sigma0 = sigma0_override;
    } else {
      // Lanczos on the symmetric E from the all-ones vector (over the unknowns
      // that exist): q_{k+1} beta_k = E q_k - alpha_k q_k - beta_{k-1} q_{k-1};
      // sigma_0 = the largest Ritz value magnitude of the tridiagonal, stopped
      // when it changes by <= 1e-12 relatively (at most 300 steps)
      DevBuf u;
      u.alloc(sizeof(double) * tot, &P.mem);
      IFMM_HIP(hipMemsetAsync(v.p, 0, sizeof(double) * tot, P.stream));
      IFMM_HIP(hipMemsetAsync(u.p, 0, sizeof(double) * tot, P.stream));
      dim3 g;
      grid1(P.n, g);
      hipLaunchKernelGGL(k_fill, g, dim3(WG), 0, P.stream, v.as<double>(), P.n, 1.0);
      int64_t cnt = P.n;
      for (int l = L; l >= 2; --l) {
        for (int part_i = 0; part_i < 2; ++part_i)
          hipLaunchKernelGGL(k_fill_valid, dim3(T.lev[l].nb), dim3(WG), 0, P.stream,
                             v.as<double>() + (part_i ? yo[l] : zo[l]), T.lev[l].nb, q, R.dr[l].as<int>(), 1.0);
        for (int x : R.r[l]) cnt += 2 * x;
      }
      IFMM_LAUNCH_CHECK();
      dim3 gt;
      grid1(tot, gt);
      hipLaunchKernelGGL(k_scale, gt, dim3(WG), 0, P.stream, v.as<double>(), tot, 1.0 / std::sqrt((double)cnt));
      double* qk = v.as<double>();    // q_k
      double* qp = u.as<double>();    // q_{k-1}, then the next q
      double* wv = w.as<double>();
      std::vector<double> al, be;
      double beta = 0, theta = 0, theta_old = -1;
      int it = 0;
      for (it = 0; it < 300; ++it) {
        applyE(qk, wv);
        // w -= beta q_{k-1}; alpha = q_k . w; w -= alpha q_k
        hipLaunchKernelGGL(k_axpy, gt, dim3(WG), 0, P.stream, wv, (const double*)qp, tot, -beta);
        const double alpha = dot(P, qk, wv, tot, part);
        hipLaunchKernelGGL(k_axpy, gt, dim3(WG), 0, P.stream, wv, (const double*)qk, tot, -alpha);
        IFMM_LAUNCH_CHECK();
        al.push_back(alpha);
        theta = tridiag_extreme_abs(al, be);
        if (it > 0 && std::fabs(theta - theta_old) <= 1e-12 * theta) break;
        theta_old = theta;
        beta = norm2(P, wv, tot, part);
        if (beta == 0.0) break;
        be.push_back(beta);
        // q_{k-1} <- q_k, q_k <- w / beta
        hipLaunchKernelGGL(k_copy_scaled, gt, dim3(WG), 0, P.stream, qp, (const double*)wv, tot, 1.0 / beta);
        IFMM_LAUNCH_CHECK();
        std::swap(qk, qp);
      }
      P.sigma0 = theta;
      P.sigma0_estimated = theta;
      P.sigma0_iters = std::min(it + 1, 300);
    }
  }
  P.st.t_sigma0_ms = now_ms() - t_s0;
  P.tau = std::max(P.eps, 64.0 * (P.precision == 32 ? Prec<float>::u : Prec<double>::u)) * P.sigma0;

  // ---- weights, top-down
  std::vector<std::vector<int64_t>> woff(L + 1), soff(L + 1);
  std::vector<std::vector<int>> gcols(L + 1);
  std::vector<DevBuf> WU(L + 1), WV(L + 1), GU(L + 1), GV(L + 1), SU(L + 1), SV(L + 1), dwoff(L + 1),
      dgcols(L + 1);
  std::vector<std::vector<double>> hsu(L + 1), hsv(L + 1);
  for (int l = 2; l <= L; ++l) {
    const HLevel& lv = T.lev[l];
    const auto& r = R.r[l];
    woff[l].resize(lv.nb);
    soff[l].resize(lv.nb);
    gcols[l].resize(lv.nb);
    std::vector<int> mrows(lv.nb);
    std::vector<int64_t> moff(lv.nb);
    int64_t wt = 0, stt = 0, mt = 0;
    for (int i = 0; i < lv.nb; ++i) {
      int rw = 0;
      for (int t = lv.in_start[i]; t < lv.in_start[i + 1]; ++t) rw += r[lv.inter[t]];
      if (l > 2) rw += gcols[l - 1][lv.parent[i]];
      mrows[i] = rw;
      moff[i] = mt;
      mt += (int64_t)rw * r[i];
      woff[l][i] = wt;
      wt += (int64_t)r[i] * r[i];
      soff[l][i] = stt;
      stt += r[i];
      gcols[l][i] = std::min(rw, r[i]);
    }
    for (auto* b : {&WU[l], &WV[l], &GU[l], &GV[l]}) b->alloc(sizeof(double) * std::max<int64_t>(wt, 1), &P.mem);
    for (auto* b : {&SU[l], &SV[l]}) b->alloc(sizeof(double) * std::max<int64_t>(stt, 1), &P.mem);
    IFMM_HIP(hipMemsetAsync(SU[l].p, 0, sizeof(double) * std::max<int64_t>(stt, 1), P.stream));
    IFMM_HIP(hipMemsetAsync(SV[l].p, 0, sizeof(double) * std::max<int64_t>(stt, 1), P.stream));
    dwoff[l] = up(P, woff[l]);
    dgcols[l] = up(P, gcols[l]);
    DevBuf dm = up(P, moff), dmr = up(P, mrows);
    // the far-field block rows are formed and factorized in chunks of boxes of
    // at most WEIGHT_CHUNK doubles (their total reaches a hundred GB at 2^20 points)
    std::vector<int> cut(1, 0);
    for (int i = 0; i < lv.nb; ++i) {
      const int64_t sz = (int64_t)mrows[i] * r[i];
      if (i > cut.back() && moff[i] + sz - moff[cut.back()] > WEIGHT_CHUNK) cut.push_back(i);
    }
    cut.push_back(lv.nb);
    int64_t mchunk = 1;
    for (size_t c = 0; c + 1 < cut.size(); ++c)
      mchunk = std::max<int64_t>(mchunk, (cut[c + 1] < lv.nb ? moff[cut[c + 1]] : mt) - moff[cut[c]]);
    DevBuf Mw, Rw, Bw;
    Mw.alloc(sizeof(double) * mchunk, &P.mem);
    Rw.alloc(sizeof(double) * std::max<int64_t>(wt, 1), &P.mem);
    Bw.alloc(sizeof(double) * std::max<int64_t>(wt, 1), &P.mem);
    for (int side = 0; side < 2; ++side)
     for (size_t ch = 0; ch + 1 < cut.size(); ++ch) {
      const int i0 = cut[ch], i1 = cut[ch + 1];
      double* Mbase = Mw.as<double>() - moff[i0];   // Mbase + moff[i] lies in the chunk buffer for i in [i0, i1)
      DevBuf& G = side ? GV[l] : GU[l];
      DevBuf& W = side ? WV[l] : WU[l];
      DevBuf& S = side ? SV[l] : SU[l];
      hipLaunchKernelGGL(k_weight_rows, dim3((unsigned)(i1 - i0)), dim3(WG), 0, P.stream, P.ldev[l].in_start.as<int>(),
                         P.ldev[l].inter.as<int>(), nullptr, lv.nb, side, P.ldev[l].in_rev.as<int>(),
                         R.Kpre[l].as<double>(), R.dkpoff[l].as<int64_t>(), R.dr[l].as<int>(),
                         l > 2 ? P.ldev[l].parent.as<int>() : nullptr, R.Pst.as<double>(),
                         l > 2 ? R.dppoff[l].as<int64_t>() : nullptr, l > 2 ? R.dpld[l].as<int>() : nullptr,
                         l > 2 ? R.dr[l - 1].as<int>() : nullptr,
                         l > 2 ? (side ? GV[l - 1].as<double>() : GU[l - 1].as<double>()) : nullptr,
                         l > 2 ? dwoff[l - 1].as<int64_t>() : nullptr, l > 2 ? dgcols[l - 1].as<int>() : nullptr,
                         Mbase, dm.as<int64_t>(), dmr.as<int>(), i0);
      IFMM_LAUNCH_CHECK();
      std::vector<QrJob> qd;   // R only: the blocked Householder QR (panels, matrix-core updates)
      CopyBatch<double, double> tb;
      std::vector<SvdDesc> sd;
      CopyBatch<double, double> gbat;
      for (int i = i0; i < i1; ++i) {
        const int kq = gcols[l][i];
        if (kq == 0) continue;
        qd.push_back({Mbase + moff[i], Rw.as<double>() + woff[l][i], mrows[i], r[i], mrows[i], kq});
        // B = R^T (r_i x kq)
        tb.add(Rw.as<double>() + woff[l][i], kq, Bw.as<double>() + woff[l][i], r[i], r[i], kq, 4);
        SvdDesc s{};
        s.B = Bw.as<double>() + woff[l][i];
        s.U = W.as<double>() + woff[l][i];
        s.S = S.as<double>() + soff[l][i];
        s.M = r[i]; s.N = kq; s.ldb = r[i]; s.ldu = r[i];
        sd.push_back(s);
        gbat.add(W.as<double>() + woff[l][i], r[i], G.as<double>() + woff[l][i], r[i], r[i], kq, 0, 1.0,
                 S.as<double>() + soff[l][i]);
      }
      qr_blocked<double>(P, qd, qrs);
      run_copy(P, tb, dscr);
      run_svd<double>(P, sd, dscr);
      run_copy(P, gbat, dscr);
      P.sync();   // the chunk buffer is refilled by the next chunk
    }
    P.download(hsu[l], SU[l].p, (size_t)std::max<int64_t>(stt, 1));
    P.download(hsv[l], SV[l].p, (size_t)std::max<int64_t>(stt, 1));
  }
  // ---- ranks kept: sigma > tau, common count for U and V
  P.r2.clear();
  P.r2.resize(L + 1);
  for (int l = 2; l <= L; ++l) {
    const HLevel& lv = T.lev[l];
    auto& k = P.r2[l].k;
    k.resize(lv.nb);
    for (int i = 0; i < lv.nb; ++i) {
      int ku = 0, kv = 0;
      for (int a = 0; a < gcols[l][i]; ++a) {
        if (hsu[l][soff[l][i] + a] > P.tau) ++ku;
        if (hsv[l][soff[l][i] + a] > P.tau) ++kv;
      }
      int kk = std::max(ku, kv);
      if (P.rank_max > 0) kk = std::min(kk, P.rank_max);
      k[i] = kk;
    }
  }
  // ---- rotate and truncate
  std::vector<DevBuf> dk(L + 1);
  for (int l = 2; l <= L; ++l) dk[l] = up(P, P.r2[l].k);
  for (int l = 2; l <= L; ++l) {
    const HLevel& lv = T.lev[l];
    R2Level& z = P.r2[l];
    const auto& k = z.k;
    z.k_off.resize(lv.inter.size());
    int64_t kt = 0;
    for (int i = 0; i < lv.nb; ++i)
      for (int t = lv.in_start[i]; t < lv.in_start[i + 1]; ++t) {
        z.k_off[t] = kt;
        kt += (int64_t)k[i] * k[lv.inter[t]];
      }
    z.K.alloc(sizeof(double) * std::max<int64_t>(kt, 1), &P.mem);
    DevBuf dko = up(P, z.k_off);
    if (!lv.inter.empty()) {
      int kmx = 0, rmx = 0;
      for (int i = 0; i < lv.nb; ++i) {
        kmx = std::max(kmx, k[i]);
        rmx = std::max(rmx, R.r[l][i]);
      }
      const int np = (int)lv.inter.size();
      if ((int64_t)kmx * rmx <= SWW)   // a wavefront per pair
        hipLaunchKernelGGL(k_krot_w, dim3((unsigned)ceil_div(np, WG / WAVE)), dim3(WG), 0, P.stream,
                           P.ldev[l].in_start.as<int>(), P.ldev[l].inter.as<int>(), lv.nb, R.Kpre[l].as<double>(),
                           R.dkpoff[l].as<int64_t>(), R.dr[l].as<int>(), WU[l].as<double>(), WV[l].as<double>(),
                           dwoff[l].as<int64_t>(), dk[l].as<int>(), z.K.as<double>(), dko.as<int64_t>(), np);
      else
        hipLaunchKernelGGL(k_krot, dim3((unsigned)np), dim3(WG), 0, P.stream, P.ldev[l].in_start.as<int>(),
                           P.ldev[l].inter.as<int>(), lv.nb, R.Kpre[l].as<double>(), R.dkpoff[l].as<int64_t>(),
                           R.dr[l].as<int>(), WU[l].as<double>(), WV[l].as<double>(), dwoff[l].as<int64_t>(),
                           dk[l].as<int>(), z.K.as<double>(), dko.as<int64_t>());
      IFMM_LAUNCH_CHECK();
    }
    z.s_off.resize(lv.nb);
    int64_t st = 0;
    CopyBatch<double, double> cs;
    for (int i = 0; i < lv.nb; ++i) { z.s_off[i] = st; st += k[i]; }
    z.SU.alloc(sizeof(double) * std::max<int64_t>(st, 1), &P.mem);
    z.SV.alloc(sizeof(double) * std::max<int64_t>(st, 1), &P.mem);
    for (int i = 0; i < lv.nb; ++i) {
      cs.add(SU[l].as<double>() + soff[l][i], 1, z.SU.as<double>() + z.s_off[i], 1, k[i], 1);
      cs.add(SV[l].as<double>() + soff[l][i], 1, z.SV.as<double>() + z.s_off[i], 1, k[i], 1);
    }
    run_copy(P, cs, dscr);
    if (l > 2) {
      const auto& kp = P.r2[l - 1].k;
      z.p_off.resize(lv.nb);
      int64_t pt = 0;
      for (int i = 0; i < lv.nb; ++i) { z.p_off[i] = pt; pt += (int64_t)k[i] * kp[lv.parent[i]]; }
      z.PU.alloc(sizeof(double) * std::max<int64_t>(pt, 1), &P.mem);
      z.PV.alloc(sizeof(double) * std::max<int64_t>(pt, 1), &P.mem);
      DevBuf dpo = up(P, z.p_off);
      for (int side = 0; side < 2; ++side) {
        DevBuf& W = side ? WV[l] : WU[l];
        DevBuf& Wp = side ? WV[l - 1] : WU[l - 1];
        hipLaunchKernelGGL(k_prot, dim3(lv.nb), dim3(WG), 0, P.stream, P.ldev[l].parent.as<int>(), lv.nb,
                           R.Pst.as<double>(), R.dppoff[l].as<int64_t>(), R.dpld[l].as<int>(), R.dr[l].as<int>(),
                           R.dr[l - 1].as<int>(), W.as<double>(), dwoff[l].as<int64_t>(), Wp.as<double>(),
                           dwoff[l - 1].as<int64_t>(), dk[l].as<int>(), dk[l - 1].as<int>(),
                           side ? z.PV.as<double>() : z.PU.as<double>(), dpo.as<int64_t>());
        IFMM_LAUNCH_CHECK();
      }
    }
    if (l == L) {
      z.u_off.resize(lv.nb);
      int64_t ut = 0;
      for (int i = 0; i < lv.nb; ++i) {
        z.u_off[i] = ut;
        ut += (T.leaf_start[i + 1] - T.leaf_start[i]) * (int64_t)k[i];
      }
      z.U.alloc(sizeof(double) * std::max<int64_t>(ut, 1), &P.mem);
      z.V.alloc(sizeof(double) * std::max<int64_t>(ut, 1), &P.mem);
      GemmBatch gb;
      for (int i = 0; i < lv.nb; ++i) {
        const int64_t s = T.leaf_start[i];
        const int m = (int)(T.leaf_start[i + 1] - s);
        const int ri = R.r[L][i];
        gb.add(R.Q.as<double>() + s * q, m, 0, WU[l].as<double>() + woff[l][i], ri, 0,
               z.U.as<double>() + z.u_off[i], m, m, k[i], ri, 1.0, 0.0);
        gb.add(R.Q.as<double>() + s * q, m, 0, WV[l].as<double>() + woff[l][i], ri, 0,
               z.V.as<double>() + z.u_off[i], m, m, k[i], ri, 1.0, 0.0);
      }
      run_gemm<double>(P, gb, dscr);
    }
  }
  P.sync();
  if (debug_on()) {
    for (int l = 2; l <= L; ++l) {
      const R2Level& z = P.r2[l];
      int64_t ks = 0;
      int kmax = 0;
      for (int x : z.k) { ks += x; kmax = std::max(kmax, x); }
      std::fprintf(stderr, "[ifmm] level %d: boxes %d sum k %lld max k %d\n", l, T.lev[l].nb, (long long)ks, kmax);
      dbg_dump<double>(P, "SU", z.SU.p, z.s_off.empty() ? 0 : (size_t)(z.s_off.back() + z.k.back()));
      dbg_dump<double>(P, "WU box0", WU[l].p, (size_t)R.r[l][0] * R.r[l][0]);
      dbg_dump<double>(P, "sU box0", SU[l].p, (size_t)R.r[l][0]);
      dbg_dump<double>(P, "K", z.K.p, z.K.bytes / sizeof(double));
      if (l == L) dbg_dump<double>(P, "U", z.U.p, z.U.bytes / sizeof(double));
    }
  }
}

}  // namespace ifmm
