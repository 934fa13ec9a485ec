// Kernels of one colour-class phase of the elimination (Alg. 2 and 3):
// gather of the pivot blocks, near-field fill scatter, gather of the
// recompression matrices, rank decision, basis change of every edge of a
// recompressed box, redirection of well-separated fill through K.
#pragma once

#include "linalg.hpp"

namespace ifmm {

// Node of the set F of one elimination: x~_j (type 0) or y_h (type 1).
struct FNode {
  int type, box, dim, off;
  int64_t src_row;   // pool offset of E(P rows, node): S(i,j) or XY(i,h); -1: the -I of y_i
  int64_t src_col;   // pool offset of E(node, P cols): S(j,i) or YX(h,i); -1: the -I of y_i
  int ld_row, ld_col;
};

struct ElimDesc {
  int box, m, r, p, f, nF, F0, pad;
  int64_t lu, w, epf, efp, xi, piv, dlt;   // class arena (lu, w, epf, efp, xi), int arena (piv), workspace (dlt)
  int64_t h, wx;                      // solve store: H = [A; G] ((m + f) x m), W_x (m x f)
  int64_t S, U, V;                    // pool offsets of S(i,i), U_i, V_i (ld m_i)
};

// Level tables shared by the kernels (device pointers).
struct LevelView {
  int nb, d, c7, c3, haspar;
  const int* coords;
  const int* m;        // x~ sizes
  const int* cap;      // rank capacity (leading dimension of y rows)
  int* r;              // committed ranks
  int* rnew;           // ranks after this phase's recompressions
  const int64_t* Kt;   // nb x 7^d pool offsets of K(i, box at offset), -1 if none
  const int* B7;       // nb x 7^d box ids at each offset, -1 if none
  const int64_t* St;   // nb x 3^d pool offsets of S(i, j)
  const int64_t* XYt;  // nb x 3^d pool offsets of XY(j, h)
  const int64_t* YXt;  // nb x 3^d pool offsets of YX(h, j)
  const int64_t* Uo;   // per box: U_i, V_i (m_i x cap_i, ld m_i), SU_i, SV_i (cap_i), PU_i, PV_i (cap_i x rpar, ld cap_i)
  const int64_t* Vo;
  const int64_t* SUo;
  const int64_t* SVo;
  const int64_t* PUo;
  const int64_t* PVo;
  const int* rpar;     // rank of the parent (columns of PU/PV)
  const int* parent;
};

__device__ inline int code7(const int* coords, int d, int i, int j) {
  int code = 0, mul = 1;
  for (int k = 0; k < d; ++k) {
    const int dd = coords[j * d + k] - coords[i * d + k];
    if (dd > 3 || dd < -3) return -1;
    code += (dd + 3) * mul;
    mul *= 7;
  }
  return code;
}

__device__ inline int code3(const int* coords, int d, int i, int j) {
  int code = 0, mul = 1;
  for (int k = 0; k < d; ++k) {
    const int dd = coords[j * d + k] - coords[i * d + k];
    if (dd > 1 || dd < -1) return -1;
    code += (dd + 1) * mul;
    mul *= 3;
  }
  return code;
}

// ---------------------------------------------------------------- gather
// blockIdx.x: elimination; blockIdx.y: F node (y == nF: the pivot block).
template <class T>
__global__ void __launch_bounds__(WG) k_gather(const ElimDesc* __restrict__ es, const FNode* __restrict__ Fs,
                                               const T* __restrict__ pool, T* __restrict__ arena) {
  const ElimDesc e = es[blockIdx.x];
  const int a = blockIdx.y;
  if (a > e.nF) return;
  const int m = e.m, r = e.r, p = e.p, f = e.f;
  T* EPP = arena + e.lu;
  T* EPF = arena + e.epf;
  T* EFP = arena + e.efp;
  if (a == e.nF) {
    for (int t = threadIdx.x; t < p * p; t += WG) {
      const int i = t % p, j = t / p;
      T v = 0;
      if (i < m && j < m) v = pool[e.S + i + (int64_t)j * m];
      else if (i < m) v = pool[e.U + i + (int64_t)(j - m) * m];
      else if (j < m) v = pool[e.V + j + (int64_t)(i - m) * m];
      EPP[i + (int64_t)j * p] = v;
    }
    return;
  }
  const FNode nd = Fs[e.F0 + a];
  const int dim = nd.dim;
  // columns off..off+dim of E_PF (p rows)
  for (int t = threadIdx.x; t < p * dim; t += WG) {
    const int i = t % p, c = t / p;
    T v = 0;
    if (nd.src_row < 0) v = (i - m == c) ? (T)-1 : (T)0;
    else if (i < m) v = pool[nd.src_row + i + (int64_t)c * nd.ld_row];
    EPF[i + (int64_t)(nd.off + c) * p] = v;
  }
  // rows off..off+dim of E_FP (p columns, leading dimension f)
  for (int t = threadIdx.x; t < dim * p; t += WG) {
    const int i = t % dim, j = t / dim;
    T v = 0;
    if (nd.src_col < 0) v = (j - m == i) ? (T)-1 : (T)0;
    else if (j < m) v = pool[nd.src_col + i + (int64_t)j * nd.ld_col];
    EFP[(nd.off + i) + (int64_t)j * f] = v;
  }
  (void)r;
}

// ------------------------------------------------------------ near scatter
// blockIdx.x: elimination; blockIdx.y: pair index a * nF + b. Adds the fill
// block D(a, b) to its edge when the pair is near (Alg. 2, "add the fill-ins").
template <class T>
__global__ void __launch_bounds__(WG) k_near_scatter(const ElimDesc* __restrict__ es, const FNode* __restrict__ Fs,
                                                     LevelView lv, const T* __restrict__ work, T* __restrict__ pool) {
  const ElimDesc e = es[blockIdx.x];
  const int pr = blockIdx.y;
  if (pr >= e.nF * e.nF) return;
  const FNode A = Fs[e.F0 + pr / e.nF];
  const FNode B = Fs[e.F0 + pr % e.nF];
  if (A.dim == 0 || B.dim == 0) return;
  int64_t dst = -1;
  int ld = 0;
  if (A.type == 1 && B.type == 1) {
    const int c = code7(lv.coords, lv.d, A.box, B.box);
    dst = lv.Kt[(int64_t)A.box * lv.c7 + c];
    ld = lv.cap[A.box];
  } else {
    const int c = code3(lv.coords, lv.d, A.box, B.box);
    if (c < 0) return;   // well separated: compressed and redirected instead
    if (A.type == 0 && B.type == 0) { dst = lv.St[(int64_t)A.box * lv.c3 + c]; ld = lv.m[A.box]; }
    else if (A.type == 0) { dst = lv.XYt[(int64_t)A.box * lv.c3 + c]; ld = lv.m[A.box]; }
    else { dst = lv.YXt[(int64_t)A.box * lv.c3 + c]; ld = lv.cap[A.box]; }
  }
  if (dst < 0) return;
  const T* D = work + e.dlt;
  for (int t = threadIdx.x; t < A.dim * B.dim; t += WG) {
    const int i = t % A.dim, j = t / A.dim;
    pool[dst + i + (int64_t)j * ld] += D[(A.off + i) + (int64_t)(B.off + j) * e.f];
  }
}

// ----------------------------------------------------- recompression input
// One recompression per affected box j (a not-yet-eliminated neighbour with
// well-separated fill): MU^T = [U_j Sigma_U | D(x_j, ws)]^T and
// MV^T = [V_j Sigma_V | D(ws, x_j)^T]^T (eqs. U_j_recomp and V_j_recomp,
// aggregated over all well-separated partners of this elimination).
struct CompDesc {
  int box, elim, a, ncols;     // affected box, elimination index, F index of x_j, columns of MU
  int64_t mu, mv;              // workspace offsets of MU^T, MV^T (ncols x m_j, ld ncols)
  int64_t ru, rv;              // workspace offsets of R factors / B = R^T (m_j x kq)
  int64_t uu, vv;              // workspace offsets of the left singular vectors (m_j x kq, ld m_j)
  int64_t su, sv;              // workspace offsets of the singular values (kq)
  int64_t tr, tt;              // workspace offsets of r_j (k x r, ld ldt) and t_j
  int64_t pu, pv;              // workspace offsets of the pivoted-QR row permutations (m_j ints + count)
  int kq, ldt;                 // kq = min(ncols, m_j) bounds the new rank; ldt = max(kq, 1)
};

constexpr int COMP_ROWS = 32;   // rows of a recompression matrix gathered by one workgroup

template <class T>
__global__ void __launch_bounds__(WG) k_comp_gather(const CompDesc* __restrict__ cs, const ElimDesc* __restrict__ es,
                                                    const FNode* __restrict__ Fs, LevelView lv,
                                                    const T* __restrict__ pool, T* __restrict__ work) {
  const CompDesc c = cs[blockIdx.x];
  const int j = c.box;
  const int mj = lv.m[j], rj = lv.r[j];
  // blockIdx.y: rows (of MU^T, MV^T) r0 .. r0 + COMP_ROWS - 1 of this matrix
  const int r0 = blockIdx.y * COMP_ROWS;
  if (r0 >= mj) return;
  const int nr = min(COMP_ROWS, mj - r0);
  T* MU = work + c.mu;
  T* MV = work + c.mv;
  const int nc = c.ncols;
  const T* U = pool + lv.Uo[j];
  const T* V = pool + lv.Vo[j];
  const T* SU = pool + lv.SUo[j];
  const T* SV = pool + lv.SVo[j];
  for (int t = threadIdx.x; t < rj * nr; t += WG) {
    const int col = t % rj, row = r0 + t / rj;
    MU[col + (int64_t)row * nc] = U[row + (int64_t)col * mj] * SU[col];
    MV[col + (int64_t)row * nc] = V[row + (int64_t)col * mj] * SV[col];
  }
  if (c.elim < 0) return;   // recompression of merged bases: no fill columns
  const ElimDesc e = es[c.elim];
  const FNode X = Fs[e.F0 + c.a];
  const T* D = work + e.dlt;
  int o = rj;
  for (int b = 0; b < e.nF; ++b) {
    const FNode B = Fs[e.F0 + b];
    if (code3(lv.coords, lv.d, j, B.box) >= 0) continue;   // near: not compressed
    for (int t = threadIdx.x; t < B.dim * nr; t += WG) {
      const int col = t % B.dim, row = r0 + t / B.dim;
      MU[(o + col) + (int64_t)row * nc] = D[(X.off + row) + (int64_t)(B.off + col) * e.f];
      MV[(o + col) + (int64_t)row * nc] = D[(B.off + col) + (int64_t)(X.off + row) * e.f];
    }
    o += B.dim;
  }
}

// Rank kept: sigma > tau on each side, the larger count, capped by capacity.
template <class T>
__global__ void k_comp_rank(const CompDesc* __restrict__ cs, int nc, LevelView lv, const T* __restrict__ work,
                            double tau, int rank_max) {
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t >= nc) return;
  const CompDesc c = cs[t];
  int ku = 0, kv = 0;
  for (int a = 0; a < c.kq; ++a) {
    if ((double)work[c.su + a] > tau) ++ku;
    if ((double)work[c.sv + a] > tau) ++kv;
  }
  int k = ku > kv ? ku : kv;
  if (rank_max > 0 && k > rank_max) k = rank_max;
  lv.rnew[c.box] = k;   // the host grows the box's capacity to k before the basis changes
}

// The common rank k may exceed the number of resolved singular directions of
// one side (singular values at or below good_level, the level under which the
// SVD neither orthogonalises nor keeps columns). Such columns are replaced by
// an orthonormal completion: each new column is the unit vector e_i with the
// largest component outside the columns kept so far (1 - sum_a U[i, a]^2 is
// largest), orthogonalised twice against them and normalised; its singular
// value is 0. blockIdx.y = side (0: U, 1: V).
constexpr size_t COMPLETE_LDS_MAX = 144 * 1024;   // dynamic LDS of k_comp_complete: m_j + k values

template <class T>
__global__ void __launch_bounds__(WG) k_comp_complete(const CompDesc* __restrict__ cs, LevelView lv,
                                                      T* __restrict__ work, double good_level) {
  extern __shared__ unsigned char cc_dyn[];
  const CompDesc c0 = cs[blockIdx.x];
  T* v = reinterpret_cast<T*>(cc_dyn);      // m_j values
  T* coef = v + lv.m[c0.box];               // k values
  __shared__ T red[WG / WAVE];
  __shared__ T bv[WG / WAVE];
  __shared__ int bi[WG / WAVE];
  __shared__ int pick;
  const CompDesc c = cs[blockIdx.x];
  const int mj = lv.m[c.box], k = lv.rnew[c.box];
  T* U = work + (blockIdx.y ? c.vv : c.uu);
  T* S = work + (blockIdx.y ? c.sv : c.su);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  int g = 0;
  while (g < k && (double)S[g] > good_level) ++g;
  for (int col = g; col < k; ++col) {
    // the unit vector least represented in the kept columns
    T best = (T)-1;
    int besti = 0;
    for (int i = threadIdx.x; i < mj; i += WG) {
      T s = 0;
      for (int a = 0; a < col; ++a) { const T x = U[i + (int64_t)a * mj]; s += x * x; }
      if ((T)1 - s > best) { best = (T)1 - s; besti = i; }
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const T ob = __shfl_xor(best, o, WAVE);
      const int oi = __shfl_xor(besti, o, WAVE);
      if (ob > best || (ob == best && oi < besti)) { best = ob; besti = oi; }
    }
    if (lane == 0) { bv[w] = best; bi[w] = besti; }
    __syncthreads();
    if (threadIdx.x == 0) {
      T b = bv[0];
      int i0 = bi[0];
      for (int q = 1; q < WG / WAVE; ++q)
        if (bv[q] > b || (bv[q] == b && bi[q] < i0)) { b = bv[q]; i0 = bi[q]; }
      pick = i0;
    }
    __syncthreads();
    const int j = pick;
    for (int i = threadIdx.x; i < mj; i += WG) v[i] = i == j ? (T)1 : (T)0;
    __syncthreads();
    for (int pass = 0; pass < 2; ++pass) {
      for (int a = threadIdx.x; a < col; a += WG) {
        T s = 0;
        for (int i = 0; i < mj; ++i) s += U[i + (int64_t)a * mj] * v[i];
        coef[a] = s;
      }
      __syncthreads();
      for (int i = threadIdx.x; i < mj; i += WG) {
        T s = v[i];
        for (int a = 0; a < col; ++a) s -= U[i + (int64_t)a * mj] * coef[a];
        v[i] = s;
      }
      __syncthreads();
    }
    T s2 = 0;
    for (int i = threadIdx.x; i < mj; i += WG) s2 += v[i] * v[i];
    const T nrm = sqrt(block_sum(s2, red));
    const T inv = nrm > (T)0 ? (T)1 / nrm : (T)0;
    for (int i = threadIdx.x; i < mj; i += WG) U[i + (int64_t)col * mj] = v[i] * inv;
    if (threadIdx.x == 0) S[col] = (T)0;
    __syncthreads();
  }
}

// r_j = Uhat^T U_j and t_j = Vhat^T V_j (k x r_old, ld cap_j).
template <class T>
__global__ void __launch_bounds__(WG) k_comp_rt(const CompDesc* __restrict__ cs, LevelView lv,
                                                const T* __restrict__ pool, T* __restrict__ work) {
  const CompDesc c = cs[blockIdx.x];
  const int j = c.box;
  const int mj = lv.m[j], r = lv.r[j], k = lv.rnew[j], cap = lv.cap[j];
  const T* U = pool + lv.Uo[j];
  const T* V = pool + lv.Vo[j];
  const T* Uh = work + c.uu;
  const T* Vh = work + c.vv;
  for (int t = threadIdx.x; t < k * r; t += WG) {
    const int a = t % k, b = t / k;
    T su = 0, sv = 0;
    for (int i = 0; i < mj; ++i) {
      su += Uh[i + (int64_t)a * mj] * U[i + (int64_t)b * mj];
      sv += Vh[i + (int64_t)a * mj] * V[i + (int64_t)b * mj];
    }
    work[c.tr + a + (int64_t)b * c.ldt] = su;
    work[c.tt + a + (int64_t)b * c.ldt] = sv;
  }
}

constexpr int XF_CHUNK = 32;        // columns (rows) of an edge transformed at a time, at most
constexpr int XF_LDS = 32 * 1024;   // bytes of LDS for the staged edge slice (256-thread variant)
constexpr int XF_SMALL_R = 32;      // ranks up to this use 64-thread workgroups with 8 KB of LDS

// Row transform of every y-y edge of an affected box j and of its transfers:
// K(j, q) <- r_j K(j, q), PU(j) <- r_j PU(j), PV(j) <- t_j PV(j)
// (eqs. K_jq_update, U_parent_j_update, V_parent_j_update).
// Edges of the affected boxes, one workgroup each: pre[ci] is the first
// workgroup of recompression ci (prefix over the recompressions of the number
// of edges of their box, + 2 for PU / PV above level 2); estart / elist list
// the offset codes of a box's existing edges (CSR over the level's boxes).
struct XfTasks {
  const int* pre;
  int ncs, extra;            // extra: 2 for the parent transfers (row transform above level 2), else 0
  const int* estart;
  const int* elist;
};

__device__ inline int2 xf_task(const XfTasks& x, const CompDesc* __restrict__ cs, int c7) {
  int lo = 0, hi = x.ncs - 1;
  const int b = blockIdx.x;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (x.pre[mid] <= b) lo = mid; else hi = mid - 1;
  }
  const int j = cs[lo].box;
  const int local = b - x.pre[lo];
  const int ne = x.estart[j + 1] - x.estart[j];
  return make_int2(lo, local < ne ? x.elist[x.estart[j] + local] : c7 + (local - ne));
}

// One workgroup per existing edge (code c7 = PU, c7 + 1 = PV).
// A slice of up to XF_CHUNK columns of the edge is staged in LDS; each thread
// computes one output row of the slice, reading its row of the transform once.
template <class T, int BS, int LDSB>
__global__ void __launch_bounds__(BS) k_row_xform(const CompDesc* __restrict__ cs, XfTasks xt, LevelView lv,
                                                  T* __restrict__ pool, const T* __restrict__ work) {
  const int2 tk = xf_task(xt, cs, lv.c7);
  const CompDesc c = cs[tk.x];
  const int j = c.box;
  const int code = tk.y;
  int64_t off;
  int cols;
  const T* X;
  if (code < lv.c7) {
    off = lv.Kt[(int64_t)j * lv.c7 + code];
    if (off < 0) return;
    cols = lv.r[lv.B7[(int64_t)j * lv.c7 + code]];
    X = work + c.tr;
  } else {
    if (!lv.haspar) return;
    off = code == lv.c7 ? lv.PUo[j] : lv.PVo[j];
    cols = lv.rpar[j];
    X = work + (code == lv.c7 ? c.tr : c.tt);
  }
  const int r = lv.r[j], k = lv.rnew[j], cap = lv.cap[j];
  if (r == 0 || cols == 0) {
    for (int t = threadIdx.x; t < k * cols; t += BS) pool[off + t % k + (int64_t)(t / k) * cap] = (T)0;
    return;
  }
  __shared__ T sh[LDSB / sizeof(T)];
  const int wmax = min(XF_CHUNK, (int)(LDSB / sizeof(T)) / r);   // r <= 1024: at least 8 columns (FP64)
  T* E = pool + off;
  for (int c0 = 0; c0 < cols; c0 += wmax) {
    const int nc = min(wmax, cols - c0);
    for (int t = threadIdx.x; t < r * nc; t += BS) {
      const int i = t % r, cc = t / r;
      sh[i + cc * r] = E[i + (int64_t)(c0 + cc) * cap];
    }
    __syncthreads();
    for (int i = threadIdx.x; i < k; i += BS) {
      T acc[XF_CHUNK];
#pragma unroll
      for (int cc = 0; cc < XF_CHUNK; ++cc) acc[cc] = 0;
      for (int b = 0; b < r; ++b) {
        const T x = X[i + (int64_t)b * c.ldt];
#pragma unroll
        for (int cc = 0; cc < XF_CHUNK; ++cc)
          if (cc < nc) acc[cc] += x * sh[b + cc * r];
      }
#pragma unroll
      for (int cc = 0; cc < XF_CHUNK; ++cc)
        if (cc < nc) E[i + (int64_t)(c0 + cc) * cap] = acc[cc];
    }
    __syncthreads();
  }
}

// Column transform: K(q, j) <- K(q, j) t_j^T for every edge into y_j (eq. K_qj_update).
// One workgroup per existing edge K(q, j) (code: offset of q from j).
// A slice of up to XF_CHUNK rows of the edge is staged in LDS; each thread
// computes one output column of the slice, reading its row of t_j once.
template <class T, int BS, int LDSB>
__global__ void __launch_bounds__(BS) k_col_xform(const CompDesc* __restrict__ cs, XfTasks xt, LevelView lv,
                                                  T* __restrict__ pool, const T* __restrict__ work) {
  const int2 tk = xf_task(xt, cs, lv.c7);
  const CompDesc c = cs[tk.x];
  const int j = c.box;
  const int code = tk.y;
  const int qb = lv.B7[(int64_t)j * lv.c7 + code];
  if (qb < 0) return;
  const int back = lv.c7 - 1 - code;   // offset of j seen from q
  const int64_t off = lv.Kt[(int64_t)qb * lv.c7 + back];
  if (off < 0) return;
  const int rows = lv.rnew[qb], r = lv.r[j], k = lv.rnew[j];
  const int ldq = lv.cap[qb], capj = lv.cap[j];
  const T* X = work + c.tt;
  T* E = pool + off;
  if (r == 0 || rows == 0) {
    for (int t = threadIdx.x; t < rows * k; t += BS) E[t % rows + (int64_t)(t / rows) * ldq] = (T)0;
    return;
  }
  __shared__ T sh[LDSB / sizeof(T)];
  const int hmax = min(XF_CHUNK, (int)(LDSB / sizeof(T)) / r);
  for (int r0 = 0; r0 < rows; r0 += hmax) {
    const int nr = min(hmax, rows - r0);
    for (int t = threadIdx.x; t < nr * r; t += BS) {
      const int i = t % nr, b = t / nr;
      sh[i + b * hmax] = E[(r0 + i) + (int64_t)b * ldq];
    }
    __syncthreads();
    for (int a = threadIdx.x; a < k; a += BS) {
      T acc[XF_CHUNK];
#pragma unroll
      for (int ii = 0; ii < XF_CHUNK; ++ii) acc[ii] = 0;
      for (int b = 0; b < r; ++b) {
        const T x = X[a + (int64_t)b * c.ldt];
#pragma unroll
        for (int ii = 0; ii < XF_CHUNK; ++ii)
          if (ii < nr) acc[ii] += sh[ii + b * hmax] * x;
      }
#pragma unroll
      for (int ii = 0; ii < XF_CHUNK; ++ii)
        if (ii < nr) E[(r0 + ii) + (int64_t)a * ldq] = acc[ii];
    }
    __syncthreads();
  }
}

// LDS writes of a wavefront visible to its other lanes (and the slot free for reuse).
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int XF_BOX_R = 32;   // per-box basis changes when every capacity of the level is at most this

// Fine levels (every capacity at most XF_BOX_R): one workgroup per recompressed
// box j for all of its row transforms K(j, q) <- r_j K(j, q) and PU, PV. The
// transforms (r_j, and t_j for PV) are staged in LDS once; each wavefront takes
// every fourth edge, stages it in its own LDS slot (the product is written back
// in place) and writes the k x cols result.
template <class T>
__global__ void __launch_bounds__(256) k_row_xform_box(const CompDesc* __restrict__ cs, XfTasks xt, LevelView lv,
                                                       T* __restrict__ pool, const T* __restrict__ work) {
  constexpr int R = XF_BOX_R;
  __shared__ T Xr[R * R], Xt[R * R];
  __shared__ T slot[4][R * R];
  const CompDesc c = cs[blockIdx.x];
  const int j = c.box;
  const int r = lv.r[j], k = lv.rnew[j], cap = lv.cap[j];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  for (int e = threadIdx.x; e < k * r; e += 256) {
    const int i = e % k, b = e / k;
    Xr[i + b * R] = work[c.tr + i + (int64_t)b * c.ldt];
    Xt[i + b * R] = work[c.tt + i + (int64_t)b * c.ldt];
  }
  __syncthreads();
  const int e0 = xt.estart[j], ne = xt.estart[j + 1] - e0;
  T* S = slot[wv];
  for (int t = wv; t < ne + xt.extra; t += 4) {
    int64_t off;
    int cols;
    const T* X = Xr;
    if (t < ne) {
      const int code = xt.elist[e0 + t];
      off = lv.Kt[(int64_t)j * lv.c7 + code];
      if (off < 0) continue;
      cols = lv.r[lv.B7[(int64_t)j * lv.c7 + code]];
    } else {
      if (!lv.haspar) continue;
      off = t == ne ? lv.PUo[j] : lv.PVo[j];
      cols = lv.rpar[j];
      if (t != ne) X = Xt;
    }
    T* E = pool + off;
    if (r == 0 || cols == 0) {
      for (int e = lane; e < k * cols; e += WAVE) E[e % k + (int64_t)(e / k) * cap] = (T)0;
      continue;
    }
    for (int e = lane; e < r * cols; e += WAVE) S[e] = E[e % r + (int64_t)(e / r) * cap];
    wave_lds_sync();
    for (int e = lane; e < k * cols; e += WAVE) {
      const int i = e % k, cc = e / k;
      T acc = 0;
      for (int b = 0; b < r; ++b) acc += X[i + b * R] * S[b + cc * r];
      E[i + (int64_t)cc * cap] = acc;
    }
    wave_lds_sync();
  }
}

// The column transforms K(q, j) <- K(q, j) t_j^T of the same boxes, one
// workgroup per recompressed box (rows = the new rank of q, at most XF_BOX_R).
template <class T>
__global__ void __launch_bounds__(256) k_col_xform_box(const CompDesc* __restrict__ cs, XfTasks xt, LevelView lv,
                                                       T* __restrict__ pool, const T* __restrict__ work) {
  constexpr int R = XF_BOX_R;
  __shared__ T Xt[R * R];
  __shared__ T slot[4][R * R];
  const CompDesc c = cs[blockIdx.x];
  const int j = c.box;
  const int r = lv.r[j], k = lv.rnew[j], capj = lv.cap[j];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  for (int e = threadIdx.x; e < k * r; e += 256) {
    const int a = e % k, b = e / k;
    Xt[a + b * R] = work[c.tt + a + (int64_t)b * c.ldt];
  }
  __syncthreads();
  const int e0 = xt.estart[j], ne = xt.estart[j + 1] - e0;
  T* S = slot[wv];
  for (int t = wv; t < ne; t += 4) {
    const int code = xt.elist[e0 + t];
    const int qb = lv.B7[(int64_t)j * lv.c7 + code];
    if (qb < 0) continue;
    const int64_t off = lv.Kt[(int64_t)qb * lv.c7 + (lv.c7 - 1 - code)];
    if (off < 0) continue;
    const int rows = lv.rnew[qb], ldq = lv.cap[qb];
    T* E = pool + off;
    if (r == 0 || rows == 0) {
      for (int e = lane; e < rows * k; e += WAVE) E[e % rows + (int64_t)(e / rows) * ldq] = (T)0;
      continue;
    }
    for (int e = lane; e < rows * r; e += WAVE) S[e] = E[e % rows + (int64_t)(e / rows) * ldq];
    wave_lds_sync();
    for (int e = lane; e < rows * k; e += WAVE) {
      const int ii = e % rows, a = e / rows;
      T acc = 0;
      for (int b = 0; b < r; ++b) acc += S[ii + b * rows] * Xt[a + b * R];
      E[ii + (int64_t)a * ldq] = acc;
    }
    wave_lds_sync();
  }
}

// Commit the new bases: U_j <- Uhat, V_j <- Vhat, Sigma <- Sigma_hat, r_j <- k.
template <class T>
__global__ void __launch_bounds__(WG) k_comp_commit(const CompDesc* __restrict__ cs, LevelView lv, T* __restrict__ pool,
                                                    const T* __restrict__ work) {
  const CompDesc c = cs[blockIdx.x];
  const int j = c.box;
  const int mj = lv.m[j], k = lv.rnew[j];
  T* U = pool + lv.Uo[j];
  T* V = pool + lv.Vo[j];
  for (int t = threadIdx.x; t < mj * k; t += WG) {
    U[t] = work[c.uu + t];
    V[t] = work[c.vv + t];
  }
  for (int a = threadIdx.x; a < k; a += WG) {
    pool[lv.SUo[j] + a] = a < c.kq ? work[c.su + a] : (T)0;
    pool[lv.SVo[j] + a] = a < c.kq ? work[c.sv + a] : (T)0;
  }
}

__global__ void k_commit_ranks(const CompDesc* __restrict__ cs, int nc, LevelView lv) {
  const int t = blockIdx.x * WG + threadIdx.x;
  if (t < nc) lv.r[cs[t].box] = lv.rnew[cs[t].box];
}

constexpr int REDIRECT_MAXM = 1024;   // largest x~ size of a box for k_redirect (LDS rows of D Vb)

// Redirect the compressed well-separated fill through K (eq. K_kj_update and
// Alg. 3): K(a, b) += op_a(D(a, b)) op_b with op = Uhat^T on an x~ row side
// and Vhat on an x~ column side. blockIdx.x: elimination; blockIdx.y: pair.
template <class T>
__global__ void __launch_bounds__(WG) k_redirect(const ElimDesc* __restrict__ es, const FNode* __restrict__ Fs,
                                                 LevelView lv, const T* __restrict__ work, T* __restrict__ pool) {
  const ElimDesc e = es[blockIdx.x];
  const int pr = blockIdx.y;
  if (pr >= e.nF * e.nF) return;
  const FNode A = Fs[e.F0 + pr / e.nF];
  const FNode B = Fs[e.F0 + pr % e.nF];
  if (A.type == 1 && B.type == 1) return;
  if (code3(lv.coords, lv.d, A.box, B.box) >= 0) return;
  const int64_t dst = lv.Kt[(int64_t)A.box * lv.c7 + code7(lv.coords, lv.d, A.box, B.box)];
  if (dst < 0) return;
  const int ld = lv.cap[A.box];
  const int ka = A.type == 0 ? lv.r[A.box] : A.dim;     // ranks already committed
  const int kb = B.type == 0 ? lv.r[B.box] : B.dim;
  if (ka == 0 || kb == 0) return;
  const T* D = work + e.dlt;
  const T* Ua = A.type == 0 ? pool + lv.Uo[A.box] : nullptr;
  const T* Vb = B.type == 0 ? pool + lv.Vo[B.box] : nullptr;
  const int ma = A.dim, mb = B.dim;
  __shared__ T sh[8 * REDIRECT_MAXM];
  T* out = pool + dst;
  // rows of (D Vb) in chunks of 8, then Ua^T times them
  for (int a0 = 0; a0 < ka; a0 += 8) {
    const int na = (ka - a0) < 8 ? (ka - a0) : 8;
    // sh[ii, jj] = sum_x opA(a0+ii, x) * D(x, :) ... computed directly per output
    for (int t = threadIdx.x; t < na * mb; t += WG) {
      const int ii = t % na, x = t / na;
      T s = 0;
      if (Ua) {
        for (int y = 0; y < ma; ++y) s += Ua[y + (int64_t)(a0 + ii) * ma] * D[(A.off + y) + (int64_t)(B.off + x) * e.f];
      } else {
        s = D[(A.off + a0 + ii) + (int64_t)(B.off + x) * e.f];
      }
      sh[ii + x * 8] = s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < na * kb; t += WG) {
      const int ii = t % na, jj = t / na;
      T s = 0;
      if (Vb) {
        for (int x = 0; x < mb; ++x) s += sh[ii + x * 8] * Vb[x + (int64_t)jj * mb];
      } else {
        s = sh[ii + jj * 8];
      }
      out[(a0 + ii) + (int64_t)jj * ld] += s;
    }
    __syncthreads();
  }
}

}  // namespace ifmm
