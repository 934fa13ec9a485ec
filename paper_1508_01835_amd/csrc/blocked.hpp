// Blocked, batched LU with partial pivoting and blocked triangular solves.
// Every matrix of a batch is processed in panels of LU_NB columns: the panel
// is factorized by one workgroup, the row interchanges are applied to the
// other columns, the block row of U is obtained by a unit-lower triangular
// solve and the trailing matrix is updated by the batched GEMM (many
// workgroups per matrix). The triangular solves with the factors follow the
// same pattern. Semantics equal LAPACK getrf / getrs: P A = L U, piv[k] is
// the row exchanged with row k.
#pragma once

#include "problem.hpp"

namespace ifmm {

constexpr int LU_NB = 32;

struct PanelDesc {
  void* A;
  int* piv;
  int n, lda, k0, nb, tag, pad;
};

// Factorize columns k0..k0+nb-1 (rows k0..n-1), swapping rows inside the panel.
template <class T>
__global__ void __launch_bounds__(WG) k_lu_panel(const PanelDesc* __restrict__ ds, int* info) {
  const PanelDesc d = ds[blockIdx.x];
  T* __restrict__ A = static_cast<T*>(d.A);
  const int n = d.n, k0 = d.k0, nb = d.nb;
  const int64_t ld = d.lda;
  __shared__ T smax[WG];
  __shared__ int sidx[WG];
  __shared__ int sp;
  __shared__ T spv;
  for (int j = 0; j < nb; ++j) {
    const int col = k0 + j;
    T best = -1;
    int bi = col;
    for (int i = col + threadIdx.x; i < n; i += WG) {
      const T v = fabs(A[i + col * ld]);
      if (v > best) { best = v; bi = i; }
    }
    smax[threadIdx.x] = best;
    sidx[threadIdx.x] = bi;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        const T o = smax[threadIdx.x + s];
        const int oi = sidx[threadIdx.x + s];
        if (o > smax[threadIdx.x] || (o == smax[threadIdx.x] && oi < sidx[threadIdx.x])) {
          smax[threadIdx.x] = o;
          sidx[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      sp = sidx[0];
      d.piv[col] = sp;
      if (!(smax[0] > (T)0) && info) atomicCAS(info, -1, d.tag);
    }
    __syncthreads();
    const int p = sp;
    if (p != col)
      for (int c = k0 + (int)threadIdx.x; c < k0 + nb; c += WG) {
        const T a = A[col + c * ld];
        A[col + c * ld] = A[p + c * ld];
        A[p + c * ld] = a;
      }
    __syncthreads();
    if (threadIdx.x == 0) spv = A[col + col * ld];
    __syncthreads();
    const T inv = spv != (T)0 ? (T)1 / spv : (T)0;
    for (int i = col + 1 + threadIdx.x; i < n; i += WG) A[i + col * ld] *= inv;
    __syncthreads();
    const int rows = n - col - 1, cols = k0 + nb - col - 1;
    for (int e = threadIdx.x; e < rows * cols; e += WG) {
      const int i = col + 1 + e % rows, c = col + 1 + e / rows;
      A[i + c * ld] -= A[i + col * ld] * A[col + c * ld];
    }
    __syncthreads();
  }
}

// Apply the panel's row interchanges to the columns outside the panel, then
// U12 = L11^-1 A12 for the columns right of the panel. blockIdx.y: column chunk.
template <class T>
__global__ void __launch_bounds__(WG) k_lu_swap_trsm(const PanelDesc* __restrict__ ds) {
  const PanelDesc d = ds[blockIdx.x];
  T* __restrict__ A = static_cast<T*>(d.A);
  const int n = d.n, k0 = d.k0, nb = d.nb;
  const int64_t ld = d.lda;
  const int c = blockIdx.y * WG + threadIdx.x;
  if (c >= n || (c >= k0 && c < k0 + nb)) return;
  for (int j = 0; j < nb; ++j) {
    const int p = d.piv[k0 + j];
    if (p != k0 + j) {
      const T a = A[(k0 + j) + c * ld];
      A[(k0 + j) + c * ld] = A[p + c * ld];
      A[p + c * ld] = a;
    }
  }
  if (c < k0 + nb) return;
  T x[LU_NB];
#pragma unroll
  for (int i = 0; i < LU_NB; ++i)
    if (i < nb) x[i] = A[(k0 + i) + c * ld];
#pragma unroll
  for (int i = 0; i < LU_NB; ++i) {
    if (i >= nb) break;
    const T xi = x[i];
#pragma unroll
    for (int r = i + 1; r < LU_NB; ++r)
      if (r < nb) x[r] -= A[(k0 + r) + (int64_t)(k0 + i) * ld] * xi;
  }
#pragma unroll
  for (int i = 0; i < LU_NB; ++i)
    if (i < nb) A[(k0 + i) + c * ld] = x[i];
}

// ------------------------------------------------------------ solves
struct TrsDesc {
  const void* LU;
  const int* piv;
  void* B;
  int n, lda, ncols, ldb, k0, nb;
};

// B <- P B (all n interchanges), one thread per column.
template <class T>
__global__ void k_apply_piv(const TrsDesc* __restrict__ ds) {
  const TrsDesc d = ds[blockIdx.x];
  const int c = blockIdx.y * WG + threadIdx.x;
  if (c >= d.ncols) return;
  T* b = static_cast<T*>(d.B) + (int64_t)c * d.ldb;
  for (int k = 0; k < d.n; ++k) {
    const int p = d.piv[k];
    if (p != k) { const T a = b[k]; b[k] = b[p]; b[p] = a; }
  }
}

// Diagonal block solve: lower unit (upper = 0) or upper non-unit (upper = 1)
// on rows k0..k0+nb-1 of every column.
template <class T>
__global__ void k_trs_diag(const TrsDesc* __restrict__ ds, int upper) {
  const TrsDesc d = ds[blockIdx.x];
  const int c = blockIdx.y * WG + threadIdx.x;
  if (c >= d.ncols) return;
  const T* __restrict__ L = static_cast<const T*>(d.LU);
  T* b = static_cast<T*>(d.B) + (int64_t)c * d.ldb;
  const int k0 = d.k0, nb = d.nb;
  const int64_t ld = d.lda;
  T x[LU_NB];
#pragma unroll
  for (int i = 0; i < LU_NB; ++i)
    if (i < nb) x[i] = b[k0 + i];
  if (!upper) {
#pragma unroll
    for (int i = 0; i < LU_NB; ++i) {
      if (i >= nb) break;
      const T xi = x[i];
#pragma unroll
      for (int r = i + 1; r < LU_NB; ++r)
        if (r < nb) x[r] -= L[(k0 + r) + (int64_t)(k0 + i) * ld] * xi;
    }
  } else {
#pragma unroll
    for (int i = LU_NB - 1; i >= 0; --i) {
      if (i >= nb) continue;
      const T xi = x[i] / L[(k0 + i) + (int64_t)(k0 + i) * ld];
      x[i] = xi;
#pragma unroll
      for (int r = 0; r < LU_NB; ++r)
        if (r < i) x[r] -= L[(k0 + r) + (int64_t)(k0 + i) * ld] * xi;
    }
  }
#pragma unroll
  for (int i = 0; i < LU_NB; ++i)
    if (i < nb) b[k0 + i] = x[i];
}

// ------------------------------------------------------------ host drivers
struct LuJob {
  void* A;
  int* piv;
  int n, lda, tag;
};

struct LuScratch {
  DevBuf pd, gd;
};

template <class T>
inline void lu_blocked(Problem& P, const std::vector<LuJob>& jobs, LuScratch& S) {
  int nmax = 0;
  for (const auto& j : jobs) nmax = std::max(nmax, j.n);
  for (int k0 = 0; k0 < nmax; k0 += LU_NB) {
    std::vector<PanelDesc> pd;
    GemmBatch gb;
    int maxcols = 0;
    for (const auto& j : jobs) {
      if (j.n <= k0) continue;
      PanelDesc d;
      d.A = j.A; d.piv = j.piv; d.n = j.n; d.lda = j.lda; d.k0 = k0; d.nb = std::min(LU_NB, j.n - k0);
      d.tag = j.tag; d.pad = 0;
      pd.push_back(d);
      maxcols = std::max(maxcols, j.n);
      const int rest = j.n - k0 - d.nb;
      if (rest > 0) {
        T* A = static_cast<T*>(j.A);
        const int64_t ld = j.lda;
        gb.add(A + (k0 + d.nb) + (int64_t)k0 * ld, j.lda, 0, A + k0 + (int64_t)(k0 + d.nb) * ld, j.lda, 0,
               A + (k0 + d.nb) + (int64_t)(k0 + d.nb) * ld, j.lda, rest, rest, d.nb, -1.0, 1.0);
      }
    }
    if (pd.empty()) break;
    const PanelDesc* dp = P.put(S.pd, pd);
    P.kbegin();
    hipLaunchKernelGGL(k_lu_panel<T>, dim3((unsigned)pd.size()), dim3(WG), 0, P.stream, dp, P.d_info);
    IFMM_LAUNCH_CHECK();
    hipLaunchKernelGGL(k_lu_swap_trsm<T>, dim3((unsigned)pd.size(), (unsigned)ceil_div(maxcols, WG)), dim3(WG), 0,
                       P.stream, dp);
    IFMM_LAUNCH_CHECK();
    P.kend();
    run_gemm<T>(P, gb, S.gd);
  }
}

struct TrsJob {
  const void* LU;
  const int* piv;
  void* B;
  int n, lda, ncols, ldb;
};

// B <- (P^T L U)^-1 B for every job (getrs).
template <class T>
inline void lu_solve_blocked(Problem& P, const std::vector<TrsJob>& jobs, LuScratch& S) {
  if (jobs.empty()) return;
  int nmax = 0, cmax = 0;
  std::vector<TrsDesc> all;
  for (const auto& j : jobs) {
    if (j.n <= 0 || j.ncols <= 0) continue;
    nmax = std::max(nmax, j.n);
    cmax = std::max(cmax, j.ncols);
    TrsDesc d;
    d.LU = j.LU; d.piv = j.piv; d.B = j.B; d.n = j.n; d.lda = j.lda; d.ncols = j.ncols; d.ldb = j.ldb;
    d.k0 = 0; d.nb = 0;
    all.push_back(d);
  }
  if (all.empty()) return;
  const unsigned gy = (unsigned)ceil_div(cmax, WG);
  {
    const TrsDesc* dd = P.put(S.pd, all);
    P.kbegin();
    hipLaunchKernelGGL(k_apply_piv<T>, dim3((unsigned)all.size(), gy), dim3(WG), 0, P.stream, dd);
    IFMM_LAUNCH_CHECK();
    P.kend();
  }
  const int nblk = (int)ceil_div(nmax, LU_NB);
  for (int pass = 0; pass < 2; ++pass) {          // 0: forward with L, 1: backward with U
    for (int s = 0; s < nblk; ++s) {
      const int bk = pass == 0 ? s : nblk - 1 - s;
      std::vector<TrsDesc> v;
      GemmBatch gb;
      for (const auto& d0 : all) {
        const int k0 = bk * LU_NB;
        if (k0 >= d0.n) continue;
        TrsDesc d = d0;
        d.k0 = k0;
        d.nb = std::min(LU_NB, d0.n - k0);
        v.push_back(d);
        const T* L = static_cast<const T*>(d.LU);
        T* B = static_cast<T*>(d.B);
        const int64_t ld = d.lda;
        if (pass == 0) {
          const int rest = d.n - k0 - d.nb;
          if (rest > 0)
            gb.add(L + (k0 + d.nb) + (int64_t)k0 * ld, d.lda, 0, B + k0, d.ldb, 0, B + k0 + d.nb, d.ldb, rest, d.ncols,
                   d.nb, -1.0, 1.0);
        } else if (k0 > 0) {
          gb.add(L + (int64_t)k0 * ld, d.lda, 0, B + k0, d.ldb, 0, B, d.ldb, k0, d.ncols, d.nb, -1.0, 1.0);
        }
      }
      if (v.empty()) continue;
      const TrsDesc* dv = P.put(S.pd, v);
      P.kbegin();
      hipLaunchKernelGGL(k_trs_diag<T>, dim3((unsigned)v.size(), gy), dim3(WG), 0, P.stream, dv, pass);
      IFMM_LAUNCH_CHECK();
      P.kend();
      run_gemm<T>(P, gb, S.gd);
    }
  }
}

}  // namespace ifmm
