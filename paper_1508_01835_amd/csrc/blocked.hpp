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

// Raw buffer access (gfx9 buffer resource: base, byte extent, 32-bit data
// format word). One 32-bit per-lane byte offset serves every column of a
// panel; the column offset is wave-uniform and goes in a scalar register, so a
// row's 32 loads need no per-column address registers. Accesses past the
// extent read zero and drop writes.
__device__ inline __amdgpu_buffer_rsrc_t buf_rsrc(void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}
template <class T>
__device__ inline T buf_ld(__amdgpu_buffer_rsrc_t r, int vo, int so);
template <>
__device__ inline double buf_ld<double>(__amdgpu_buffer_rsrc_t r, int vo, int so) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, 0));
}
template <>
__device__ inline float buf_ld<float>(__amdgpu_buffer_rsrc_t r, int vo, int so) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, vo, so, 0));
}
__device__ inline void buf_st(double v, __amdgpu_buffer_rsrc_t r, int vo, int so) {
  using B = decltype(__builtin_amdgcn_raw_buffer_load_b64(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(B, v), r, vo, so, 0);
}
__device__ inline void buf_st(float v, __amdgpu_buffer_rsrc_t r, int vo, int so) {
  using B = decltype(__builtin_amdgcn_raw_buffer_load_b32(r, 0, 0, 0));
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(B, v), r, vo, so, 0);
}


struct PanelDesc {
  void* A;
  int* piv;
  int n, lda, k0, nb, tag, pad;
};

// Factorize columns k0..k0+nb-1 (rows k0..n-1), swapping rows inside the panel.
// Each thread owns the rows i = k0 + tid + k WG. Per column: the pivot (largest
// magnitude, smallest row on ties) by wavefront shuffles and one exchange
// through LDS; the swap of the pivot row, which also goes to LDS; then each
// thread scales its rows' multipliers and updates their remaining panel
// columns with all loads of a chunk in flight, keeping the magnitude of the
// next column as its pivot candidate (so the next pivot needs no extra pass).
template <class T, bool INLDS>
__device__ __forceinline__ void lu_panel_run(const PanelDesc& d, int* info, T* __restrict__ L) {
  constexpr int NW = WG / WAVE;
  constexpr int QC = 8;
  T* __restrict__ A = static_cast<T*>(d.A);
  const int n = d.n, k0 = d.k0, nb = d.nb;
  const int64_t ld = d.lda;
  __shared__ T wbest[NW];
  __shared__ int wbi[NW];
  __shared__ T prow[LU_NB];   // pivot row after the swap, zero outside the columns to update
  __shared__ T pdiag;
  __shared__ int sp;
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  // the panel's columns from row 0: one per-lane offset for all of a row's columns
  T* P = A + (int64_t)k0 * ld;
  const int ldb = (int)ld * (int)sizeof(T);   // the host checks LU_NB lda sizeof(T) < 2^31
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(P, (uint32_t)(((int64_t)(nb - 1) * ld + n) * sizeof(T)));
  // INLDS: the panel rows k0..n-1 live in LDS (column-major, leading dimension n - k0) while it is factorized
  const int ml = n - k0;
  auto ldv = [&](int c, int i) -> T {
    if constexpr (INLDS) return L[(i - k0) + c * ml];
    else return buf_ld<T>(rs, i * (int)sizeof(T), c * ldb);
  };
  auto stv = [&](int c, int i, T v) {
    if constexpr (INLDS) L[(i - k0) + c * ml] = v;
    else buf_st(v, rs, i * (int)sizeof(T), c * ldb);
  };
  if constexpr (INLDS) {
    for (int c = 0; c < nb; ++c)
      for (int i = tid; i < ml; i += WG) L[i + c * ml] = buf_ld<T>(rs, (k0 + i) * (int)sizeof(T), c * ldb);
    __syncthreads();
  }
  T best = (T)-1;
  int bi = k0;
  for (int i = k0 + tid; i < n; i += WG) {
    const T v = fabs(ldv(0, i));
    if (v > best) { best = v; bi = i; }
  }
  for (int j = 0; j < nb; ++j) {
    const int col = k0 + j;
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const T ob = __shfl_xor(best, o, WAVE);
      const int oi = __shfl_xor(bi, o, WAVE);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    }
    if (lane == 0) { wbest[wv] = best; wbi[wv] = bi; }
    __syncthreads();
    if (tid == 0) {
      T b = wbest[0];
      int i0 = wbi[0];
      for (int w = 1; w < NW; ++w)
        if (wbest[w] > b || (wbest[w] == b && wbi[w] < i0)) { b = wbest[w]; i0 = wbi[w]; }
      sp = i0;
      d.piv[col] = i0;
      if (!(b > (T)0) && info) atomicCAS(info, -1, d.tag);
    }
    __syncthreads();
    const int p = sp;
    if (tid < LU_NB) {
      T b = 0;
      if (tid < nb) {
        const T a = ldv(tid, col);
        b = ldv(tid, p);
        if (p != col) {
          stv(tid, col, b);
          stv(tid, p, a);
        }
      }
      if (tid == j) pdiag = b;
      prow[tid] = tid > j && tid < nb ? b : (T)0;
    }
    __syncthreads();
    const T inv = pdiag != (T)0 ? (T)1 / pdiag : (T)0;
    best = (T)-1;
    bi = col + 1;
    for (int i = k0 + tid; i < n; i += WG) {
      if (i <= col) continue;
      const T l = ldv(j, i) * inv;
#pragma unroll
      for (int q = 0; q < LU_NB; q += QC) {
        if (q + QC - 1 > j && q < nb) {
          T x[QC];
#pragma unroll
          for (int k = 0; k < QC; ++k) x[k] = ldv(min(q + k, nb - 1), i);
#pragma unroll
          for (int k = 0; k < QC; ++k) x[k] -= l * prow[q + k];
          if (q + QC <= nb) {
#pragma unroll
            for (int k = 0; k < QC; ++k) stv(q + k, i, x[k]);
          } else {
#pragma unroll
            for (int k = 0; k < QC; ++k)
              if (q + k < nb) stv(q + k, i, x[k]);
          }
          if (j + 1 >= q && j + 1 < q + QC) {
            T y = x[0];
#pragma unroll
            for (int k = 1; k < QC; ++k) y = j + 1 == q + k ? x[k] : y;
            const T v = fabs(y);
            if (v > best) { best = v; bi = i; }
          }
        }
      }
      stv(j, i, l);   // after the chunk that rewrote column col unchanged
    }
  }
  if constexpr (INLDS) {
    __syncthreads();
    for (int c = 0; c < nb; ++c)
      for (int i = tid; i < ml; i += WG) buf_st(L[i + c * ml], rs, (k0 + i) * (int)sizeof(T), c * ldb);
  }
}

// lds_rows > 0: every panel of the launch has at most lds_rows rows and is
// factorized in dynamic LDS (lds_rows x LU_NB elements).
template <class T>
__global__ void __launch_bounds__(WG) k_lu_panel(const PanelDesc* __restrict__ ds, int* info, int lds_rows) {
  extern __shared__ unsigned char lu_dyn[];
  const PanelDesc d = ds[blockIdx.x];
  if (lds_rows > 0)
    lu_panel_run<T, true>(d, info, reinterpret_cast<T*>(lu_dyn));
  else
    lu_panel_run<T, false>(d, info, nullptr);
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
    if (i < nb) {
      const T xi = x[i];
#pragma unroll
      for (int r = i + 1; r < LU_NB; ++r)
        if (r < nb) x[r] -= A[(k0 + r) + (int64_t)(k0 + i) * ld] * xi;
    }
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
__global__ void __launch_bounds__(WG) k_apply_piv(const TrsDesc* __restrict__ ds) {
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
__global__ void __launch_bounds__(WG) k_trs_diag(const TrsDesc* __restrict__ ds, int upper) {
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
      if (i < nb) {
        const T xi = x[i];
#pragma unroll
        for (int r = i + 1; r < LU_NB; ++r)
          if (r < nb) x[r] -= L[(k0 + r) + (int64_t)(k0 + i) * ld] * xi;
      }
    }
  } else {
#pragma unroll
    for (int i = LU_NB - 1; i >= 0; --i) {
      if (i < nb) {
        const T xi = x[i] / L[(k0 + i) + (int64_t)(k0 + i) * ld];
        x[i] = xi;
#pragma unroll
        for (int r = 0; r < LU_NB; ++r)
          if (r < i) x[r] -= L[(k0 + r) + (int64_t)(k0 + i) * ld] * xi;
      }
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

constexpr size_t LU_LDS_MAX = 144 * 1024;   // dynamic LDS of the panel kernel (gfx950: 160 KB per workgroup)

template <class T>
inline void lu_blocked(Problem& P, const std::vector<LuJob>& jobs, LuScratch& S) {
  static const bool attr = [] {   // once per process (thread-safe initialisation)
    IFMM_HIP(hipFuncSetAttribute((const void*)k_lu_panel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)LU_LDS_MAX));
    return true;
  }();
  (void)attr;
  int nmax = 0;
  for (const auto& j : jobs) {
    nmax = std::max(nmax, j.n);
    // the panel kernel addresses a panel with 32-bit byte offsets
    if ((int64_t)j.lda * LU_NB * (int64_t)sizeof(T) >= ((int64_t)1 << 31))
      fail(IFMM_ERR_ARG, "LU of a matrix with leading dimension " + std::to_string(j.lda) + ": above the panel limit");
  }
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
    // panels that fit are factorized in LDS (one load and one store of the panel)
    int rows = 0;
    for (const auto& q : pd) rows = std::max(rows, q.n - q.k0);
    const size_t lds = (size_t)rows * LU_NB * sizeof(T);
    const bool inlds = lds <= LU_LDS_MAX && !force_streamed();
    P.kbegin();
    hipLaunchKernelGGL(k_lu_panel<T>, dim3((unsigned)pd.size()), dim3(WG), inlds ? lds : 0, P.stream, dp, P.d_info,
                       inlds ? rows : 0);
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

// ============================================================ blocked QR
// Householder QR in panels of QR_NB columns with the compact WY form
// H_j0 ... H_j0+nb-1 = I - V T V^T: the panel kernel factorizes the panel and
// writes V (unit lower trapezoidal, explicit zeros above) and T; the trailing
// columns are updated by A2 <- A2 - V (T^T (V^T A2)) with the batched GEMM.
// Only R is produced (the recompression needs the left singular vectors of
// R^T, not Q).
constexpr int QR_NB = 32;
constexpr int QR_WG = 512;    // threads of the panel kernel (8 wavefronts, 256 registers each)

struct QrPanel {
  void* A;
  void* V;      // (M - j0) x nb, leading dimension M - j0
  void* Tm;     // nb x nb
  void* alph;   // N diagonal entries of R (per matrix)
  int M, N, lda, j0, nb, pad;
};

// One panel of QR_NB columns per workgroup. Each thread owns the panel rows
// i = tid + k QR_WG and reads a row's panel columns together (independent
// loads from one per-lane offset), so the panel streams at bandwidth instead of
// one dependent column walk per wavefront. One pass over the panel per
// Householder column j does three things:
//   applies reflector j - 1 to the columns right of it and stores column
//   j - 1 as v_{j-1};
//   sums the squares of the updated column j below its diagonal;
//   sums S_c = sum_{i > j} y_i x_ic, the products of that column with every
//   panel column.
// With the broadcast row j, the coefficients of reflector j follow:
// v_j^T x_c = x_jc + S_c / (x_jj - alpha). For c > j they are the update
// coefficients; for c < j they are the Gram entries V^T v_j that build T.
// T follows from the Gram entries row by row (row i of T needs only row i).
// FULL: the panel has exactly QR_NB columns, so no column test is needed and
// stores cover whole chunks (unchanged columns are rewritten as read).
// Otherwise columns past the panel are read as aliases and never stored.
template <class T>
struct QrShared {
  T tau[QR_NB];
  T part[QR_WG / WAVE][QR_NB];
  T sred[QR_WG / WAVE];
  T Stot[QR_NB];        // S_c of the column being prepared
  T stot;               // its squares below the diagonal
  T rowj[QR_NB];        // its diagonal row, after the updates so far
  T G[QR_NB * QR_NB];   // G[k + j QR_NB] = V(:,k)^T V(:,j), k < j
  T Ts[QR_NB * QR_NB];
};

// Lp: LDS copy of the first QR_WG panel rows (row i < QR_WG at Lp[i + c QR_WG]),
// loaded once at the start and written back at the end; row i is the first
// row of thread i, so a panel of at most QR_WG rows touches HBM once each way.
template <class T, bool FULL>
__device__ __forceinline__ void qr_panel_run(const QrPanel& d, QrShared<T>& shm, T* __restrict__ Lp) {
  constexpr int NW = QR_WG / WAVE;
  constexpr int QC = 4;   // columns per store chunk
  T* __restrict__ A = static_cast<T*>(d.A);
  T* __restrict__ V = static_cast<T*>(d.V);
  T* __restrict__ Tm = static_cast<T*>(d.Tm);
  T* __restrict__ alph = static_cast<T*>(d.alph);
  const int j0 = d.j0;
  const int nb = FULL ? QR_NB : d.nb;
  const int64_t lda = d.lda;
  const int mv = d.M - j0;
  T* tau = shm.tau;
  auto& part = shm.part;
  T* sred = shm.sred;
  T* Stot = shm.Stot;
  T& stot = shm.stot;
  T* rowj = shm.rowj;
  T* G = shm.G;
  T* Ts = shm.Ts;
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  T* P = A + j0 + (int64_t)j0 * lda;   // panel: P[i + c lda], i < mv, c < nb
  const int ldb = (int)lda * (int)sizeof(T);   // the host checks QR_NB lda sizeof(T) < 2^31
  const __amdgpu_buffer_rsrc_t rs = buf_rsrc(P, (uint32_t)(((int64_t)(nb - 1) * lda + mv) * sizeof(T)));
  // element (i, c); past a partial panel, columns alias its last one (loaded, never stored)
  auto ld = [&](int c, int i) {
    const int cc = FULL || c < nb ? c : nb - 1;
    if (i < QR_WG) return Lp[i + cc * QR_WG];
    return buf_ld<T>(rs, i * (int)sizeof(T), cc * ldb);
  };
  auto st = [&](int c, int i, T v) {
    if (i < QR_WG) Lp[i + c * QR_WG] = v;
    else buf_st(v, rs, i * (int)sizeof(T), c * ldb);
  };
  if (tid < mv)
    for (int c = 0; c < nb; ++c) Lp[tid + c * QR_WG] = buf_ld<T>(rs, tid * (int)sizeof(T), c * ldb);
  auto load_row = [&](int i, T (&x)[QR_NB]) {
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) x[c] = ld(c, i);
  };
  // store the columns >= c0 of row i (FULL: whole chunks from the one holding c0)
  auto store_row = [&](int i, const T (&x)[QR_NB], int c0) {
#pragma unroll
    for (int q = 0; q < QR_NB; q += QC) {
      if (q + QC - 1 >= c0) {
#pragma unroll
        for (int k = 0; k < QC; ++k)
          if (FULL || (q + k >= c0 && q + k < nb)) st(q + k, i, x[q + k]);
      }
    }
  };
  // block sums of S[] and s into Stot and stot
  auto reduce = [&](const T (&S)[QR_NB], T s) {
    const T r = wave_sum32_scatter(S, lane);
    s = wave_sum(s);
    if ((lane & 1) == 0) part[wv][lane >> 1] = r;
    if (lane == 0) sred[wv] = s;
    __syncthreads();
    if (tid < QR_NB) {
      T t = 0;
      for (int w = 0; w < NW; ++w) t += part[w][tid];
      Stot[tid] = t;
    } else if (tid == QR_NB) {
      T t = 0;
      for (int w = 0; w < NW; ++w) t += sred[w];
      stot = t;
    }
    __syncthreads();
  };

  // The panel is scaled once by the exact power of two that brings its largest
  // entry into [1, 2), so that squares of tiny or huge entries neither underflow
  // nor overflow; the Householder vectors are scale-free, the R entries are
  // scaled back at the end.
  T am = 0;
  for (int i = tid; i < mv; i += QR_WG) {
    T x[QR_NB];
    load_row(i, x);
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) am = fmax(am, fabs(x[c]));
  }
  am = block_max(am, sred);
  const int sh = am > (T)0 ? -ilogb((double)am) : 0;
  // scaling pass, which also prepares column 0
  {
    T S[QR_NB], s = 0;
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) S[c] = 0;
    for (int i = tid; i < mv; i += QR_WG) {
      T x[QR_NB];
      load_row(i, x);
      if (sh != 0) {
#pragma unroll
        for (int c = 0; c < QR_NB; ++c) x[c] = ldexp(x[c], sh);
        store_row(i, x, 0);
      }
      if (i == 0) {
#pragma unroll
        for (int c = 0; c < QR_NB; ++c) rowj[c] = x[c];
      } else {
        const T y = x[0];
        s += y * y;
#pragma unroll
        for (int c = 0; c < QR_NB; ++c) S[c] += y * x[c];
      }
    }
    reduce(S, s);
  }

  T scal_prev = 1;
  for (int j = 0; j < nb; ++j) {
    // reflector j (every thread computes the same values from the block sums)
    const T x0 = rowj[j], s = stot;
    T tj = 0, al = x0, scal = 0;
    if (s > (T)0) {
      al = x0 >= (T)0 ? -sqrt(x0 * x0 + s) : sqrt(x0 * x0 + s);
      tj = (al - x0) / al;
      scal = (T)1 / (x0 - al);
    }
    // coefficients of the rank-one update (zero up to column j, so those
    // columns are rewritten unchanged); the pass left column j - 1 unscaled in
    // its products, hence the factor scal_prev on that Gram entry
    T coef[QR_NB];
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) coef[c] = c > j ? tj * (rowj[c] + scal * Stot[c]) : (T)0;
    const T cnext = j + 1 < nb ? tj * (rowj[j + 1] + scal * Stot[j + 1]) : (T)0;
    if (tid < j) G[tid + j * QR_NB] = (rowj[tid] + scal * Stot[tid]) * (tid == j - 1 ? scal_prev : (T)1);
    if (tid == 0) { tau[j] = tj; alph[j0 + j] = ldexp(al, -sh); }
    scal_prev = scal;
    __syncthreads();   // rowj, Stot and stot are rewritten below
    // apply reflector j, store v_j, prepare column j + 1
    const bool next = j + 1 < nb;
    T S[QR_NB], sn = 0;
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) S[c] = 0;
    for (int i = tid; i < mv; i += QR_WG) {
      if (i < j) continue;
      T x[QR_NB];
      load_row(i, x);
      const T xj = ld(j, i), xn = next ? ld(j + 1, i) : (T)0;
      const T v = i > j ? xj * scal : (T)1;
#pragma unroll
      for (int c = 0; c < QR_NB; ++c) x[c] -= coef[c] * v;
      store_row(i, x, j);
      st(j, i, v);   // after the chunk that rewrote column j unchanged
      if (next) {
        if (i == j + 1) {
#pragma unroll
          for (int c = 0; c < QR_NB; ++c) rowj[c] = x[c];
        } else if (i > j + 1) {
          const T y = xn - cnext * v;
          sn += y * y;
#pragma unroll
          for (int c = 0; c < QR_NB; ++c) S[c] += y * x[c];
        }
      }
    }
    if (next) reduce(S, sn);
  }
  __syncthreads();
  // R entries of the panel rows, strictly right of the diagonal, back to their scale
  for (int e = tid; e < nb * nb; e += QR_WG) {
    const int r = e % nb, c = e / nb;
    if (r < c) st(c, r, ldexp(ld(c, r), -sh));
  }
  // V with explicit unit diagonal and zeros above it (own rows only)
  for (int i = tid; i < mv; i += QR_WG) {
    T x[QR_NB];
    load_row(i, x);
#pragma unroll
    for (int c = 0; c < QR_NB; ++c) {
      if (FULL || c < nb) {
        T v = 0;
        if (tau[c] != (T)0) v = i == c ? (T)1 : (i > c ? x[c] : (T)0);
        V[i + (int64_t)c * mv] = v;
      }
    }
  }
  // T: T_ii = tau_i, T(i, j) = -tau_j sum_{k=i}^{j-1} T(i, k) G(k, j); row i
  // depends only on row i, so lane i of the first wavefront builds it
  if (tid < nb) {
    const int i = tid;
    for (int j = 0; j < nb; ++j) {
      T val = 0;
      if (j == i) {
        val = tau[i];
      } else if (j > i && tau[j] != (T)0) {
        T sacc = 0;
        for (int k = i; k < j; ++k) sacc += Ts[i + k * QR_NB] * G[k + j * QR_NB];
        val = -tau[j] * sacc;
      }
      Ts[i + j * QR_NB] = val;
      Tm[i + j * nb] = val;
    }
  }
  // the LDS rows back to the matrix (the unscaled R rows included)
  __syncthreads();
  if (tid < mv)
    for (int c = 0; c < nb; ++c) buf_st(Lp[tid + c * QR_WG], rs, tid * (int)sizeof(T), c * ldb);
}

constexpr size_t QR_LDS = (size_t)QR_WG * QR_NB;   // elements of the LDS panel rows

template <class T>
__global__ void __launch_bounds__(QR_WG) k_qr_panel(const QrPanel* __restrict__ ds) {
  extern __shared__ unsigned char qr_dyn[];
  __shared__ QrShared<T> shm;
  const QrPanel d = ds[blockIdx.x];
  T* Lp = reinterpret_cast<T*>(qr_dyn);
  if (d.nb == QR_NB)
    qr_panel_run<T, true>(d, shm, Lp);
  else
    qr_panel_run<T, false>(d, shm, Lp);
}

// R (kq x N, leading dimension ldr) from the factorized A and its diagonal.
struct QrOut {
  const void* A;
  const void* alph;
  void* R;
  int M, N, lda, ldr;
};

template <class T>
__global__ void k_qr_extract(const QrOut* __restrict__ ds) {
  const QrOut d = ds[blockIdx.x];
  const T* A = static_cast<const T*>(d.A);
  const T* al = static_cast<const T*>(d.alph);
  T* R = static_cast<T*>(d.R);
  const int kq = d.M < d.N ? d.M : d.N;
  for (int64_t e = threadIdx.x; e < (int64_t)kq * d.N; e += WG) {
    const int i = (int)(e % kq), c = (int)(e / kq);
    T v = 0;
    if (i == c) v = al[i];
    else if (i < c) v = A[i + (int64_t)c * d.lda];
    R[i + (int64_t)c * d.ldr] = v;
  }
}

struct QrJob {
  void* A;
  void* R;
  int M, N, lda, ldr;
};

// R-only Householder QR of a narrow M x N matrix (N <= 64), a column per lane:
// lanes g NP .. g NP + NP - 1 of a wavefront own the columns of job g (NP =
// 16, 32 or 64, so 4, 2 or 1 jobs per wavefront), and the rows stream through
// in chunks of QcCh<T> rows (each lane holds its column of the chunk in registers)
// while the running triangle R sits in LDS, packed by columns, column c with
// lane c. The chunk is folded into R by one reflector per column j, acting on
// row j of R and column j of the chunk: column j is broadcast to the job's
// lanes, and every trailing column takes its dot product with it in its own
// lane, so no reduction crosses lanes. The reflector convention is the panel kernel's
// (alpha = -sign(x0) ||x||, tau = (alpha - x0) / alpha, tau = 0 for a zero
// column) and each job is scaled once by an exact power of two. A is left as
// it was; R (min(M, N) x N, ldr, zero below the diagonal) is written at the end.
template <class T>
struct QcCh {   // rows per chunk: a step's latency is paid once for twice the rows in FP32
  static constexpr int v = sizeof(T) == 4 ? 64 : 32;
};
constexpr int QC_NMAX = 64;

template <class T, int NP>
struct QrCols {
  static constexpr int G = WAVE / NP;                 // jobs per wavefront
  static constexpr int TRI = NP * (NP + 1) / 2;       // packed upper triangle of R
  static constexpr int WAVES = 4;                     // at most 66.5 KB of LDS (FP64, NP = 64)
};
// R[i, c] (i <= c) of the packed column-major upper triangle
__device__ inline int qc_tri(int i, int c) { return c * (c + 1) / 2 + i; }

template <int G, class T>
__device__ inline T qc_bcast(T x, int src) {
  if constexpr (G == 1) {   // one job per wavefront: the source lane is uniform
    if constexpr (sizeof(T) == 8) {
      const int64_t b = __double_as_longlong((double)x);
      const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), src);
      const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
      return (T)__longlong_as_double(((int64_t)hi << 32) | (uint32_t)lo);
    } else {
      return __int_as_float(__builtin_amdgcn_readlane(__float_as_int((float)x), src));
    }
  } else {
    return __shfl(x, src, WAVE);
  }
}

template <class T, int NP, int NT = QrCols<T, NP>::WAVES * WAVE>
__global__ void __launch_bounds__(NT) k_qr_cols(const QrJob* __restrict__ js, int nj) {
  constexpr int G = QrCols<T, NP>::G, WAVES = QrCols<T, NP>::WAVES, TRI = QrCols<T, NP>::TRI;
  __shared__ T Rs[WAVES][G][TRI];   // the running triangle, packed by columns
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int g = lane / NP, c = lane % NP;
  const int t = ((int)blockIdx.x * WAVES + w) * G + g;
  QrJob d{};
  if (t < nj) d = js[t];
  const T* __restrict__ A = static_cast<const T*>(d.A);
  const int M = t < nj ? d.M : 0, N = t < nj ? d.N : 0;
  const int64_t lda = d.lda;
  const bool col = c < N;
  T* R = Rs[w][g];
  for (int i = 0; i <= c; ++i) R[qc_tri(i, c)] = 0;
  // exact power-of-two scaling by the job's largest magnitude
  T am = 0;
  if (col)
    for (int i = 0; i < M; ++i) am = fmax(am, fabs(A[i + c * lda]));
#pragma unroll
  for (int o = NP / 2; o > 0; o >>= 1) am = fmax(am, __shfl_xor(am, o, WAVE));
  const int sh = am > (T)0 ? -ilogb((double)am) : 0;
  // the wavefront walks the largest of its jobs' row and column counts
  int Mw = M, Nw = N;
#pragma unroll
  for (int o = NP; o < WAVE; o <<= 1) {
    Mw = max(Mw, __shfl_xor(Mw, o, WAVE));
    Nw = max(Nw, __shfl_xor(Nw, o, WAVE));
  }
  constexpr int CH = QcCh<T>::v;
  T x[CH], v[CH];
  for (int i0 = 0; i0 < Mw; i0 += CH) {
#pragma unroll
    for (int i = 0; i < CH; ++i) x[i] = (col && i0 + i < M) ? ldexp(A[i0 + i + c * lda], sh) : (T)0;
    for (int j = 0; j < Nw; ++j) {
      const int src = g * NP + j;   // lane of column j of this job (a zero column when j >= N)
      // four partial sums each: independent chains instead of one 32-long
      T s4[4] = {0, 0, 0, 0}, d4[4] = {0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < CH; ++i) {
        v[i] = qc_bcast<G>(x[i], src);
        s4[i & 3] += v[i] * v[i];
        d4[i & 3] += v[i] * x[i];
      }
      const T s = (s4[0] + s4[1]) + (s4[2] + s4[3]), dot = (d4[0] + d4[1]) + (d4[2] + d4[3]);
      const T x0 = R[qc_tri(j, j)];
      if (j < N && s > (T)0) {
        const T al = x0 >= (T)0 ? -sqrt(x0 * x0 + s) : sqrt(x0 * x0 + s);
        const T tj = (al - x0) / al;
        const T scal = (T)1 / (x0 - al);
        if (c > j && col) {
          const T wc = tj * (R[qc_tri(j, c)] + scal * dot);
          R[qc_tri(j, c)] -= wc;
          const T f = wc * scal;
#pragma unroll
          for (int i = 0; i < CH; ++i) x[i] -= f * v[i];
        } else if (c == j) {
#pragma unroll
          for (int i = 0; i < CH; ++i) x[i] = 0;
          R[qc_tri(j, j)] = al;
        }
      }
    }
  }
  const int kq = M < N ? M : N;
  if (col) {
    T* __restrict__ Ro = static_cast<T*>(d.R);
    for (int i = 0; i < kq; ++i) Ro[i + c * d.ldr] = i <= c ? ldexp(R[qc_tri(i, c)], -sh) : (T)0;
  }
}

struct QrScratch {
  DevBuf w, pd, gd, nw;
};

// Narrow jobs on the column-per-lane kernel. A wavefront streams its rows one
// chunk after the other, so the time of a launch is that of its tallest job:
// a job of more than QR_SEG_MAX rows is cut into segments of about
// QR_SEG_ROWS rows (at least 64 >= N, so every segment's triangle is a full
// N x N), and the stacked triangles (S N rows) form the job of the next
// level, cut again while still too tall (a fixed-order reduction tree).
constexpr int QR_SEG_MAX = 1024, QR_SEG_ROWS = 512;

template <class T>
inline void qr_narrow_launch(Problem& P, std::vector<QrJob>& v) {
  // one launch per column class (16, 32, 64), the jobs of a class contiguous
  std::stable_sort(v.begin(), v.end(), [](const QrJob& a, const QrJob& b) {
    return (a.N > 16) + (a.N > 32) < (b.N > 16) + (b.N > 32);
  });
  DevBuf unused;
  const QrJob* dv = P.put(unused, v);
  size_t b0 = 0;
  while (b0 < v.size()) {
    const int cls = (v[b0].N > 16) + (v[b0].N > 32);
    size_t b1 = b0;
    while (b1 < v.size() && (v[b1].N > 16) + (v[b1].N > 32) == cls) ++b1;
    const int n = (int)(b1 - b0);
    if (cls == 0) {
      constexpr int per = QrCols<T, 16>::G * QrCols<T, 16>::WAVES;
      hipLaunchKernelGGL((k_qr_cols<T, 16>), dim3((unsigned)ceil_div(n, per)), dim3(QrCols<T, 16>::WAVES * WAVE), 0,
                         P.stream, dv + b0, n);
    } else if (cls == 1) {
      constexpr int per = QrCols<T, 32>::G * QrCols<T, 32>::WAVES;
      hipLaunchKernelGGL((k_qr_cols<T, 32>), dim3((unsigned)ceil_div(n, per)), dim3(QrCols<T, 32>::WAVES * WAVE), 0,
                         P.stream, dv + b0, n);
    } else {
      constexpr int per = QrCols<T, 64>::G * QrCols<T, 64>::WAVES;
      hipLaunchKernelGGL((k_qr_cols<T, 64>), dim3((unsigned)ceil_div(n, per)), dim3(QrCols<T, 64>::WAVES * WAVE), 0,
                         P.stream, dv + b0, n);
    }
    IFMM_LAUNCH_CHECK();
    b0 = b1;
  }
}

template <class T>
inline void qr_narrow_run(Problem& P, const std::vector<QrJob>& narrow, QrScratch& S) {
  double fl = 0;   // Householder R of an M x N matrix: 2 a b^2 - 2/3 b^3, a = max(M, N), b = min(M, N)
  for (const auto& j : narrow) {
    const double a = std::max(j.M, j.N), b = std::min(j.M, j.N);
    fl += 2.0 * a * b * b - 2.0 / 3.0 * b * b * b;
  }
  auto nseg = [](const QrJob& j) { return j.M > QR_SEG_MAX && j.M > j.N ? (int)ceil_div(j.M, QR_SEG_ROWS) : 1; };
  // stacked triangles of the first level bound every later level (each is at most a quarter of the one before)
  int64_t stack = 0;
  for (const auto& j : narrow) {
    const int ns = nseg(j);
    if (ns > 1) stack += (int64_t)ns * j.N * j.N;
  }
  if (stack > 0 && (size_t)stack * 2 * sizeof(T) > S.nw.bytes) {
    P.sync();
    S.nw.alloc((size_t)stack * 2 * sizeof(T) + 64, &P.mem);
  }
  T* buf[2] = {stack > 0 ? S.nw.template as<T>() : nullptr, stack > 0 ? S.nw.template as<T>() + stack : nullptr};
  std::vector<QrJob> cur(narrow), next, run;
  int levels = 0;
  int64_t rows0 = 0, rows_more = 0;
  P.kone_begin(KF_QR_NARROW, fl);
  for (int lev = 0; !cur.empty(); ++lev) {
    run.clear();
    next.clear();
    T* W = buf[lev & 1];
    int64_t off = 0;
    for (const auto& j : cur) {
      (lev == 0 ? rows0 : rows_more) += j.M;
      const int ns = nseg(j);
      if (ns == 1) {
        run.push_back(j);
        continue;
      }
      const int ld = ns * j.N;
      const int per = j.M / ns;   // > QR_SEG_ROWS (ns - 1) / ns >= 256 >= N; the last segment takes the rest
      for (int k = 0; k < ns; ++k) {
        const int r0 = k * per, mk = k + 1 < ns ? per : j.M - r0;
        run.push_back({static_cast<T*>(j.A) + r0, W + off + (int64_t)k * j.N, mk, j.N, j.lda, ld});
      }
      next.push_back({W + off, j.R, ld, j.N, ld, j.ldr});
      off += (int64_t)ns * j.N * j.N;
    }
    qr_narrow_launch<T>(P, run);
    cur.swap(next);
    levels = lev + 1;
  }
  P.kone_end();
  if (P.kt.on && P.kcur >= 0) P.kt.flops[P.kcur] -= fl;
  if (qr_stats_on()) {
    int mx = 0, nx = 0;
    for (const auto& j : narrow) { mx = std::max(mx, j.M); nx = std::max(nx, j.N); }
    std::fprintf(stderr, "[ifmm-qr] narrow jobs=%zu sumM=%lld maxM=%d maxN=%d levels=%d rows_after_first=%lld\n",
                 narrow.size(), (long long)rows0, mx, nx, levels, (long long)rows_more);
  }
}

template <class T>
inline void qr_blocked(Problem& P, const std::vector<QrJob>& jobs_in, QrScratch& S) {
  if (jobs_in.empty()) return;
  // matrices of at most 64 columns: the column-per-lane streaming kernel
  std::vector<QrJob> narrow, jobs;
  for (const auto& j : jobs_in) (j.N <= QC_NMAX && j.R && !force_streamed() ? narrow : jobs).push_back(j);
  if (!narrow.empty()) qr_narrow_run<T>(P, narrow, S);
  if (jobs.empty()) return;
  static const bool attr = [] {   // once per process (thread-safe initialisation)
    IFMM_HIP(hipFuncSetAttribute((const void*)k_qr_panel<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)(QR_LDS * sizeof(T))));
    return true;
  }();
  (void)attr;
  // workspace per job: alph (N), V ((M) x QR_NB), T (QR_NB^2), W1, W2 (QR_NB x N)
  std::vector<int64_t> off(jobs.size());
  int64_t tot = 0;
  int nmax = 0;
  for (size_t b = 0; b < jobs.size(); ++b) {
    const auto& j = jobs[b];
    // the panel kernel addresses a panel with 32-bit byte offsets
    if ((int64_t)j.lda * QR_NB * (int64_t)sizeof(T) >= ((int64_t)1 << 31))
      fail(IFMM_ERR_ARG, "QR of a matrix with leading dimension " + std::to_string(j.lda) + ": above the panel limit");
    off[b] = tot;
    tot += j.N + (int64_t)j.M * QR_NB + QR_NB * QR_NB + 2 * (int64_t)QR_NB * j.N + 8;
    nmax = std::max(nmax, std::min(j.M, j.N));
  }
  if ((size_t)tot * sizeof(T) > S.w.bytes) {
    P.sync();
    S.w.alloc((size_t)tot * sizeof(T) * 5 / 4 + 64, &P.mem);
  }
  T* W = S.w.template as<T>();
  double panel_total = 0;
  for (int j0 = 0; j0 < nmax; j0 += QR_NB) {
    std::vector<QrPanel> pv;
    GemmBatch g1, g2, g3;
    for (size_t b = 0; b < jobs.size(); ++b) {
      const auto& j = jobs[b];
      const int kq = std::min(j.M, j.N);
      if (j0 >= kq) continue;
      const int nb = std::min(QR_NB, kq - j0);
      T* al = W + off[b];
      T* Vb = al + j.N;
      T* Tb = Vb + (int64_t)j.M * QR_NB;
      T* W1 = Tb + QR_NB * QR_NB;
      T* W2 = W1 + (int64_t)QR_NB * j.N;
      QrPanel q;
      q.A = j.A; q.V = Vb; q.Tm = Tb; q.alph = al;
      q.M = j.M; q.N = j.N; q.lda = j.lda; q.j0 = j0; q.nb = nb; q.pad = 0;
      pv.push_back(q);
      const int rest = j.N - j0 - nb;
      if (rest > 0) {
        T* A2 = static_cast<T*>(j.A) + j0 + (int64_t)(j0 + nb) * j.lda;
        const int mv = j.M - j0;
        g1.add(Vb, mv, 1, A2, j.lda, 0, W1, nb, nb, rest, mv, 1.0, 0.0);          // W1 = V^T A2
        g2.add(Tb, nb, 1, W1, nb, 0, W2, nb, nb, rest, nb, 1.0, 0.0);            // W2 = T^T W1
        g3.add(Vb, mv, 0, W2, nb, 0, A2, j.lda, mv, rest, nb, -1.0, 1.0);        // A2 -= V W2
      }
    }
    if (pv.empty()) break;
    if ((trace_on() || qr_stats_on()) && j0 == 0) {
      int64_t sm = 0;
      int mx = 0, nx = 0;
      for (const auto& q : pv) { sm += q.M; mx = std::max(mx, q.M); nx = std::max(nx, q.N); }
      std::fprintf(stderr, "[ifmm-trace] qr level=%d jobs=%zu maxM=%d meanM=%.0f maxN=%d panels=%d\n",
                   P.trace_level, pv.size(), mx, (double)sm / pv.size(), nx, (nmax + QR_NB - 1) / QR_NB);
    }
    const QrPanel* dp = P.put(S.pd, pv);
    double fl = 0;   // Householder panel: 2 (M - j0) nb^2 - 2/3 nb^3
    for (const auto& q : pv) fl += 2.0 * (q.M - q.j0) * (double)q.nb * q.nb - 2.0 / 3.0 * (double)q.nb * q.nb * q.nb;
    panel_total += fl;
    P.kone_begin(KF_QR_PANEL, fl);
    hipLaunchKernelGGL(k_qr_panel<T>, dim3((unsigned)pv.size()), dim3(QR_WG), QR_LDS * sizeof(T), P.stream, dp);
    IFMM_LAUNCH_CHECK();
    P.kone_end();
    run_gemm<T>(P, g1, S.gd);
    run_gemm<T>(P, g2, S.gd);
    run_gemm<T>(P, g3, S.gd);
  }
  std::vector<QrOut> ov;
  for (size_t b = 0; b < jobs.size(); ++b) {
    const auto& j = jobs[b];
    if (!j.R || std::min(j.M, j.N) == 0) continue;
    ov.push_back({j.A, W + off[b], j.R, j.M, j.N, j.lda, j.ldr});
  }
  if (!ov.empty()) {
    const QrOut* d = P.put(S.pd, ov);
    P.kbegin();
    hipLaunchKernelGGL(k_qr_extract<T>, dim3((unsigned)ov.size()), dim3(WG), 0, P.stream, d);
    IFMM_LAUNCH_CHECK();
    P.kend();
  }
  // the panels' share of the caller's QR flops is counted in their own family
  if (P.kt.on && P.kcur >= 0) P.kt.flops[P.kcur] -= panel_total;
}

}  // namespace ifmm
