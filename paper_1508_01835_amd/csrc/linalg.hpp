// Batched, variable-size dense linear algebra on gfx950: GEMM, LU with partial
// pivoting and its solve, Householder QR, block copies.
// Every batch is described by an array of descriptors in device memory; one
// workgroup (or a set of tiles) serves one descriptor.
#pragma once

#include <type_traits>

#include "common.hpp"

namespace ifmm {

constexpr int WG = 256;     // threads per workgroup (4 wavefronts of 64)
constexpr int WAVE = 64;

// ---------------------------------------------------------------- reductions
template <class T>
__device__ inline T wave_sum(T v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
  return v;
}

template <class T>
__device__ inline T block_sum(T v, T* sh /* >= WG/WAVE */) {
  v = wave_sum(v);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) s += sh[i];
  __syncthreads();
  return s;
}

// Sum of 32 per-lane values over the 64 lanes of a wavefront, reduce-scattered:
// each exchange halves the values a lane keeps, so the whole reduction takes
// 32 shuffles instead of 32 x 6. On return lanes 2c and 2c+1 hold the sum of
// value c.
template <class T>
__device__ inline T wave_sum32_scatter(const T (&v)[32], int lane) {
  T a[16];
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const T keep = hi ? v[k + 16] : v[k], send = hi ? v[k] : v[k + 16];
      a[k] = keep + __shfl_xor(send, 32, WAVE);
    }
  }
  T b[8];
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T keep = hi ? a[k + 8] : a[k], send = hi ? a[k] : a[k + 8];
      b[k] = keep + __shfl_xor(send, 16, WAVE);
    }
  }
  T c[4];
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T keep = hi ? b[k + 4] : b[k], send = hi ? b[k] : b[k + 4];
      c[k] = keep + __shfl_xor(send, 8, WAVE);
    }
  }
  T e[2];
  {
    const bool hi = lane & 4;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T keep = hi ? c[k + 2] : c[k], send = hi ? c[k] : c[k + 2];
      e[k] = keep + __shfl_xor(send, 4, WAVE);
    }
  }
  const bool hi = lane & 2;
  T f = (hi ? e[1] : e[0]) + __shfl_xor(hi ? e[0] : e[1], 2, WAVE);
  return f + __shfl_xor(f, 1, WAVE);
}

template <class T>
__device__ inline T wave_max(T v) {
  for (int o = WAVE / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
  return v;
}

template <class T>
__device__ inline T block_max(T v, T* sh /* >= WG/WAVE */) {
  v = wave_max(v);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < (int)(blockDim.x / WAVE); ++i) s = fmax(s, sh[i]);
  __syncthreads();
  return s;
}

// =================================================================== GEMM
// C = alpha * op(A) * op(B) + beta * C, op(A) is M x K, op(B) is K x N.
struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  int M, N, K;
  int lda, ldb, ldc;
  int tA, tB;
  double alpha, beta;
  int tile0;       // first tile of this problem in the flattened grid
  int tiles_n;     // tiles along N
};

constexpr int GT = 64;   // output tile edge
constexpr int GK = 16;   // K chunk

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// One 16 x 16 x 4 matrix-core step in the precision of T (FP32 accumulates in
// FP32, FP64 in FP64). Both take from lane l the entry A[l % 16][l / 16] of a
// 16 x 4 slice and B[l / 16][l % 16] of a 4 x 16 slice. Their outputs are laid
// out differently: lane l's register r holds D[4 r + l / 16][l % 16] for
// v_mfma_f64_16x16x4f64 and D[4 (l / 16) + r][l % 16] for
// v_mfma_f32_16x16x4f32 (both checked on the device).
__device__ inline v4d mfma16(double a, double b, v4d c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
__device__ inline v4f mfma16(float a, float b, v4f c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
template <class T>
__device__ inline int mfma16_row(int lane, int r) {
  return std::is_same<T, double>::value ? 4 * r + (lane >> 4) : 4 * (lane >> 4) + r;
}

// Batched GEMM on the matrix cores: a 64 x 64 output tile per workgroup, each
// wavefront a 32 x 32 quarter (rows 32 (w / 2).., columns 32 (w % 2)..) as
// 2 x 2 blocks of 16 x 16; op(A) and op(B) staged through LDS in K chunks of 16.
template <class T>
__global__ void __launch_bounds__(WG) k_gemm(const GemmDesc* __restrict__ ds, int nd) {
  // find the problem owning this tile (descriptors sorted by tile0)
  int lo = 0, hi = nd - 1;
  const int t = blockIdx.x;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (ds[mid].tile0 <= t) lo = mid; else hi = mid - 1;
  }
  const GemmDesc d = ds[lo];
  const int local = t - d.tile0;
  const int tm = local / d.tiles_n, tn = local % d.tiles_n;
  const int m0 = tm * GT, n0 = tn * GT;
  if (m0 >= d.M || n0 >= d.N) return;
  const T* __restrict__ A = static_cast<const T*>(d.A);
  const T* __restrict__ B = static_cast<const T*>(d.B);
  T* __restrict__ C = static_cast<T*>(d.C);
  __shared__ T As[GK][GT + 1];
  __shared__ T Bs[GK][GT + 1];
  using acc_t = typename std::conditional<std::is_same<T, double>::value, v4d, v4f>::type;
  acc_t mfa[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) mfa[i] = acc_t{0, 0, 0, 0};
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int rb0 = 32 * (wv >> 1), cb0 = 32 * (wv & 1);
  for (int k0 = 0; k0 < d.K; k0 += GK) {
    // load op(A)[m0:m0+64, k0:k0+16] and op(B)[k0:k0+16, n0:n0+64]
    for (int e = threadIdx.x; e < GT * GK; e += WG) {
      int mm, kk;
      if (d.tA == 0) { mm = e % GT; kk = e / GT; } else { kk = e % GK; mm = e / GK; }
      const int gm = m0 + mm, gk = k0 + kk;
      T v = 0;
      if (gm < d.M && gk < d.K)
        v = d.tA == 0 ? A[(int64_t)gm + (int64_t)gk * d.lda] : A[(int64_t)gk + (int64_t)gm * d.lda];
      As[kk][mm] = v;
      int nn;
      if (d.tB == 0) { kk = e % GK; nn = e / GK; } else { nn = e % GT; kk = e / GT; }
      const int gn = n0 + nn;
      const int gk2 = k0 + kk;
      T w = 0;
      if (gn < d.N && gk2 < d.K)
        w = d.tB == 0 ? B[(int64_t)gk2 + (int64_t)gn * d.ldb] : B[(int64_t)gn + (int64_t)gk2 * d.ldb];
      Bs[kk][nn] = w;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < GK; k4 += 4) {
      const int kk = k4 + (lane >> 4);
      const T a0 = As[kk][rb0 + (lane & 15)], a1 = As[kk][rb0 + 16 + (lane & 15)];
      const T b0 = Bs[kk][cb0 + (lane & 15)], b1 = Bs[kk][cb0 + 16 + (lane & 15)];
      mfa[0] = mfma16(a0, b0, mfa[0]);
      mfa[1] = mfma16(a0, b1, mfa[1]);
      mfa[2] = mfma16(a1, b0, mfa[2]);
      mfa[3] = mfma16(a1, b1, mfa[3]);
    }
    __syncthreads();
  }
  const T alpha = (T)d.alpha, beta = (T)d.beta;
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int gn = n0 + cb0 + 16 * (blk & 1) + (lane & 15);
    if (gn >= d.N) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gm = m0 + rb0 + 16 * (blk >> 1) + mfma16_row<T>(lane, r);
      if (gm >= d.M) continue;
      T* c = &C[(int64_t)gm + (int64_t)gn * d.ldc];
      const T v = mfa[blk][r];
      *c = beta == (T)0 ? alpha * v : alpha * v + beta * (*c);
    }
  }
}

// Host-side batch builder: append problems, then launch once.
struct GemmBatch {
  std::vector<GemmDesc> v;
  int tiles = 0;
  void add(const void* A, int lda, int tA, const void* B, int ldb, int tB, void* C, int ldc,
           int M, int N, int K, double alpha, double beta) {
    if (M <= 0 || N <= 0) return;
    GemmDesc d;
    d.A = A; d.B = B; d.C = C; d.M = M; d.N = N; d.K = K; d.lda = lda; d.ldb = ldb; d.ldc = ldc;
    d.tA = tA; d.tB = tB; d.alpha = alpha; d.beta = beta;
    d.tiles_n = (int)ceil_div(N, GT);
    d.tile0 = tiles;
    tiles += (int)ceil_div(M, GT) * d.tiles_n;
    v.push_back(d);
  }
  void clear() { v.clear(); tiles = 0; }
};

// ================================================================ LU
struct LuDesc {
  void* A;       // n x n, column-major, leading dimension lda; overwritten by L\U
  int* piv;      // n: row k was swapped with row piv[k] (0-based)
  int n, lda;
  int tag;       // reported through *info when a zero pivot is met
  int pad;
};

template <class T>
__global__ void __launch_bounds__(WG) k_lu(const LuDesc* __restrict__ ds, int* info) {
  const LuDesc d = ds[blockIdx.x];
  T* __restrict__ A = static_cast<T*>(d.A);
  const int n = d.n;
  const int64_t ld = d.lda;
  __shared__ T smax[WG];
  __shared__ int sidx[WG];
  __shared__ T spv;
  __shared__ int sp;
  for (int k = 0; k < n; ++k) {
    T best = -1;
    int bi = k;
    for (int i = k + threadIdx.x; i < n; i += WG) {
      T v = fabs(A[i + k * ld]);
      if (v > best) { best = v; bi = i; }
    }
    smax[threadIdx.x] = best;
    sidx[threadIdx.x] = bi;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        T o = smax[threadIdx.x + s];
        int oi = sidx[threadIdx.x + s];
        if (o > smax[threadIdx.x] || (o == smax[threadIdx.x] && oi < sidx[threadIdx.x])) {
          smax[threadIdx.x] = o;
          sidx[threadIdx.x] = oi;
        }
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      sp = sidx[0];
      d.piv[k] = sp;
      if (!(smax[0] > (T)0) && info) atomicCAS(info, -1, d.tag);
    }
    __syncthreads();
    const int p = sp;
    if (p != k)
      for (int j = threadIdx.x; j < n; j += WG) {
        T a = A[k + j * ld];
        A[k + j * ld] = A[p + j * ld];
        A[p + j * ld] = a;
      }
    __syncthreads();
    if (threadIdx.x == 0) spv = A[k + k * ld];
    __syncthreads();
    const T pv = spv;
    const T inv = pv != (T)0 ? (T)1 / pv : (T)0;
    for (int i = k + 1 + threadIdx.x; i < n; i += WG) A[i + k * ld] *= inv;
    __syncthreads();
    const int rem = n - k - 1;
    for (int e = threadIdx.x; e < rem * rem; e += WG) {
      const int i = k + 1 + e % rem, j = k + 1 + e / rem;
      A[i + j * ld] -= A[i + k * ld] * A[k + j * ld];
    }
    __syncthreads();
  }
}

// Solve (L U) X = P B in place: B is n x nrhs (leading dimension ldb).
struct LuSolveDesc {
  const void* LU;
  const int* piv;
  void* B;
  int n, lda, nrhs, ldb;
  int blk0;     // first 1D block of this problem
  int pad;
};

template <class T>
__global__ void __launch_bounds__(WG) k_lu_solve(const LuSolveDesc* __restrict__ ds, int nd) {
  int lo = 0, hi = nd - 1;
  const int t = blockIdx.x;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (ds[mid].blk0 <= t) lo = mid; else hi = mid - 1;
  }
  const LuSolveDesc d = ds[lo];
  const int col = (t - d.blk0) * WG + threadIdx.x;
  if (col >= d.nrhs) return;
  const T* __restrict__ LU = static_cast<const T*>(d.LU);
  T* __restrict__ b = static_cast<T*>(d.B) + (int64_t)col * d.ldb;
  const int n = d.n;
  const int64_t ld = d.lda;
  for (int k = 0; k < n; ++k) {
    const int p = d.piv[k];
    if (p != k) { T a = b[k]; b[k] = b[p]; b[p] = a; }
  }
  for (int k = 0; k < n; ++k) {
    const T bk = b[k];
    if (bk != (T)0)
      for (int i = k + 1; i < n; ++i) b[i] -= LU[i + k * ld] * bk;
  }
  for (int k = n - 1; k >= 0; --k) {
    const T bk = b[k] / LU[k + k * ld];
    b[k] = bk;
    if (bk != (T)0)
      for (int i = 0; i < k; ++i) b[i] -= LU[i + k * ld] * bk;
  }
}

struct LuSolveBatch {
  std::vector<LuSolveDesc> v;
  int blocks = 0;
  void add(const void* LU, int lda, const int* piv, void* B, int ldb, int n, int nrhs) {
    if (n <= 0 || nrhs <= 0) return;
    LuSolveDesc d;
    d.LU = LU; d.piv = piv; d.B = B; d.n = n; d.lda = lda; d.nrhs = nrhs; d.ldb = ldb;
    d.blk0 = blocks; d.pad = 0;
    blocks += (int)ceil_div(nrhs, WG);
    v.push_back(d);
  }
};

// ================================================================ QR
// Householder QR of A (M x N, lda), in place. On exit R (kq x N, upper
// trapezoidal, kq = min(M, N)) is written to Rout (ldr) and, if Qout is not
// null, the thin orthonormal factor Q (M x kq) to Qout (ldq).
struct QrDesc {
  void* A;
  void* R;
  void* Q;
  int M, N, lda, ldr, ldq;
  int pad;
};

constexpr int QR_MAXK = 1024;

template <class T>
__global__ void __launch_bounds__(WG) k_qr(const QrDesc* __restrict__ ds) {
  const QrDesc d = ds[blockIdx.x];
  T* __restrict__ A = static_cast<T*>(d.A);
  T* __restrict__ R = static_cast<T*>(d.R);
  T* __restrict__ Q = static_cast<T*>(d.Q);
  const int M = d.M, N = d.N;
  const int64_t lda = d.lda, ldr = d.ldr, ldq = d.ldq;
  const int kq = M < N ? M : N;
  __shared__ T tau[QR_MAXK];
  __shared__ T alph[QR_MAXK];
  __shared__ T red[WG / WAVE];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = WG / WAVE;
  for (int j = 0; j < kq; ++j) {
    // reflector H = I - tau v v^T with v_j = 1 and beta = -sign(x0) ||x||; the
    // norm is taken on the column scaled by the power of two nearest its
    // largest entry (exact, and finite for subnormal columns) so that tiny or
    // huge columns neither underflow nor overflow
    T amax = 0;
    for (int i = j + threadIdx.x; i < M; i += WG) amax = fmax(amax, fabs(A[i + j * lda]));
    amax = block_max(amax, red);
    const T x0 = A[j + j * lda];
    T tj = 0, al = x0;
    if (amax > (T)0) {
      const int sh = -ilogb((double)amax);
      T s = 0;
      for (int i = j + threadIdx.x; i < M; i += WG) { const T x = ldexp(A[i + j * lda], sh); s += x * x; }
      s = block_sum(s, red);
      const T x0s = ldexp(x0, sh);
      const T als = x0s >= (T)0 ? -sqrt(s) : sqrt(s);
      al = ldexp(als, -sh);
      tj = (als - x0s) / als;
      const T scal = (T)1 / (x0s - als);
      for (int i = j + 1 + threadIdx.x; i < M; i += WG) A[i + j * lda] = ldexp(A[i + j * lda], sh) * scal;
      __syncthreads();
      if (threadIdx.x == 0) A[j + j * lda] = (T)1;
    }
    if (threadIdx.x == 0) { tau[j] = tj; alph[j] = al; }
    __syncthreads();
    if (tj != (T)0) {
      for (int c = j + 1 + wv; c < N; c += nw) {
        T dot = 0;
        for (int i = j + lane; i < M; i += WAVE) dot += A[i + j * lda] * A[i + c * lda];
        dot = wave_sum(dot) * tj;
        for (int i = j + lane; i < M; i += WAVE) A[i + c * lda] -= dot * A[i + j * lda];
      }
    }
    __syncthreads();
  }
  if (R) {
    for (int e = threadIdx.x; e < kq * N; e += WG) {
      const int i = e % kq, c = e / kq;
      T v = 0;
      if (i == c) v = alph[i];
      else if (i < c) v = A[i + c * lda];
      R[i + c * ldr] = v;
    }
  }
  if (Q) {
    for (int e = threadIdx.x; e < M * kq; e += WG) {
      const int i = e % M, c = e / M;
      Q[i + c * ldq] = i == c ? (T)1 : (T)0;
    }
    __syncthreads();
    for (int j = kq - 1; j >= 0; --j) {
      const T tj = tau[j];
      if (tj != (T)0) {
        for (int c = j + wv; c < kq; c += nw) {
          T dot = 0;
          for (int i = j + lane; i < M; i += WAVE) dot += A[i + j * lda] * Q[i + c * ldq];
          dot = wave_sum(dot) * tj;
          for (int i = j + lane; i < M; i += WAVE) Q[i + c * ldq] -= dot * A[i + j * lda];
        }
      }
      __syncthreads();
    }
  }
}

// ============================================================ block copies
// dst[i, j] (op)= alpha * src[i, j] * (cs ? cs[j] : 1). mode 0: assign,
// 1: accumulate, 2: assign alpha * identity (src unused), 3: assign zero,
// 4: assign alpha * src[j, i] (transpose; dst is rows x cols).
template <class Ts, class Td>
struct CopyDesc {
  const Ts* src;
  Td* dst;
  const Ts* cs;
  int rows, cols, lds, ldd;
  int mode, j0;   // j0: first column of this piece (large copies are split into pieces of columns)
  double alpha;
};

template <class Ts, class Td>
__global__ void __launch_bounds__(WG) k_copy(const CopyDesc<Ts, Td>* __restrict__ ds, int nd) {
  const int b = blockIdx.y * gridDim.x + blockIdx.x;
  if (b >= nd) return;
  const CopyDesc<Ts, Td> d = ds[b];
  auto one = [&](int i, int jl) {
    const int j = jl + d.j0;
    Td* o = &d.dst[i + (int64_t)j * d.ldd];
    if (d.mode == 3) { *o = (Td)0; return; }
    if (d.mode == 2) { *o = i == j ? (Td)d.alpha : (Td)0; return; }
    if (d.mode == 4) { *o = (Td)(d.alpha * (double)d.src[j + (int64_t)i * d.lds]); return; }
    double v = d.alpha * (double)d.src[i + (int64_t)j * d.lds];
    if (d.cs) v *= (double)d.cs[j];
    if (d.mode == 1) *o = (Td)((double)*o + v);
    else *o = (Td)v;
  };
  if (d.rows >= WAVE) {   // a wavefront per column of the piece, lanes down the rows: coalesced
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
    for (int j = wv; j < d.cols; j += WG / WAVE)
      for (int i = lane; i < d.rows; i += WAVE) one(i, j);
  } else {                // short columns: several per wavefront
    const int64_t total = (int64_t)d.rows * d.cols;
    if (total < (int64_t)1 << 31) {
      for (int e = threadIdx.x; e < (int)total; e += WG) one(e % d.rows, e / d.rows);
    } else {
      for (int64_t e = threadIdx.x; e < total; e += WG) one((int)(e % d.rows), (int)(e / d.rows));
    }
  }
}

template <class Ts, class Td>
struct CopyBatch {
  std::vector<CopyDesc<Ts, Td>> v;
  void add(const Ts* src, int lds, Td* dst, int ldd, int rows, int cols, int mode = 0,
           double alpha = 1.0, const Ts* cs = nullptr) {
    if (rows <= 0 || cols <= 0) return;
    // pieces of at most 32 columns (one workgroup each) for tall copies
    const int piece = rows >= 64 ? 32 : cols;
    for (int j0 = 0; j0 < cols; j0 += piece) {
      CopyDesc<Ts, Td> d;
      d.src = src; d.dst = dst; d.cs = cs; d.rows = rows; d.cols = std::min(piece, cols - j0); d.lds = lds;
      d.ldd = ldd; d.mode = mode; d.j0 = j0; d.alpha = alpha;
      v.push_back(d);
    }
  }
};

}  // namespace ifmm
