// Batched one-sided Jacobi SVD (Hestenes) of variable-size matrices. The
// recompressions need the left singular vectors and the singular values only:
// the columns of B are orthogonalised by plane rotations, their norms are the
// singular values and the normalised columns the left singular vectors.
//
// Two schemes, chosen per matrix:
//  - small: one workgroup per matrix, the matrix copied into LDS (the many
//    small matrices of the fine levels);
//  - block: the columns are split in blocks of nb; one round of a round-robin
//    tournament over the blocks is one launch in which one workgroup takes one
//    pair of blocks into LDS and rotates its column pairs: in round 0 all
//    pairs of its 2 nb columns, in later rounds only the pairs across the two
//    blocks, so that a sweep visits every column pair once. All pairs of all
//    matrices of a batch run side by side, so a colour class with only a few
//    large matrices still spreads over the chip.
//
// Rotation rule (both schemes), with a, b the squared norms of columns p, q
// and g their inner product: rotate iff |g| > tol sqrt(a b), with
// tol = max(4, sqrt(M)) u: the computed cosine carries a rounding error that
// grows like sqrt(M) u, and chasing cosines below that only re-rotates noise
// (the threshold of LAPACK's one-sided Jacobi). Columns of norm below defl
// (absolute) are frozen: they lie far under the truncation threshold and are
// discarded by the caller.
#pragma once

#include "problem.hpp"

namespace ifmm {

struct SvdDesc {
  void* B;              // M x N, ldb; overwritten
  void* U;              // M x N, ldu: normalised columns by decreasing norm (zero norm: zeros)
  void* S;              // N: the singular values, decreasing
  const int* nlive;     // optional (device): only the first *nlive columns of B are nonzero
  const int* perm;      // optional (device, M): row i of B is row perm[i] of U
  int M, N, ldb, ldu;
};

constexpr int SVD_MAXN = 1024;   // widest problem of the step-wise pivoted QR (LDS arrays and rows per thread)
constexpr int SVD_MAXK = 2048;   // most live columns of one Jacobi SVD (the pivoted QR keeps at most that many)

// live columns: at most SVD_MAXK
__device__ inline int svd_cols(const SvdDesc& d) {
  return d.nlive ? max(0, min(min(d.N, SVD_MAXK), *d.nlive)) : d.N;
}
constexpr int SVD_WG = 1024;                // 16 wavefronts: 16 column pairs at once
constexpr size_t SVD_LDS_MAX = 128 * 1024;  // dynamic LDS per workgroup (gfx950: 160 KB, 24 KB static for the norms)

// Rotates columns p and q of B (ld) when the rule above asks for it; one
// wavefront. nrm2 holds the squared column norms: only the inner product is
// reduced across the wavefront, and the two norms are updated exactly for the
// rotation that zeroes it (a' = a - t g, b' = b + t g); callers recompute them
// at every sweep (meeting) start, as LAPACK's one-sided Jacobi does. Returns
// whether it rotated (uniform over the wavefront).
template <class T>
__device__ inline bool jacobi_rot(T* __restrict__ B, int64_t ld, int M, int p, int q, T tol, T defl2, int lane,
                                  T* nrm2) {
  const T a = nrm2[p], b = nrm2[q];
  if (a < defl2 || b < defl2) return false;
  T g = 0;
  for (int i = lane; i < M; i += WAVE) g += B[i + p * ld] * B[i + q * ld];
  g = wave_sum(g);
  if (!(fabs(g) > tol * sqrt(a * b))) return false;
  const T zeta = (b - a) / ((T)2 * g);
  const T t = (zeta >= (T)0 ? (T)1 : (T)-1) / (fabs(zeta) + sqrt((T)1 + zeta * zeta));
  const T c = (T)1 / sqrt((T)1 + t * t);
  const T s = c * t;
  for (int i = lane; i < M; i += WAVE) {
    const T x = B[i + p * ld], y = B[i + q * ld];
    B[i + p * ld] = c * x - s * y;
    B[i + q * ld] = s * x + c * y;
  }
  if (lane == 0) {
    nrm2[p] = fmax((T)0, a - t * g);
    nrm2[q] = b + t * g;
  }
  return true;
}

// Squared norms of the nc columns of B into nrm2; whole workgroup.
template <class T>
__device__ inline void col_norms2(const T* __restrict__ B, int64_t ld, int M, int nc, T* nrm2) {
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  for (int c = wv; c < nc; c += nw) {
    T s = 0;
    for (int i = lane; i < M; i += WAVE) { const T x = B[i + c * ld]; s += x * x; }
    s = wave_sum(s);
    if (lane == 0) nrm2[c] = s;
  }
  __syncthreads();
}

// Pair (x, y) of player slot pr in round r of a round-robin tournament over
// np (even) players: player 0 stays, the others rotate.
__device__ inline void rr_pair(int np, int r, int pr, int& x, int& y) {
  if (pr == 0) { x = 0; y = 1 + (r % (np - 1)); }
  else {
    x = 1 + ((r + pr) % (np - 1));
    y = 1 + ((r + np - 1 - pr) % (np - 1));
  }
}

// Cyclic sweeps over the nc columns of B (ld) until a sweep rotates nothing or
// max_sweeps; whole workgroup. Returns the sweeps done, *any = whether any
// rotation happened.
template <class T>
__device__ inline int jacobi_sweeps(T* __restrict__ B, int64_t ld, int M, int nc, T tol, T defl2, int max_sweeps,
                                    int* any, int* flag, T* nrm2) {
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  const int np = nc + (nc & 1);
  int sweeps = 0;
  if (nc < 2) return 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    sweeps = sweep + 1;
    if (threadIdx.x == 0) *flag = 0;
    col_norms2(B, ld, M, nc, nrm2);
    bool rot = false;
    for (int r = 0; r < np - 1; ++r) {
      for (int pr = wv; pr < np / 2; pr += nw) {
        int x, y;
        rr_pair(np, r, pr, x, y);
        if (x < nc && y < nc) rot |= jacobi_rot(B, ld, M, min(x, y), max(x, y), tol, defl2, lane, nrm2);
      }
      __syncthreads();
    }
    if (rot && lane == 0) *flag = 1;
    __syncthreads();
    const int f = *flag;
    __syncthreads();
    if (!f) break;
    *any = 1;
  }
  return sweeps;
}

// Column norms, order by decreasing norm (ties by index), U = B / norm,
// S = norm * 2^-sh over the N live columns (rows placed through perm when
// given); columns N..Nout-1 of U and S are zero. Whole workgroup; N <= SVD_MAXK.
template <class T>
__device__ inline void svd_finish(const T* __restrict__ B, int64_t ldb, int M, int N, int Nout, T* __restrict__ U,
                                  int64_t ldu, T* __restrict__ S, int sh, const int* __restrict__ perm, T* nrm,
                                  int* order) {
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
  for (int c = wv; c < N; c += nw) {
    T s = 0;
    for (int i = lane; i < M; i += WAVE) { const T x = B[i + c * ldb]; s += x * x; }
    s = wave_sum(s);
    if (lane == 0) nrm[c] = sqrt(s);
  }
  __syncthreads();
  // rank of each column in decreasing order of norm; a NaN norm ranks last
  // (as -1) so that the ranks stay a permutation
  for (int c = threadIdx.x; c < N; c += blockDim.x) {
    const T v = nrm[c] == nrm[c] ? nrm[c] : (T)-1;
    int rk = 0;
    for (int j = 0; j < N; ++j) {
      const T w = nrm[j] == nrm[j] ? nrm[j] : (T)-1;
      rk += (w > v) || (w == v && j < c);
    }
    order[rk] = c;
  }
  __syncthreads();
  for (int c = wv; c < N; c += nw) {
    const int src = order[c];
    const T s = nrm[src];
    for (int i = lane; i < M; i += WAVE)
      U[(perm ? perm[i] : i) + c * ldu] = s > (T)0 ? B[i + src * ldb] / s : (T)0;
    if (lane == 0) S[c] = ldexp(s, -sh);
  }
  for (int c = N + wv; c < Nout; c += nw) {
    for (int i = lane; i < M; i += WAVE) U[i + c * ldu] = (T)0;
    if (lane == 0) S[c] = (T)0;
  }
}

// B scaled into D (ldd) by 2^sh, the power of two that brings the largest
// entry into [1, 2) (exact; finite also for subnormal entries); whole
// workgroup. Returns sh (0 for a zero matrix).
template <class T>
__device__ inline int svd_scale(const T* B, int64_t ldb, int M, int N, T* D, int64_t ldd, T* red) {
  T m = 0;
  for (int64_t e = threadIdx.x; e < (int64_t)M * N; e += blockDim.x) m = fmax(m, fabs(B[e % M + (e / M) * ldb]));
  const T amax = block_max(m, red);
  const int sh = amax > (T)0 ? -ilogb((double)amax) : 0;
  for (int64_t e = threadIdx.x; e < (int64_t)M * N; e += blockDim.x)
    D[e % M + (e / M) * ldd] = ldexp(B[e % M + (e / M) * ldb], sh);
  return sh;
}

// ------------------------------------------------------------- small scheme
template <class T>
__global__ void __launch_bounds__(SVD_WG) k_svd_small(const SvdDesc* __restrict__ ds, double u, int max_sweeps, double defl, int use_lds,
                                                   int* __restrict__ sweeps_out) {
  extern __shared__ unsigned char svd_dyn[];
  __shared__ T red[SVD_WG / WAVE];
  __shared__ T nrm[SVD_MAXK];
  __shared__ int order[SVD_MAXK];
  __shared__ int flag;
  const SvdDesc d = ds[blockIdx.x];
  T* Bg = static_cast<T*>(d.B);
  const int M = d.M, N = svd_cols(d);
  // the matrix is rotated in LDS when it fits, in place otherwise
  T* B = use_lds ? reinterpret_cast<T*>(svd_dyn) : Bg;
  const int64_t ldb = use_lds ? (int64_t)M : (int64_t)d.ldb;
  const int sh = svd_scale(Bg, d.ldb, M, N, B, ldb, red);
  __syncthreads();
  const T defl_s = (T)ldexp(defl, sh);
  const T tol = (T)(u * fmax(4.0, sqrt((double)M)));
  int any = 0;
  const int sw = jacobi_sweeps(B, ldb, M, N, tol, defl_s * defl_s, max_sweeps, &any, &flag, nrm);
  if (sweeps_out && threadIdx.x == 0) atomicMax(sweeps_out, sw);
  svd_finish(B, ldb, M, N, d.N, static_cast<T*>(d.U), d.ldu, static_cast<T*>(d.S), sh, d.perm, nrm, order);
}

// ------------------------------------------------------------- lane scheme
// Matrices of at most NP rows and NP live columns (NP = 16, 32 or 64): a lane
// per column pair. The NP / 2 lanes of a matrix each take one pair of the
// round of the same tournament as the small scheme, form its inner product
// over the rows and rotate it, so a round costs one pass over the rows and no
// cross-lane reduction; 128 / NP matrices share a wavefront and each keeps
// its own sweep count. Same rotation rule, sweeps and outputs as k_svd_small.
template <class T, int NP>
struct SvdLanes {
  static constexpr int PPW = 2 * WAVE / NP;    // matrices per wavefront
  static constexpr int WAVES = 4 * 16 / NP;    // wavefronts per workgroup
};

template <class T, int NP, int NT = SvdLanes<T, NP>::WAVES * WAVE>
__global__ void __launch_bounds__(NT) k_svd_lanes(const SvdDesc* __restrict__ ds, int nd, double u, int max_sweeps,
                                                  double defl) {
  constexpr int PPW = SvdLanes<T, NP>::PPW, WAVES = SvdLanes<T, NP>::WAVES, H = NP / 2;
  __shared__ T Bs[WAVES][PPW][NP][NP + 1];   // Bs[.][.][c][i] = B[i, c]
  __shared__ T nrs[WAVES][PPW][NP];
  __shared__ int ords[WAVES][PPW][NP];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int grp = lane / H, k = lane % H;
  const int prob = ((int)blockIdx.x * WAVES + w) * PPW + grp;
  const bool valid = prob < nd;
  SvdDesc d{};
  if (valid) d = ds[prob];
  const T* Bg = static_cast<const T*>(d.B);
  const int M = valid ? d.M : 0, N = valid ? svd_cols(d) : 0;
  T (*B)[NP + 1] = Bs[w][grp];
  T* nr = nrs[w][grp];
  int* ord = ords[w][grp];
  auto wsync = [] {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  };
  // exact power-of-two scaling of each matrix: its largest entry into [1, 2)
  T am = 0;
  for (int c = k; c < N; c += H)
    for (int i = 0; i < M; ++i) am = fmax(am, fabs(Bg[i + (int64_t)c * d.ldb]));
#pragma unroll
  for (int o = H / 2; o > 0; o >>= 1) am = fmax(am, __shfl_xor(am, o, WAVE));
  const int sh = am > (T)0 ? -ilogb((double)am) : 0;
  for (int c = k; c < NP; c += H)
    for (int i = 0; i < NP; ++i) B[c][i] = (c < N && i < M) ? ldexp(Bg[i + (int64_t)c * d.ldb], sh) : (T)0;
  const T defl_s = (T)ldexp(defl, sh);
  const T defl2 = defl_s * defl_s;
  const T tol = (T)(u * fmax(4.0, sqrt((double)max(M, 1))));
  auto norms2 = [&] {   // squared norms of the lane's two columns
    for (int c = k; c < N; c += H) {
      T s0 = 0, s1 = 0;
      for (int i = 0; i < M; i += 2) {
        s0 += B[c][i] * B[c][i];
        s1 += B[c][i + 1] * B[c][i + 1];   // row M (when M is odd) is zero padding
      }
      nr[c] = s0 + s1;
    }
  };
  const int np = N + (N & 1);
  bool live = N >= 2;   // this matrix still sweeps
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (!__builtin_amdgcn_ballot_w64(live)) break;
    if (live) norms2();
    wsync();
    bool rot = false;
    const int rmax = np - 1;
    int rw = live ? rmax : 0;   // rounds of the wavefront: the largest of its live matrices
#pragma unroll
    for (int o = H; o < WAVE; o <<= 1) rw = max(rw, __shfl_xor(rw, o, WAVE));
    for (int r = 0; r < rw; ++r) {
      if (live && r < rmax && k < np / 2) {
        int x, y;
        rr_pair(np, r, k, x, y);
        if (x < N && y < N) {
          const int p = min(x, y), q = max(x, y);
          const T a = nr[p], b = nr[q];
          if (a >= defl2 && b >= defl2) {
            T g0 = 0, g1 = 0;
            for (int i = 0; i < M; i += 2) {
              g0 += B[p][i] * B[q][i];
              g1 += B[p][i + 1] * B[q][i + 1];
            }
            const T g = g0 + g1;
            if (fabs(g) > tol * sqrt(a * b)) {
              const T zeta = (b - a) / ((T)2 * g);
              const T t = (zeta >= (T)0 ? (T)1 : (T)-1) / (fabs(zeta) + sqrt((T)1 + zeta * zeta));
              const T c = (T)1 / sqrt((T)1 + t * t);
              const T sn = c * t;
              for (int i = 0; i < M; ++i) {
                const T xp = B[p][i], yq = B[q][i];
                B[p][i] = c * xp - sn * yq;
                B[q][i] = sn * xp + c * yq;
              }
              nr[p] = fmax((T)0, a - t * g);
              nr[q] = b + t * g;
              rot = true;
            }
          }
        }
      }
      wsync();
    }
    // a matrix whose sweep rotated nothing is done
    bool any = rot;
#pragma unroll
    for (int o = H / 2; o > 0; o >>= 1) any = any || __shfl_xor((int)any, o, WAVE);
    live = live && any;
  }
  // finish: norms, decreasing order (ties by index, NaN last), U = B / norm, S
  for (int c = k; c < N; c += H) {
    T s0 = 0, s1 = 0;
    for (int i = 0; i < M; i += 2) {
      s0 += B[c][i] * B[c][i];
      s1 += B[c][i + 1] * B[c][i + 1];
    }
    nr[c] = sqrt(s0 + s1);
  }
  wsync();
  for (int c = k; c < N; c += H) {
    const T v = nr[c] == nr[c] ? nr[c] : (T)-1;
    int rk = 0;
    for (int j = 0; j < N; ++j) {
      const T x = nr[j] == nr[j] ? nr[j] : (T)-1;
      rk += (x > v) || (x == v && j < c);
    }
    ord[rk] = c;
  }
  wsync();
  if (!valid) return;
  T* U = static_cast<T*>(d.U);
  T* S = static_cast<T*>(d.S);
  for (int c = k; c < d.N; c += H) {
    if (c < N) {
      const int src = ord[c];
      const T sv = nr[src];
      for (int i = 0; i < M; ++i) U[(d.perm ? d.perm[i] : i) + (int64_t)c * d.ldu] = sv > (T)0 ? B[src][i] / sv : (T)0;
      S[c] = ldexp(sv, -sh);
    } else {
      for (int i = 0; i < M; ++i) U[i + (int64_t)c * d.ldu] = (T)0;
      S[c] = (T)0;
    }
  }
}

// ------------------------------------------------------------- block scheme
// Per matrix: shs[s] = the scaling exponent sh; flags[2s] = rotations in the
// current sweep, flags[2s + 1] = converged.
// Block bookkeeping per matrix (nbm = largest block count of the batch):
// bst[0, nbm): round stamp of the last change of each block's columns;
// bst[nbm + x nbm + y]: stamp of the last meeting of blocks x and y (y = x:
// block x alone) that rotated nothing, -1 if none since. A meeting is skipped
// when both blocks are unchanged since their last such meeting: the pairs it
// would check are still within the threshold.
template <class T>
__global__ void __launch_bounds__(SVD_WG) k_svd_prep(const SvdDesc* __restrict__ ds, int* __restrict__ shs,
                                                  int* __restrict__ flags, int* __restrict__ bst, int nbm) {
  __shared__ T red[SVD_WG / WAVE];
  const SvdDesc d = ds[blockIdx.x];
  T* B = static_cast<T*>(d.B);
  const int N = svd_cols(d);
  const int sh = svd_scale(B, d.ldb, d.M, N, B, d.ldb, red);
  int* st = bst + (int64_t)blockIdx.x * (nbm + nbm * nbm);
  for (int e = threadIdx.x; e < nbm + nbm * nbm; e += SVD_WG) st[e] = -1;
  if (threadIdx.x == 0) {
    shs[blockIdx.x] = sh;
    flags[2 * blockIdx.x] = 0;
    flags[2 * blockIdx.x + 1] = N < 2 ? 1 : 0;
  }
}

// One tournament round: blockIdx.y = matrix, blockIdx.x = pair of column blocks.
template <class T>
__global__ void __launch_bounds__(SVD_WG) k_svd_round(const SvdDesc* __restrict__ ds,
                                                   const int* __restrict__ shs, int* __restrict__ flags, int nb,
                                                   int round, double u, double defl, int inner_sweeps,
                                                   int* __restrict__ bst, int nbm, int stamp) {
  extern __shared__ unsigned char svd_dyn[];
  __shared__ int flag;
  __shared__ T nrm2[64];
  const int s = blockIdx.y;
  if (flags[2 * s + 1]) return;
  const SvdDesc d = ds[s];
  const int M = d.M, N = svd_cols(d);
  const int nblk = (N + nb - 1) / nb, np = nblk + (nblk & 1);
  if (round >= np - 1 || (int)blockIdx.x >= np / 2) return;
  int x, y;
  rr_pair(np, round, blockIdx.x, x, y);
  const int c0[2] = {x < nblk ? x * nb : 0, y < nblk ? y * nb : 0};
  const int w[2] = {x < nblk ? min(nb, N - x * nb) : 0, y < nblk ? min(nb, N - y * nb) : 0};
  const int nc = w[0] + w[1];
  if (nc < 2) return;
  if (round > 0 && (w[0] == 0 || w[1] == 0)) return;   // a block alone has no cross pairs
  int* st = bst + (int64_t)s * (nbm + nbm * nbm);
  const int bx = x < nblk ? x : y, by = y < nblk ? y : x;   // a bye meets its partner alone
  int* clean = st + nbm + bx * nbm + by;
  if (*clean >= 0 && st[bx] < *clean && st[by] < *clean) return;
  T* __restrict__ Bg = static_cast<T*>(d.B);
  T* __restrict__ L = reinterpret_cast<T*>(svd_dyn);
  for (int64_t e = threadIdx.x; e < (int64_t)M * nc; e += blockDim.x) {
    const int c = (int)(e / M), i = (int)(e % M);
    const int gc = c < w[0] ? c0[0] + c : c0[1] + (c - w[0]);
    L[e] = Bg[i + (int64_t)gc * d.ldb];
  }
  __syncthreads();
  const T defl_s = (T)ldexp(defl, shs[s]);
  const T tol = (T)(u * fmax(4.0, sqrt((double)M)));
  int any = 0;
  if (round == 0) {
    // every block takes part in round 0: its pairs inside the block are visited here, once per sweep
    jacobi_sweeps(L, (int64_t)M, M, nc, tol, defl_s * defl_s, inner_sweeps, &any, &flag, nrm2);
  } else if (w[0] > 0 && w[1] > 0) {
    // only the pairs across the two blocks: in step t wavefront a pairs column a of the first block with
    // column (a + t) mod R of the second, so no column is used twice in a step and every cross pair once
    const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = blockDim.x / WAVE;
    const int R = max(w[0], w[1]);
    if (threadIdx.x == 0) flag = 0;
    col_norms2(L, (int64_t)M, M, nc, nrm2);
    bool rot = false;
    for (int t = 0; t < R; ++t) {
      for (int a = wv; a < w[0]; a += nw) {
        const int b = (a + t) % R;
        if (b < w[1]) rot |= jacobi_rot(L, (int64_t)M, M, a, w[0] + b, tol, defl_s * defl_s, lane, nrm2);
      }
      __syncthreads();
    }
    if (rot && lane == 0) flag = 1;
    __syncthreads();
    any = flag;
  }
  if (!any) {   // nothing rotated: global memory already holds these columns
    if (threadIdx.x == 0) *clean = stamp;
    return;
  }
  for (int64_t e = threadIdx.x; e < (int64_t)M * nc; e += blockDim.x) {
    const int c = (int)(e / M), i = (int)(e % M);
    const int gc = c < w[0] ? c0[0] + c : c0[1] + (c - w[0]);
    Bg[i + (int64_t)gc * d.ldb] = L[e];
  }
  if (threadIdx.x == 0) {
    atomicAdd(&flags[2 * s], 1);
    st[bx] = stamp;
    st[by] = stamp;
    *clean = -1;
  }
}

// End of a sweep: a matrix whose sweep rotated nothing has converged.
__global__ void k_svd_sweep_end(int* __restrict__ flags, int n, int sweep, int* __restrict__ sweeps_out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n || flags[2 * s + 1]) return;
  if (flags[2 * s] == 0) {
    flags[2 * s + 1] = 1;
    if (sweeps_out) atomicMax(sweeps_out, sweep + 1);
  }
  flags[2 * s] = 0;
}

template <class T>
__global__ void __launch_bounds__(SVD_WG) k_svd_block_finish(const SvdDesc* __restrict__ ds,
                                                          const int* __restrict__ shs) {
  __shared__ T nrm[SVD_MAXK];
  __shared__ int order[SVD_MAXK];
  const SvdDesc d = ds[blockIdx.x];
  svd_finish(static_cast<const T*>(d.B), d.ldb, d.M, svd_cols(d), d.N, static_cast<T*>(d.U), d.ldu,
             static_cast<T*>(d.S), shs[blockIdx.x], d.perm, nrm, order);
}

// ------------------------------------------- truncated column-pivoted QR
// Preconditioner of the Jacobi SVD of B = R^T (Drmac-Veselic: Jacobi on the
// transposed triangular factor of a column-pivoted QR converges in a few
// sweeps). R is m x n (ld) with m <= n. Householder QR with column pivoting
// (largest remaining partial column norm; partial norms downdated and
// recomputed on cancellation) stops at the first step s where the Frobenius
// norm of the unfactorised block R[s:, s:] is at most max(delta,
// 4 u ||R||_F), so that B = P Y Q^T + E with ||E||_F below that level,
// Y = R'[0:k, :]^T (n x k) and P the column permutation. Since the left
// singular vectors of B are P times those of Y, the Jacobi SVD of Y (rows
// placed through perm) replaces that of B.
// Output: Y (n x m area, ld ldy; columns >= k not written), perm (n), *kout;
// R is overwritten.
struct QrcpDesc {
  void* R;
  void* Y;
  int* perm;
  int* kout;
  int m, n, ldr, ldy;
  int* over;   // set to 1 when more than SVD_MAXK directions stay above the stop level (the SVD takes at most that)
};

// Dynamic LDS of k_qrcp for an m x n problem: partial norms (two copies) and
// pivots of the n columns, the Householder vector of m rows.
template <class T>
inline size_t qrcp_lds(int m, int n) {
  return ((sizeof(T) * 2 + sizeof(int)) * (size_t)n + 15) / 16 * 16 + sizeof(T) * (size_t)m;
}
constexpr size_t QRCP_LDS_MAX = 144 * 1024;

// The same truncated pivoted QR for n <= NP (NP = 16, 32 or 64), a lane per
// column: 64 / NP problems share a wavefront, lane c of a problem owns
// column c (its partial norms and its place in the pivoted order), and the
// problem's R sits in LDS. The pivot is a reduction over the problem's lanes
// (largest partial norm, first place on ties); columns are not moved, their
// places are; the reflector's norm is a reduction with lane i reading row i
// (m <= n <= NP); each trailing column applies it, downdates or recomputes
// its partial norm in its own lane. Same stop rule and outputs as k_qrcp.
template <class T, int NP>
struct QrcpLanes {
  static constexpr int G = WAVE / NP;
  static constexpr int PER_WAVE = (int)sizeof(T) * G * NP * (NP + 1);
  static constexpr int WAVES = PER_WAVE * 8 <= 69632 ? 8 : PER_WAVE * 4 <= 69632 ? 4 : 2;
};

template <class T, int NP, int NT = QrcpLanes<T, NP>::WAVES * WAVE>
__global__ void __launch_bounds__(NT) k_qrcp_lanes(const QrcpDesc* __restrict__ ds, int nd, double delta) {
  constexpr int G = QrcpLanes<T, NP>::G, WAVES = QrcpLanes<T, NP>::WAVES;
  __shared__ T Rs[WAVES][G][NP][NP + 1];   // Rs[.][.][c][i] = R[i, c]
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int g = lane / NP, c = lane % NP;
  const int prob = ((int)blockIdx.x * WAVES + w) * G + g;
  const bool valid = prob < nd;
  QrcpDesc d{};
  if (valid) d = ds[prob];
  const int m = valid ? d.m : 0, n = valid ? d.n : 0;
  const bool col = c < n;
  T (*R)[NP + 1] = Rs[w][g];
  const T* Rg = static_cast<const T*>(d.R);
  auto gmax = [](T v) {
#pragma unroll
    for (int o = NP / 2; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, WAVE));
    return v;
  };
  auto gsum = [](T v) {
#pragma unroll
    for (int o = NP / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    return v;
  };
  T am = 0;
  if (col)
    for (int i = 0; i < m; ++i) am = fmax(am, fabs(Rg[i + (int64_t)c * d.ldr]));
  am = gmax(am);
  const int sh = am > (T)0 ? -ilogb((double)am) : 0;
  T s2 = 0;
  for (int i = 0; i < NP; ++i) {
    const T x = (col && i < m) ? ldexp(Rg[i + (int64_t)c * d.ldr], sh) : (T)0;
    R[c][i] = x;
    s2 += x * x;
  }
  T vn1 = col ? sqrt(s2) : (T)0, vn2 = vn1;
  int pos = c;                  // place of this column in the pivoted order
  bool done = !col;             // chosen as a pivot (or no column)
  const T dl = (T)ldexp(delta, sh);
  const T tol3z = sqrt((T)Prec<T>::u);
  const int kfull = min(m, n);
  int k = 0;
  bool stopped = false;
  T stop = 0;
  int kw = kfull;   // steps of the wavefront: the largest of its problems
#pragma unroll
  for (int o = NP; o < WAVE; o <<= 1) kw = max(kw, __shfl_xor(kw, o, WAVE));
  bool act = valid;   // this problem still factors
  for (int s = 0; s < kw; ++s) {
    act = act && s < kfull && !stopped;
    // pivot: the largest remaining partial norm, first place on ties; remaining Frobenius norm
    T best = (!done && act) ? vn1 : (T)-1;
    int bp = (!done && act) ? pos : NP;
    T ss = (!done && act) ? vn1 * vn1 : (T)0;
#pragma unroll
    for (int o = NP / 2; o > 0; o >>= 1) {
      const T ob = __shfl_xor(best, o, WAVE);
      const int op = __shfl_xor(bp, o, WAVE);
      if (ob > best || (ob == best && op < bp)) { best = ob; bp = op; }
      ss += __shfl_xor(ss, o, WAVE);
    }
    if (s == 0) stop = fmax(dl, (T)4 * (T)Prec<T>::u * sqrt(ss));
    if (act && sqrt(ss) <= stop) { stopped = true; act = false; }
    // the pivot column: the lane whose place is bp; it moves to place s, the column at place s to bp
    const bool piv = act && !done && pos == bp;
    int pl = piv ? c : -1;
#pragma unroll
    for (int o = NP / 2; o > 0; o >>= 1) pl = max(pl, __shfl_xor(pl, o, WAVE));
    if (act && !done && pos == s) pos = bp;
    if (piv) { pos = s; done = true; }
    // reflector of column pl, rows s..m-1; lane i reads row i
    T x0 = 0, x2 = 0;
    if (act) {
      x0 = R[pl][s];
      const T xi = (c > s && c < m) ? R[pl][c] : (T)0;
      x2 = xi * xi;
    }
    x2 = gsum(x2);
    T tau = 0, beta = x0, scale = 0;
    if (x2 > (T)0) {
      beta = x0 >= (T)0 ? -sqrt(x0 * x0 + x2) : sqrt(x0 * x0 + x2);
      tau = (beta - x0) / beta;
      scale = (T)1 / (x0 - beta);
    }
    if (act && !done) {   // a trailing column: apply, then downdate or recompute the partial norm
      T wv = R[c][s];
      for (int i = s + 1; i < m; ++i) wv += R[pl][i] * scale * R[c][i];
      wv *= tau;
      T rest = 0;
      const T rs = R[c][s] - wv;
      R[c][s] = rs;
      for (int i = s + 1; i < m; ++i) {
        const T x = R[c][i] - wv * (R[pl][i] * scale);
        R[c][i] = x;
        rest += x * x;
      }
      if (vn1 != (T)0) {
        const T r = fabs(rs) / vn1;
        const T t = fmax((T)0, ((T)1 + r) * ((T)1 - r));
        const T q = vn1 / vn2;
        if (t * q * q <= tol3z) { vn1 = sqrt(rest); vn2 = vn1; }
        else vn1 *= sqrt(t);
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (act && c == pl) {   // the pivot column itself: beta on the diagonal, zeros below
      R[c][s] = beta;
      for (int i = s + 1; i < m; ++i) R[c][i] = (T)0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (act) k = s + 1;
  }
  if (!valid || !col) return;
  // Y = R'[0:k, :]^T: the column at place p gives row p of Y
  T* __restrict__ Y = static_cast<T*>(d.Y);
  for (int r = 0; r < k; ++r) Y[pos + (int64_t)r * d.ldy] = pos >= r ? ldexp(R[c][r], -sh) : (T)0;
  d.perm[pos] = c;
  if (c == 0) {
    *d.kout = k;
    if (!stopped && k == SVD_MAXK && kfull > SVD_MAXK && d.over) *d.over = 1;
  }
}

template <class T>
__global__ void __launch_bounds__(SVD_WG) k_qrcp(const QrcpDesc* __restrict__ ds, double delta) {
  extern __shared__ unsigned char qrcp_dyn[];
  const QrcpDesc d0 = ds[blockIdx.x];
  T* vn1 = reinterpret_cast<T*>(qrcp_dyn);
  T* vn2 = vn1 + d0.n;
  int* pv = reinterpret_cast<int*>(vn2 + d0.n);
  T* hv = reinterpret_cast<T*>(qrcp_dyn + ((sizeof(T) * 2 + sizeof(int)) * (size_t)d0.n + 15) / 16 * 16);
  __shared__ T redv[SVD_WG / WAVE], reds[SVD_WG / WAVE];
  __shared__ int redi[SVD_WG / WAVE];
  __shared__ T sh_tau, sh_stop;
  __shared__ int sh_piv;
  const QrcpDesc d = ds[blockIdx.x];
  T* __restrict__ R = static_cast<T*>(d.R);
  const int m = d.m, n = d.n;
  const int64_t ld = d.ldr;
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = SVD_WG / WAVE;
  // exact power-of-two scaling of R so that squares of small entries do not underflow
  T am = 0;
  for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += SVD_WG) am = fmax(am, fabs(R[e % m + (e / m) * ld]));
  am = block_max(am, redv);
  const int sh = am > (T)0 ? -ilogb((double)am) : 0;
  for (int c = wv; c < n; c += nw) {
    T s = 0;
    for (int i = lane; i < m; i += WAVE) {
      const T x = ldexp(R[i + c * ld], sh);
      R[i + c * ld] = x;
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) { vn1[c] = vn2[c] = sqrt(s); pv[c] = c; }
  }
  __syncthreads();
  delta = ldexp(delta, sh);
  const T tol3z = sqrt((T)Prec<T>::u);
  const int kfull = min(m, n), kmax = min(kfull, SVD_MAXK);
  int k = 0;
  bool stopped = false;
  for (int s = 0; s < kmax; ++s) {
    // pivot = the largest remaining partial norm (first on ties); remaining Frobenius norm
    T best = (T)-1, ss = 0;
    int bi = s;
    for (int j = s + threadIdx.x; j < n; j += SVD_WG) {
      const T x = vn1[j];
      ss += x * x;
      if (x > best) { best = x; bi = j; }
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
      const T ob = __shfl_xor(best, o, WAVE);
      const int oi = __shfl_xor(bi, o, WAVE);
      if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      ss += __shfl_xor(ss, o, WAVE);
    }
    if (lane == 0) { redv[wv] = best; redi[wv] = bi; reds[wv] = ss; }
    __syncthreads();
    if (threadIdx.x == 0) {
      T b = redv[0], t = reds[0];
      int i0 = redi[0];
      for (int w = 1; w < nw; ++w) {
        if (redv[w] > b || (redv[w] == b && redi[w] < i0)) { b = redv[w]; i0 = redi[w]; }
        t += reds[w];
      }
      if (s == 0) sh_stop = fmax((T)delta, (T)4 * (T)Prec<T>::u * sqrt(t));
      sh_piv = sqrt(t) <= sh_stop ? -1 : i0;
    }
    __syncthreads();
    const int piv = sh_piv;
    if (piv < 0) { stopped = true; break; }
    if (piv != s) {
      for (int i = threadIdx.x; i < m; i += SVD_WG) {
        const T a = R[i + (int64_t)s * ld];
        R[i + (int64_t)s * ld] = R[i + (int64_t)piv * ld];
        R[i + (int64_t)piv * ld] = a;
      }
      if (threadIdx.x == 0) {
        T t = vn1[s]; vn1[s] = vn1[piv]; vn1[piv] = t;
        t = vn2[s]; vn2[s] = vn2[piv]; vn2[piv] = t;
        const int q = pv[s]; pv[s] = pv[piv]; pv[piv] = q;
      }
    }
    __syncthreads();
    // Householder reflector H = I - tau v v^T with v_s = 1 zeroing R[s+1:, s]
    // x0 is read before the reduction's barriers: thread 0 overwrites R[s, s] after them
    const T x0 = R[s + (int64_t)s * ld];
    T x2 = 0;
    for (int i = s + 1 + threadIdx.x; i < m; i += SVD_WG) { const T x = R[i + (int64_t)s * ld]; x2 += x * x; }
    x2 = block_sum(x2, redv);
    T tau = 0, beta = x0, scale = 0;
    if (x2 > (T)0) {
      beta = x0 >= (T)0 ? -sqrt(x0 * x0 + x2) : sqrt(x0 * x0 + x2);
      tau = (beta - x0) / beta;
      scale = (T)1 / (x0 - beta);
    }
    for (int i = s + threadIdx.x; i < m; i += SVD_WG) {
      hv[i] = i == s ? (T)1 : R[i + (int64_t)s * ld] * scale;
      R[i + (int64_t)s * ld] = i == s ? beta : (T)0;
    }
    if (threadIdx.x == 0) sh_tau = tau;
    __syncthreads();
    tau = sh_tau;
    // apply to the trailing columns, four per wavefront at a time (their
    // reductions overlap), and downdate their partial norms; lane 0 holds row
    // s, and the rest of a column is reduced only when its norm is recomputed
    for (int jc = s + 1 + wv * 4; jc < n; jc += nw * 4) {
      T w[4] = {0, 0, 0, 0};
      for (int i = s + lane; i < m; i += WAVE) {
        const T h = hv[i];
#pragma unroll
        for (int g = 0; g < 4; ++g)
          if (jc + g < n) w[g] += h * R[i + (int64_t)(jc + g) * ld];
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) w[g] = wave_sum(w[g]) * tau;
      T rs[4] = {0, 0, 0, 0}, rest[4] = {0, 0, 0, 0};
      for (int i = s + lane; i < m; i += WAVE) {
        const T h = hv[i];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          if (jc + g < n) {
            const T x = R[i + (int64_t)(jc + g) * ld] - w[g] * h;
            R[i + (int64_t)(jc + g) * ld] = x;
            if (i == s) rs[g] = x;
            else rest[g] += x * x;
          }
        }
      }
#pragma unroll
      for (int g = 0; g < 4; ++g) {
        const int j = jc + g;
        if (j < n) {
          int need = 0;   // 1: recompute the partial norm, 2: downdate it by t
          T t = 0;
          if (lane == 0 && vn1[j] != (T)0) {
            const T r = fabs(rs[g]) / vn1[j];
            t = fmax((T)0, ((T)1 + r) * ((T)1 - r));
            const T q = vn1[j] / vn2[j];
            need = t * q * q <= tol3z ? 1 : 2;
          }
          need = __shfl(need, 0, WAVE);
          if (need == 1) {
            const T tot = wave_sum(rest[g]);
            if (lane == 0) { vn1[j] = sqrt(tot); vn2[j] = vn1[j]; }
          } else if (need == 2 && lane == 0) {
            vn1[j] *= sqrt(t);
          }
        }
      }
    }
    __syncthreads();
    k = s + 1;
  }
  // Y = R'[0:k, :]^T, upper trapezoidal rows become lower trapezoidal columns
  T* __restrict__ Y = static_cast<T*>(d.Y);
  for (int64_t e = threadIdx.x; e < (int64_t)n * k; e += SVD_WG) {
    const int i = (int)(e % n), c = (int)(e / n);
    Y[i + (int64_t)c * d.ldy] = i >= c ? ldexp(R[c + (int64_t)i * ld], -sh) : (T)0;
  }
  for (int i = threadIdx.x; i < n; i += SVD_WG) d.perm[i] = pv[i];
  if (threadIdx.x == 0) *d.kout = k;
  if (threadIdx.x == 0 && !stopped && k == SVD_MAXK && kmax < kfull && d.over) *d.over = 1;
}

// Sum of 16 per-lane values over the 64 lanes of a wavefront, reduce-scattered
// (each exchange halves the values a lane keeps): on return lanes 4c..4c+3
// hold the sum of value c.
template <class T>
__device__ inline T wave_sum16_scatter(const T (&v)[16], int lane) {
  T a[8];
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const T keep = hi ? v[k + 8] : v[k], send = hi ? v[k] : v[k + 8];
      a[k] = keep + __shfl_xor(send, 32, WAVE);
    }
  }
  T c[4];
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T keep = hi ? a[k + 4] : a[k], send = hi ? a[k] : a[k + 4];
      c[k] = keep + __shfl_xor(send, 16, WAVE);
    }
  }
  T e[2];
  {
    const bool hi = lane & 8;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const T keep = hi ? c[k + 2] : c[k], send = hi ? c[k] : c[k + 2];
      e[k] = keep + __shfl_xor(send, 8, WAVE);
    }
  }
  const bool hi = lane & 4;
  T f = (hi ? e[1] : e[0]) + __shfl_xor(hi ? e[0] : e[1], 4, WAVE);
  f += __shfl_xor(f, 2, WAVE);
  return f + __shfl_xor(f, 1, WAVE);
}

// ------------------------------------------------------------ step-wise QRCP
// The same factorization for launches with few problems, where one workgroup
// per problem would leave most of the chip idle: one launch per Householder
// step, each problem's columns split into blocks of QS_CB owned by one
// workgroup. Every workgroup of a problem derives the pivot and the reflector
// from the same data in the same order, so they agree bitwise and none waits
// for another inside a launch. Columns are not moved: the pivot of step s is
// recorded in pos[s] (for the output order), and the partial norms are kept
// twice, read from the copy of step parity s and written to the other one,
// where a pivoted column carries the norm -1 so that later steps skip it.
// Pivot ties go to the smallest column index; the columns left at the stop
// follow in increasing index.
constexpr int QS_CB = 16;    // columns per workgroup
constexpr int QS_WG = 256;   // threads per workgroup (four wavefronts, four columns each)

struct QrcpStepDesc {
  void* R;          // m x n, ld ldr, scaled in place
  void* Y;          // output as in QrcpDesc
  int* perm;
  int* kout;
  void* vn;         // 4 n: vn1, vn2 of parity 0, then of parity 1
  void* beta;       // min(m, n): R(s, pos[s])
  void* thr;        // stop level (set at step 0)
  int* pos;         // min(m, n): pivot column of step s
  int* st;          // st[0]: -1 running, else the number of steps taken; st[1]: scale exponent
  int m, n, ldr, ldy;
};

struct QsBlock {
  int prob, c0, c1, first;   // problem, owned columns [c0, c1), first block of its problem
};

// scale by the exact power of two that brings max |R| into [1, 2); column norms
template <class T>
__global__ void __launch_bounds__(SVD_WG) k_qrcp_init(const QrcpStepDesc* __restrict__ ds, int* nstopped) {
  __shared__ T red[SVD_WG / WAVE];
  const QrcpStepDesc d = ds[blockIdx.x];
  T* __restrict__ R = static_cast<T*>(d.R);
  T* __restrict__ vn = static_cast<T*>(d.vn);
  const int m = d.m, n = d.n;
  const int64_t ld = d.ldr;
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE, nw = SVD_WG / WAVE;
  if (blockIdx.x == 0 && threadIdx.x == 0) *nstopped = 0;
  T am = 0;
  for (int c = wv; c < n; c += nw)
    for (int i = lane; i < m; i += WAVE) am = fmax(am, fabs(R[i + c * ld]));
  am = block_max(am, red);
  const int sh = am > (T)0 ? -ilogb((double)am) : 0;
  for (int c = wv; c < n; c += nw) {
    T s = 0;
    for (int i = lane; i < m; i += WAVE) {
      const T x = ldexp(R[i + c * ld], sh);
      R[i + c * ld] = x;
      s += x * x;
    }
    s = wave_sum(s);
    if (lane == 0) vn[c] = vn[n + c] = sqrt(s);
  }
  if (threadIdx.x == 0) { d.st[0] = -1; d.st[1] = sh; }
}

template <class T>
__global__ void __launch_bounds__(QS_WG) k_qrcp_step(const QrcpStepDesc* __restrict__ ds,
                                                     const QsBlock* __restrict__ blocks, int s, double delta,
                                                     int* nstopped) {
  constexpr int NW = QS_WG / WAVE;
  __shared__ T hv[SVD_MAXN];
  __shared__ T redv[NW], reds[NW];
  __shared__ int redi[NW];
  __shared__ T part[NW][QS_CB];
  __shared__ T rsh[QS_CB];          // updated row s of the owned columns
  const QsBlock b = blocks[blockIdx.x];
  const QrcpStepDesc d = ds[b.prob];
  const int st0 = d.st[0];
  if (st0 >= 0 && st0 <= s) return;   // stopped (the last step records k = s + 1 while others still update)
  const int m = d.m, n = d.n, kmax = min(m, n);
  if (s >= kmax) return;
  T* __restrict__ R = static_cast<T*>(d.R);
  const int64_t ld = d.ldr;
  const int tid = threadIdx.x, lane = tid % WAVE, wv = tid / WAVE;
  const T* vn1 = static_cast<const T*>(d.vn) + (s & 1) * 2 * n;
  const T* vn2 = vn1 + n;
  T* wn1 = static_cast<T*>(d.vn) + ((s + 1) & 1) * 2 * n;
  T* wn2 = wn1 + n;
  // pivot = the largest remaining partial norm (smallest index on ties); remaining Frobenius norm.
  // Columns pivoted at earlier steps carry the partial norm -1.
  T best = (T)-1, ss = 0;
  int bi = n;
  for (int c = tid; c < n; c += QS_WG) {
    const T x = vn1[c];
    if (x < (T)0) continue;
    ss += x * x;
    if (x > best) { best = x; bi = c; }
  }
  for (int o = WAVE / 2; o > 0; o >>= 1) {
    const T ob = __shfl_xor(best, o, WAVE);
    const int oi = __shfl_xor(bi, o, WAVE);
    if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
    ss += __shfl_xor(ss, o, WAVE);
  }
  if (lane == 0) { redv[wv] = best; redi[wv] = bi; reds[wv] = ss; }
  __syncthreads();
  T tot = reds[0];
  int piv = redi[0];
  best = redv[0];
  for (int w = 1; w < NW; ++w) {
    if (redv[w] > best || (redv[w] == best && redi[w] < piv)) { best = redv[w]; piv = redi[w]; }
    tot += reds[w];
  }
  const int sh = d.st[1];
  T* thrp = static_cast<T*>(d.thr);
  const T thr = s == 0 ? fmax((T)ldexp(delta, sh), (T)4 * (T)Prec<T>::u * sqrt(tot)) : *thrp;
  if (s == 0 && b.first && tid == 0) *thrp = thr;
  if (sqrt(tot) <= thr || piv >= n) {
    if (b.first && tid == 0) { d.st[0] = s; atomicAdd(nstopped, 1); }
    return;
  }
  // reflector H = I - tau v v^T with v_s = 1 zeroing the pivot column below row s
  const T* Rp = R + (int64_t)piv * ld;
  const T x0 = Rp[s];
  T x2 = 0;
  for (int i = s + 1 + tid; i < m; i += QS_WG) { const T x = Rp[i]; x2 += x * x; }
  x2 = block_sum(x2, redv);
  T tau = 0, beta = x0, scale = 0;
  if (x2 > (T)0) {
    beta = x0 >= (T)0 ? -sqrt(x0 * x0 + x2) : sqrt(x0 * x0 + x2);
    tau = (beta - x0) / beta;
    scale = (T)1 / (x0 - beta);
  }
  for (int i = s + tid; i < m; i += QS_WG) hv[i] = i == s ? (T)1 : Rp[i] * scale;
  if (b.first && tid == 0) {
    d.pos[s] = piv;
    static_cast<T*>(d.beta)[s] = beta;
    if (s + 1 == kmax) { d.st[0] = kmax; atomicAdd(nstopped, 1); }
  }
  __syncthreads();
  // the owned block: rows s.. held in registers, row s + tid + r QS_WG in slot r
  // (past the last row the slot repeats row m - 1 with a zero reflector entry)
  constexpr int RPT = SVD_MAXN / QS_WG;
  const int c0 = b.c0, nc = b.c1 - b.c0, nr = (m - s + QS_WG - 1) / QS_WG;
  T x[RPT][QS_CB], hr[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    hr[r] = 0;
    if (r < nr) {
      const int i = s + tid + r * QS_WG;
      const int ii = i < m ? i : m - 1;
      hr[r] = i < m ? hv[i] : (T)0;
#pragma unroll
      for (int g = 0; g < QS_CB; ++g) x[r][g] = R[ii + (int64_t)(c0 + (g < nc ? g : 0)) * ld];
    }
  }
  // w = tau v^T (block), reduced over the workgroup
  T acc[QS_CB];
#pragma unroll
  for (int g = 0; g < QS_CB; ++g) {
    acc[g] = 0;
#pragma unroll
    for (int r = 0; r < RPT; ++r)
      if (r < nr) acc[g] += hr[r] * x[r][g];
  }
  T wsum = wave_sum16_scatter(acc, lane);
  if ((lane & 3) == 0) part[wv][lane >> 2] = wsum;
  __syncthreads();
  T w[QS_CB];
#pragma unroll
  for (int g = 0; g < QS_CB; ++g) {
    T t = 0;
    for (int q = 0; q < NW; ++q) t += part[q][g];
    w[g] = t * tau;
  }
  // rank-one update of the live columns; new row s and squares below it
  T rest[QS_CB];
#pragma unroll
  for (int g = 0; g < QS_CB; ++g) rest[g] = 0;
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (r < nr) {
      const int i = s + tid + r * QS_WG;
      if (i < m) {
#pragma unroll
        for (int g = 0; g < QS_CB; ++g) {
          const int j = c0 + g;
          if (g < nc && vn1[j] >= (T)0 && j != piv) {
            const T y = x[r][g] - w[g] * hr[r];
            R[i + (int64_t)j * ld] = y;
            if (i == s) rsh[g] = y;
            else rest[g] += y * y;
          }
        }
      }
    }
  }
  wsum = wave_sum16_scatter(rest, lane);
  __syncthreads();   // every wavefront has read part[] for w
  if ((lane & 3) == 0) part[wv][lane >> 2] = wsum;
  __syncthreads();
  // downdate (or recompute) the partial norms into the other parity
  if (tid < nc) {
    const int j = c0 + tid;
    if (vn1[j] < (T)0 || j == piv) {   // pivoted: marked for the next steps
      wn1[j] = (T)-1;
      wn2[j] = (T)-1;
    } else {
      const T a1 = vn1[j], a2 = vn2[j];
      T n1 = a1, n2 = a2;
      if (a1 != (T)0) {
        const T r = fabs(rsh[tid]) / a1;
        const T t = fmax((T)0, ((T)1 + r) * ((T)1 - r));
        const T q = a1 / a2;
        if (t * q * q <= sqrt((T)Prec<T>::u)) {
          T tot2 = 0;
          for (int q2 = 0; q2 < NW; ++q2) tot2 += part[q2][tid];
          n1 = n2 = sqrt(tot2);
        } else {
          n1 = a1 * sqrt(t);
        }
      }
      wn1[j] = n1;
      wn2[j] = n2;
    }
  }
}

// Y = R'[0:k, :]^T in pivot order, then the remaining columns by index; perm; k
template <class T>
__global__ void __launch_bounds__(SVD_WG) k_qrcp_finish(const QrcpStepDesc* __restrict__ ds) {
  __shared__ int order[SVD_MAXN];
  __shared__ unsigned char done[SVD_MAXN];
  const QrcpStepDesc d = ds[blockIdx.x];
  const T* __restrict__ R = static_cast<const T*>(d.R);
  const T* __restrict__ beta = static_cast<const T*>(d.beta);
  T* __restrict__ Y = static_cast<T*>(d.Y);
  const int m = d.m, n = d.n, kmax = min(m, n);
  const int64_t ld = d.ldr;
  const int k = d.st[0] >= 0 ? d.st[0] : kmax;
  const int sh = d.st[1];
  for (int c = threadIdx.x; c < n; c += SVD_WG) done[c] = 0;
  __syncthreads();
  for (int j = threadIdx.x; j < k; j += SVD_WG) { done[d.pos[j]] = 1; order[j] = d.pos[j]; }
  __syncthreads();
  if (threadIdx.x == 0) {
    int q = k;
    for (int c = 0; c < n; ++c)
      if (!done[c]) order[q++] = c;
    *d.kout = k;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < n; i += SVD_WG) d.perm[i] = order[i];
  for (int64_t e = threadIdx.x; e < (int64_t)n * k; e += SVD_WG) {
    const int i = (int)(e % n), c = (int)(e / n);
    T v = 0;
    if (i == c) v = beta[c];
    else if (i > c) v = R[c + (int64_t)order[i] * ld];
    Y[i + (int64_t)c * d.ldy] = ldexp(v, -sh);
  }
}

// Step-wise path: init, one launch per step (the host reads the count of
// stopped problems every QS_POLL steps), finish.
constexpr int QS_POLL = 16;

template <class T>
inline void run_qrcp_steps(Problem& P, const std::vector<QrcpDesc>& v, DevBuf& scratch, DevBuf& work,
                           double delta) {
  const int np = (int)v.size();
  std::vector<int64_t> toff(np), ioff(np);
  int64_t tt = 0, ti = 0;
  int kall = 0;
  for (int p = 0; p < np; ++p) {
    const int km = std::min(v[p].m, v[p].n);
    toff[p] = tt;
    tt += 4 * (int64_t)v[p].n + km + 1;
    ioff[p] = ti;
    ti += km + 2;
    kall = std::max(kall, km);
  }
  const size_t bytes = (size_t)tt * sizeof(T) + (size_t)(ti + 1) * sizeof(int) + 256;
  if (bytes > work.bytes) {
    P.sync();
    work.alloc(bytes + bytes / 4, &P.mem);
  }
  T* tw = work.template as<T>();
  int* iw = reinterpret_cast<int*>(tw + tt);
  int* nst = iw + ti;
  std::vector<QrcpStepDesc> dv(np);
  std::vector<QsBlock> bl;
  for (int p = 0; p < np; ++p) {
    const auto& q = v[p];
    const int km = std::min(q.m, q.n);
    T* t0 = tw + toff[p];
    dv[p] = {q.R, q.Y, q.perm, q.kout, t0, t0 + 4 * (int64_t)q.n, t0 + 4 * (int64_t)q.n + km,
             iw + ioff[p], iw + ioff[p] + km, q.m, q.n, q.ldr, q.ldy};
    for (int c0 = 0; c0 < q.n; c0 += QS_CB) bl.push_back({p, c0, std::min(q.n, c0 + QS_CB), c0 == 0 ? 1 : 0});
  }
  const QrcpStepDesc* dd = P.put(scratch, dv);
  const QsBlock* db = P.put(scratch, bl);
  P.kone_begin(KF_QRCP_STEP, 0);
  hipLaunchKernelGGL(k_qrcp_init<T>, dim3((unsigned)np), dim3(SVD_WG), 0, P.stream, dd, nst);
  IFMM_LAUNCH_CHECK();
  P.kone_end();
  for (int s = 0; s < kall; ++s) {
    double fl = 0;   // Householder step: products with the trailing block and its rank-one update
    for (const auto& q : v)
      if (s < std::min(q.m, q.n)) fl += 4.0 * (q.m - s) * (double)(q.n - s);
    P.kone_begin(KF_QRCP_STEP, fl);
    hipLaunchKernelGGL(k_qrcp_step<T>, dim3((unsigned)bl.size()), dim3(QS_WG), 0, P.stream, dd, db, s, delta, nst);
    IFMM_LAUNCH_CHECK();
    P.kone_end();
    if ((s + 1) % QS_POLL == 0 && s + 1 < kall) {
      std::vector<int> h;
      P.download(h, nst, 1);
      if (h[0] >= np) break;
    }
  }
  P.kone_begin(KF_QRCP_STEP, 0);
  hipLaunchKernelGGL(k_qrcp_finish<T>, dim3((unsigned)np), dim3(SVD_WG), 0, P.stream, dd);
  IFMM_LAUNCH_CHECK();
  P.kone_end();
}

// Launches whose problems would fill less than half of the compute units
// take the step-wise path.
template <class T>
inline void run_qrcp(Problem& P, const std::vector<QrcpDesc>& v, DevBuf& scratch, DevBuf& work, double delta) {
  if (v.empty()) return;
  int64_t nblk = 0;
  bool large = false;   // a problem beyond the step-wise kernel's LDS arrays: one workgroup per problem
  size_t lds = 0;
  for (const auto& q : v) {
    if (q.m > q.n) fail(IFMM_ERR_INTERNAL, "QRCP shape out of range");
    nblk += ceil_div(q.n, QS_CB);
    large = large || q.n > SVD_MAXN || q.m > SVD_MAXN;
    lds = std::max(lds, qrcp_lds<T>(q.m, q.n));
  }
  if (lds > QRCP_LDS_MAX) fail(IFMM_ERR_ARG, "a recompressed box is too large for the pivoted QR (x~ size)");
  if (qr_stats_on()) {
    int64_t sm = 0, sn = 0;
    int mm = 0, mn = 0, h[5] = {0, 0, 0, 0, 0};
    for (const auto& q : v) {
      sm += q.m; sn += q.n; mm = std::max(mm, q.m); mn = std::max(mn, q.n);
      ++h[q.n <= 16 ? 0 : q.n <= 32 ? 1 : q.n <= 64 ? 2 : q.n <= 128 ? 3 : 4];
    }
    std::fprintf(stderr, "[ifmm-qr] qrcp n=%zu sumM=%lld sumN=%lld maxM=%d maxN=%d le16=%d le32=%d le64=%d le128=%d gt=%d\n",
                 v.size(), (long long)sm, (long long)sn, mm, mn, h[0], h[1], h[2], h[3], h[4]);
  }
  // problems of at most 64 columns: a lane per column
  std::vector<QrcpDesc> lanes[3], rest;
  for (const auto& q : v) {
    if (q.n <= 64 && !force_streamed()) lanes[q.n <= 16 ? 0 : q.n <= 32 ? 1 : 2].push_back(q);
    else rest.push_back(q);
  }
  if (rest.size() < v.size()) {
    double fl = 0;
    for (const auto& lv : lanes)
      for (const auto& q : lv) fl += 2.0 * q.n * (double)q.m * q.m - 2.0 / 3.0 * (double)q.m * q.m * q.m;
    P.kone_begin(KF_QRCP, fl);
    auto go = [&](auto np_tag, const std::vector<QrcpDesc>& lv) {
      constexpr int NP = decltype(np_tag)::value;
      if (lv.empty()) return;
      const QrcpDesc* dl = P.put(scratch, lv);
      constexpr int per = QrcpLanes<T, NP>::G * QrcpLanes<T, NP>::WAVES;
      hipLaunchKernelGGL((k_qrcp_lanes<T, NP>), dim3((unsigned)ceil_div((int64_t)lv.size(), per)),
                         dim3(QrcpLanes<T, NP>::WAVES * WAVE), 0, P.stream, dl, (int)lv.size(), delta);
      IFMM_LAUNCH_CHECK();
    };
    go(std::integral_constant<int, 16>(), lanes[0]);
    go(std::integral_constant<int, 32>(), lanes[1]);
    go(std::integral_constant<int, 64>(), lanes[2]);
    P.kone_end();
    if (rest.empty()) return;
    run_qrcp<T>(P, rest, scratch, work, delta);
    return;
  }
  if (!large && !force_streamed() && v.size() < 128 && nblk <= 2048) {
    run_qrcp_steps<T>(P, v, scratch, work, delta);
    return;
  }
  static const bool attr = [] {
    IFMM_HIP(hipFuncSetAttribute((const void*)k_qrcp<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)QRCP_LDS_MAX));
    return true;
  }();
  (void)attr;
  const QrcpDesc* d = P.put(scratch, v);
  // Householder QR flops of the untruncated factorization (m <= n): 2 n m^2 - 2/3 m^3
  double fl = 0;
  for (const auto& q : v) fl += 2.0 * q.n * (double)q.m * q.m - 2.0 / 3.0 * (double)q.m * q.m * q.m;
  P.kone_begin(KF_QRCP, fl);
  hipLaunchKernelGGL(k_qrcp<T>, dim3((unsigned)v.size()), dim3(SVD_WG), lds, P.stream, d, delta);
  IFMM_LAUNCH_CHECK();
  P.kone_end();
}

// live[t] = the live column count of problem t (what the pivoted QR kept).
__global__ void k_svd_live(const SvdDesc* __restrict__ ds, int n, int* __restrict__ live) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) live[t] = svd_cols(ds[t]);
}

// ------------------------------------------------------------------ launcher
// defl: singular directions below this absolute level are not resolved (they
// fall far under the truncation threshold and are discarded).
template <class T>
inline void run_svd(Problem& P, const std::vector<SvdDesc>& v_in, DevBuf& scratch, double defl = 0.0) {
  if (v_in.empty()) return;
  // Problems whose allocated width would send them to the block scheme: read
  // the live column counts first (one synchronisation), so that a problem
  // whose pivoted QR kept few columns takes the LDS scheme and the block
  // scheme plans its rounds for the live columns only.
  std::vector<SvdDesc> v = v_in;
  std::vector<int> livecount(v.size(), -1);
  {
    bool any = false;
    for (const auto& s : v) any = any || (s.nlive && (size_t)s.M * s.N * sizeof(T) > SVD_LDS_MAX);
    if (any) {
      const SvdDesc* d0 = P.put(scratch, v);
      DevBuf lv;
      lv.alloc(sizeof(int) * v.size(), &P.mem);
      hipLaunchKernelGGL(k_svd_live, dim3((unsigned)ceil_div((int64_t)v.size(), 256)), dim3(256), 0, P.stream, d0,
                         (int)v.size(), lv.as<int>());
      IFMM_LAUNCH_CHECK();
      P.download(livecount, lv.p, v.size());
    }
  }
  if (v.empty()) return;
  if (qr_stats_on()) {   // shapes of the batch: count, sum and max of M and N, histogram of max(M, N)
    int64_t sm = 0, sn = 0;
    int mm = 0, mn = 0, h[5] = {0, 0, 0, 0, 0};
    for (size_t t = 0; t < v.size(); ++t) {
      const int nc = livecount[t] >= 0 ? livecount[t] : v[t].N;
      sm += v[t].M; sn += nc; mm = std::max(mm, v[t].M); mn = std::max(mn, nc);
      const int x = std::max(v[t].M, nc);
      ++h[x <= 16 ? 0 : x <= 32 ? 1 : x <= 64 ? 2 : x <= 128 ? 3 : 4];
    }
    std::fprintf(stderr, "[ifmm-qr] svd n=%zu sumM=%lld sumN=%lld maxM=%d maxN=%d le16=%d le32=%d le64=%d le128=%d gt=%d\n",
                 v.size(), (long long)sm, (long long)sn, mm, mn, h[0], h[1], h[2], h[3], h[4]);
  }
  static const bool attr = [] {   // once per process (thread-safe initialisation)
    IFMM_HIP(hipFuncSetAttribute((const void*)k_svd_small<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)SVD_LDS_MAX));
    IFMM_HIP(hipFuncSetAttribute((const void*)k_svd_round<T>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)SVD_LDS_MAX));
    return true;
  }();
  (void)attr;
  std::vector<SvdDesc> small, big, lanes[3];   // lane scheme: NP = 16, 32, 64
  std::vector<int> bigN;   // columns the block scheme plans for (live when known)
  size_t lds = 0;
  int bigM = 0, bigBlocks = 0;
  for (size_t t = 0; t < v.size(); ++t) {
    const auto& s = v[t];
    if (s.N > SVD_MAXN && !s.nlive) fail(IFMM_ERR_INTERNAL, "SVD wider than SVD_MAXN");
    const int ncols = livecount[t] >= 0 ? livecount[t] : s.N;
    const size_t b = (size_t)s.M * ncols * sizeof(T);
    const int mx = std::max(s.M, s.N);
    if (mx <= 64 && !force_streamed()) lanes[mx <= 16 ? 0 : mx <= 32 ? 1 : 2].push_back(s);
    else if (b <= SVD_LDS_MAX && !force_streamed()) { small.push_back(s); lds = std::max(lds, b); }
    else { big.push_back(s); bigN.push_back(ncols); bigM = std::max(bigM, s.M); }
  }
  // column block width of the block scheme: two blocks of M_max rows in LDS
  int nb = 16;
  while (nb > 2 && (size_t)bigM * 2 * nb * sizeof(T) > SVD_LDS_MAX) nb /= 2;
  for (int nc : bigN) bigBlocks = std::max(bigBlocks, (nc + nb - 1) / nb);
  const double u = Prec<T>::u;
  const int max_sweeps = 60;
  // algorithmic flops of an SVD with left vectors (LAWN 41 style): 4 M N^2 + 8 N^3
  double fl_small = 0, fl_big = 0, fl_lanes = 0;
  for (const auto& lv : lanes)
    for (const auto& s : lv) fl_lanes += 4.0 * s.M * (double)s.N * s.N + 8.0 * (double)s.N * s.N * s.N;
  if (fl_lanes > 0) {
    P.kone_begin(KF_SVD_SMALL, fl_lanes);
    auto go = [&](auto np_tag, const std::vector<SvdDesc>& lv) {
      constexpr int NP = decltype(np_tag)::value;
      if (lv.empty()) return;
      const SvdDesc* dl = P.put(scratch, lv);
      constexpr int per = SvdLanes<T, NP>::PPW * SvdLanes<T, NP>::WAVES;
      hipLaunchKernelGGL((k_svd_lanes<T, NP>), dim3((unsigned)ceil_div((int64_t)lv.size(), per)),
                         dim3(SvdLanes<T, NP>::WAVES * WAVE), 0, P.stream, dl, (int)lv.size(), Prec<T>::u, max_sweeps,
                         defl);
      IFMM_LAUNCH_CHECK();
    };
    go(std::integral_constant<int, 16>(), lanes[0]);
    go(std::integral_constant<int, 32>(), lanes[1]);
    go(std::integral_constant<int, 64>(), lanes[2]);
    P.kone_end();
  }
  if (small.empty() && big.empty()) return;
  for (const auto& s : small) fl_small += 4.0 * s.M * (double)s.N * s.N + 8.0 * (double)s.N * s.N * s.N;
  for (const auto& s : big) fl_big += 4.0 * s.M * (double)s.N * s.N + 8.0 * (double)s.N * s.N * s.N;
  const size_t ns = small.size();
  small.insert(small.end(), big.begin(), big.end());
  const SvdDesc* d = P.put(scratch, small);
  const bool tr = trace_on();
  int* sw = nullptr;
  std::chrono::steady_clock::time_point t0;
  if (tr) {
    P.trace_buf.reserve(64, &P.mem);
    sw = P.trace_buf.as<int>();
    IFMM_HIP(hipMemsetAsync(sw, 0, sizeof(int), P.stream));
    P.sync();
    t0 = std::chrono::steady_clock::now();
  }
  if (ns) {
    P.kone_begin(KF_SVD_SMALL, fl_small);
    hipLaunchKernelGGL(k_svd_small<T>, dim3((unsigned)ns), dim3(SVD_WG), lds, P.stream, d, u, max_sweeps, defl, 1,
                       sw);
    IFMM_LAUNCH_CHECK();
    P.kone_end();
  }
  P.kbegin();
  int outer = 0;
  int64_t nrounds = 0;
  if (!big.empty()) {
    const int nbig = (int)big.size();
    const SvdDesc* db = d + ns;
    const int nbm = bigBlocks + (bigBlocks & 1);
    P.svd_state.reserve(sizeof(int) * ((size_t)3 * nbig + (size_t)nbig * (nbm + nbm * nbm)) + 64, &P.mem);
    int* shs = P.svd_state.as<int>();
    int* flags = shs + nbig;
    int* bst = flags + 2 * nbig;
    hipLaunchKernelGGL(k_svd_prep<T>, dim3(nbig), dim3(SVD_WG), 0, P.stream, db, shs, flags, bst, nbm);
    IFMM_LAUNCH_CHECK();
    const int np = bigBlocks + (bigBlocks & 1);
    const size_t lds_b = (size_t)bigM * 2 * nb * sizeof(T);
    std::vector<int> hf;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
      P.kend();
      for (int r = 0; r < np - 1; ++r) {
        P.kone_begin(KF_SVD_ROUND, 0);
        hipLaunchKernelGGL(k_svd_round<T>, dim3((unsigned)(np / 2), (unsigned)nbig), dim3(SVD_WG), lds_b, P.stream,
                           db, (const int*)shs, flags, nb, r, u, defl, 1, bst, nbm, sweep * 4096 + r);
        IFMM_LAUNCH_CHECK();
        P.kone_end();
        ++nrounds;
      }
      P.kbegin();
      hipLaunchKernelGGL(k_svd_sweep_end, dim3((unsigned)ceil_div(nbig, 256)), dim3(256), 0, P.stream, flags, nbig,
                         sweep, sw);
      IFMM_LAUNCH_CHECK();
      outer = sweep + 1;
      if (sweep >= 3 && (sweep % 2 == 1)) {   // poll the converged flags now and then
        P.download(hf, flags, (size_t)2 * nbig);
        bool all = true;
        for (int s = 0; s < nbig; ++s) all = all && hf[2 * s + 1];
        if (all) break;
      }
    }
    hipLaunchKernelGGL(k_svd_block_finish<T>, dim3(nbig), dim3(SVD_WG), 0, P.stream, db, (const int*)shs);
    IFMM_LAUNCH_CHECK();
  }
  P.kend();
  // the block scheme's algorithmic flops, shared evenly by its round launches
  if (P.kt.on && nrounds > 0) P.kt.flops[KF_SVD_ROUND] += fl_big;
  if (tr) {
    P.sync();
    const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    std::vector<int> h;
    P.download(h, sw, 1);
    int mm = 0, mn = 0;
    double work = 0;
    for (const auto& s : v) { mm = std::max(mm, s.M); mn = std::max(mn, s.N); work += 3.0 * s.M * (double)s.N * s.N; }
    std::fprintf(stderr,
                 "[ifmm-trace] svd level=%d count=%zu small=%zu maxM=%d maxN=%d sweep_work=%.3e sweeps=%d outer=%d "
                 "nb=%d ms=%.3f\n",
                 P.trace_level, v.size(), ns, mm, mn, work, h[0], outer, nb, ms);
  }
}

}  // namespace ifmm
