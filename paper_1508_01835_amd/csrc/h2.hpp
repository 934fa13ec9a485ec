// R1: the Chebyshev H2 representation of A (Sec. 2.1, eqs. A_decomp_l3 and
// A_decomp_l2; Sec. 3 opening) and its product y = A~ x (the black-box FMM
// product that GMRES uses in Sec. 3.2).
//   leaf U_i = V_i : Lagrange basis of box i at its points      (m_i x q)
//   transfer T_b   : parent basis at the child's nodes           (q x q), b = child position
//   M2L Kbar(l, d) : kernel between the nodes of two boxes at offset d (q x q)
//   P2P            : kernel between the points of adjacent leaves, evaluated on the fly
// q = n^d, first-kind Chebyshev nodes cos((2k+1) pi / (2n)), k = 0..n-1,
// tensor index m = sum_k m_k n^k.
#pragma once

#include <cmath>

#include "linalg.hpp"
#include "tree.hpp"

namespace ifmm {

constexpr int MAXN = 8;          // Chebyshev order limit
constexpr int P2P_TILE = 256;    // source points staged in LDS at a time

struct KernelFn {
  int kind;
  double param, shift;
};

__host__ __device__ inline double kappa(const KernelFn& k, double r) {
  switch (k.kind) {
    case IFMM_K_IMQ: return 1.0 / sqrt(r * r + k.param * k.param);
    case IFMM_K_GAUSS: return exp(-(r * r) / (k.param * k.param));
    case IFMM_K_PAPER:
      if (r == 0.0) return 1.0;
      return r < k.param ? r / k.param : k.param / r;
    default: return 1.0 + r * r;
  }
}

struct ChebConst {
  int n, d, q;
  double t[MAXN];
};

__host__ __device__ inline double lagrange1(const ChebConst& c, int m, double x) {
  double v = 1.0;
  for (int k = 0; k < c.n; ++k)
    if (k != m) v *= (x - c.t[k]) / (c.t[m] - c.t[k]);
  return v;
}

__host__ __device__ inline double lagrange_nd(const ChebConst& c, int m, const double* x) {
  double v = 1.0;
  for (int k = 0; k < c.d; ++k) {
    const int mk = m % c.n;
    m /= c.n;
    v *= lagrange1(c, mk, x[k]);
  }
  return v;
}

__host__ __device__ inline void node_ref(const ChebConst& c, int m, double* x) {
  for (int k = 0; k < c.d; ++k) {
    x[k] = c.t[m % c.n];
    m /= c.n;
  }
}

// Leaf interpolation matrices, column-major per leaf at offset leaf_start[i] * q.
__global__ void k_leaf_ubar(const double* __restrict__ pts, const int64_t* __restrict__ leaf_start,
                            const int* __restrict__ coords, int nb, ChebConst c, double o0, double o1,
                            double o2, double h, double* __restrict__ ubar) {
  const int i = blockIdx.x;
  if (i >= nb) return;
  const int64_t s = leaf_start[i], m = leaf_start[i + 1] - s;
  const double o[3] = {o0, o1, o2};
  double ctr[3];
  for (int k = 0; k < c.d; ++k) ctr[k] = o[k] + ((double)coords[i * c.d + k] + 0.5) * h;
  double* U = ubar + s * c.q;
  for (int64_t e = threadIdx.x; e < m * c.q; e += WG) {
    const int64_t a = e % m;
    const int mm = (int)(e / m);
    double x[3];
    for (int k = 0; k < c.d; ++k) x[k] = (pts[(s + a) * c.d + k] - ctr[k]) * (2.0 / h);
    U[a + (int64_t)mm * m] = lagrange_nd(c, mm, x);
  }
}

// M2L table of one level: 7^d offsets, each q x q column-major.
__global__ void k_m2l_table(ChebConst c, KernelFn kf, double h, double* __restrict__ tab) {
  const int code = blockIdx.x;
  int dl[3] = {0, 0, 0};
  int r = code;
  for (int k = 0; k < c.d; ++k) { dl[k] = r % 7 - 3; r /= 7; }
  double* K = tab + (int64_t)code * c.q * c.q;
  for (int e = threadIdx.x; e < c.q * c.q; e += WG) {
    const int m = e % c.q, mp = e / c.q;
    double xi[3], xj[3];
    node_ref(c, m, xi);
    node_ref(c, mp, xj);
    double r2 = 0;
    for (int k = 0; k < c.d; ++k) {
      const double a = xi[k] * (0.5 * h);
      const double b = xj[k] * (0.5 * h) + (double)dl[k] * h;
      const double df = a - b;
      r2 += df * df;
    }
    K[m + (int64_t)mp * c.q] = kappa(kf, sqrt(r2));
  }
}

// ------------------------------------------------------------------ matvec
// Multipole/local arrays: per box a q x nrhs column-major block.
__global__ void k_p2m(const double* __restrict__ ubar, const int64_t* __restrict__ leaf_start, int nb,
                      int q, const double* __restrict__ x, int64_t ldx, int nrhs,
                      double* __restrict__ w) {
  const int i = blockIdx.x;
  if (i >= nb) return;
  const int64_t s = leaf_start[i], m = leaf_start[i + 1] - s;
  const double* U = ubar + s * q;
  for (int e = threadIdx.x; e < q * nrhs; e += WG) {
    const int mm = e % q, rr = e / q;
    double acc = 0;
    for (int64_t a = 0; a < m; ++a) acc += U[a + (int64_t)mm * m] * x[(s + a) + rr * ldx];
    w[(int64_t)i * q * nrhs + e] = acc;
  }
}

// Upward pass (M2M): w_p = sum_c T_c^T w_c; tcodes[c] = child position bits.
__global__ void k_m2m(const int* __restrict__ ch_start, const int* __restrict__ cbits, int nbp, int q,
                      int nrhs, const double* __restrict__ T, const double* __restrict__ wc,
                      double* __restrict__ wp) {
  const int p = blockIdx.x;
  if (p >= nbp) return;
  for (int e = threadIdx.x; e < q * nrhs; e += WG) {
    const int mp = e % q, rr = e / q;
    double acc = 0;
    for (int c = ch_start[p]; c < ch_start[p + 1]; ++c) {
      const double* Tc = T + (int64_t)cbits[c] * q * q;
      const double* w = wc + (int64_t)c * q * nrhs + (int64_t)rr * q;
      for (int m = 0; m < q; ++m) acc += Tc[m + (int64_t)mp * q] * w[m];
    }
    wp[(int64_t)p * q * nrhs + e] = acc;
  }
}

// Interaction lists (M2L): g_i = sum_{j in I(i)} Kbar(offset(i, j)) w_j.
__global__ void k_m2l(const int* __restrict__ in_start, const int* __restrict__ inter,
                      const int* __restrict__ coords, int nb, int d, int q, int nrhs,
                      const double* __restrict__ tab, const double* __restrict__ w,
                      double* __restrict__ g) {
  const int i = blockIdx.x;
  if (i >= nb) return;
  for (int e = threadIdx.x; e < q * nrhs; e += WG) {
    const int m = e % q, rr = e / q;
    double acc = 0;
    for (int t = in_start[i]; t < in_start[i + 1]; ++t) {
      const int j = inter[t];
      int code = 0, mul = 1;
      for (int k = 0; k < d; ++k) {
        code += (coords[j * d + k] - coords[i * d + k] + 3) * mul;
        mul *= 7;
      }
      const double* K = tab + (int64_t)code * q * q;
      const double* wj = w + (int64_t)j * q * nrhs + (int64_t)rr * q;
      for (int mp = 0; mp < q; ++mp) acc += K[m + (int64_t)mp * q] * wj[mp];
    }
    g[(int64_t)i * q * nrhs + e] = acc;
  }
}

// M2L on the FP64 matrix cores, for q <= 16 RB: per target box i,
// g_i (q x nrhs) = sum over I(i) of K_code (q x q) w_j (q x nrhs), i.e. one
// contraction of depth |I(i)| q. The four wavefronts of the workgroup take
// every fourth source of the list and accumulate 16 x 16 blocks with
// v_mfma_f64_16x16x4f64 (lane l supplies A[l % 16][l / 16] and B[l / 16][l % 16]
// of a 16 x 4 and a 4 x 16 slice; register r of lane l holds D[4 r + l / 16][l % 16]);
// entries past q or nrhs are supplied as zero. The four partial sums are added
// through LDS in a fixed order. Columns of the right-hand sides in blocks of 16.
template <int RB>
__global__ void __launch_bounds__(256) k_m2l_mfma(const int* __restrict__ in_start, const int* __restrict__ inter,
                                                  const int* __restrict__ coords, int nb, int d, int q, int nrhs,
                                                  const double* __restrict__ tab, const double* __restrict__ w,
                                                  double* __restrict__ g) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  __shared__ double red[4][RB * 256];
  const int i = blockIdx.x;
  if (i >= nb) return;
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int t0 = in_start[i], t1 = in_start[i + 1];
  int ci[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) ci[k] = coords[i * d + k];
  for (int cb = 0; cb < nrhs; cb += 16) {
    v4d acc[RB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) acc[rb] = v4d{0, 0, 0, 0};
    const int rr = cb + (lane & 15);
    const bool colok = rr < nrhs;
    for (int t = t0 + wv; t < t1; t += 4) {
      const int j = inter[t];
      int code = 0, mul = 1;
      for (int k = 0; k < d; ++k) {
        code += (coords[j * d + k] - ci[k] + 3) * mul;
        mul *= 7;
      }
      const double* K = tab + (int64_t)code * q * q;
      const double* wj = w + (int64_t)j * q * nrhs + (int64_t)rr * q;
      for (int k4 = 0; k4 < q; k4 += 4) {
        const int mp = k4 + (lane >> 4);
        const double b = (mp < q && colok) ? wj[mp] : 0.0;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
          const int m = rb * 16 + (lane & 15);
          const double a = (m < q && mp < q) ? K[m + (int64_t)mp * q] : 0.0;
          acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[rb], 0, 0, 0);
        }
      }
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int r = 0; r < 4; ++r) red[wv][rb * 256 + (4 * r + (lane >> 4)) * 16 + (lane & 15)] = acc[rb][r];
    __syncthreads();
    for (int e = threadIdx.x; e < RB * 256; e += 256) {
      const int rb = e / 256, row = (e % 256) / 16, col = e % 16;
      const int m = rb * 16 + row, c = cb + col;
      if (m < q && c < nrhs)
        g[(int64_t)i * q * nrhs + (int64_t)c * q + m] = ((red[0][e] + red[1][e]) + red[2][e]) + red[3][e];
    }
    __syncthreads();
  }
}

// M2L by offset tiles (orders with 32 < q <= 64): the targets of one child
// position share the same list of interaction offsets, so a workgroup takes
// up to T of them (T x nrhs <= 64 output columns) and walks that list once:
// per offset it stages the translation table K~_o (q x q) and the T source
// vectors in LDS and adds their product on the FP64 matrix cores. A table is
// then read once per workgroup instead of once per (target, source) pair.
// Every output column sums its offsets in list order, whatever T and nrhs.
struct M2LGroups {
  int start[9];   // group b = targets of child position b at tord[start[b] .. start[b + 1])
  int wg0[9];     // first workgroup of group b
};

constexpr int M2L_QP = 64;   // padded table order of k_m2l_tile

__global__ void __launch_bounds__(256) k_m2l_tile(const int* __restrict__ tord, const int* __restrict__ bo,
                                                  const int* __restrict__ inter, int nofs,
                                                  const int* __restrict__ ocode, M2LGroups gr, int ngroups, int T,
                                                  int q, int nrhs, const double* __restrict__ tab,
                                                  const double* __restrict__ w, double* __restrict__ g) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  __shared__ double As[M2L_QP][M2L_QP + 1];   // As[k][m] = K~_o[m, k]
  __shared__ double Bs[M2L_QP][M2L_QP + 1];   // Bs[k][col] = w_src(col)[k]
  __shared__ int src[M2L_QP];                 // source box of each output column for this offset
  int b = 0;
  while (b + 1 < ngroups && gr.wg0[b + 1] <= (int)blockIdx.x) ++b;
  const int t0 = gr.start[b] + ((int)blockIdx.x - gr.wg0[b]) * T;
  const int cnt = min(T, gr.start[b + 1] - t0);
  const int ncol = cnt * nrhs;
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int rb0 = 32 * (wv >> 1), cb0 = 32 * (wv & 1);
  v4d acc[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) acc[i] = v4d{0, 0, 0, 0};
  const int* codes = ocode + b * nofs;
  for (int k = 0; k < nofs; ++k) {
    __syncthreads();
    if (threadIdx.x < M2L_QP) {
      const int col = threadIdx.x;
      const int pr = col < ncol ? bo[(int64_t)tord[t0 + col / nrhs] * nofs + k] : -1;
      src[col] = pr >= 0 ? inter[pr] : -1;
    }
    const double* K = tab + (int64_t)codes[k] * q * q;
    for (int e = threadIdx.x; e < M2L_QP * M2L_QP; e += 256) {
      const int m = e % M2L_QP, kk = e / M2L_QP;
      As[kk][m] = (m < q && kk < q) ? K[m + (int64_t)kk * q] : 0.0;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < M2L_QP * M2L_QP; e += 256) {
      const int kk = e % M2L_QP, col = e / M2L_QP;
      const int j = src[col];
      Bs[kk][col] = (j >= 0 && kk < q) ? w[((int64_t)j * nrhs + col % nrhs) * q + kk] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int k4 = 0; k4 < M2L_QP; k4 += 4) {
      const int kk = k4 + (lane >> 4);
      const double a0 = As[kk][rb0 + (lane & 15)], a1 = As[kk][rb0 + 16 + (lane & 15)];
      const double b0 = Bs[kk][cb0 + (lane & 15)], b1 = Bs[kk][cb0 + 16 + (lane & 15)];
      acc[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, acc[0], 0, 0, 0);
      acc[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, acc[1], 0, 0, 0);
      acc[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, acc[2], 0, 0, 0);
      acc[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, acc[3], 0, 0, 0);
    }
  }
  // lane l's register r of a 16 x 16 block holds row 4 r + l / 16, column l % 16
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int col = cb0 + 16 * (blk & 1) + (lane & 15);
    if (col >= ncol) continue;
    const int tg = tord[t0 + col / nrhs], rr = col % nrhs;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = rb0 + 16 * (blk >> 1) + 4 * r + (lane >> 4);
      if (m < q) g[((int64_t)tg * nrhs + rr) * q + m] = acc[blk][r];
    }
  }
}

// Downward pass (L2L): g_c += T_c g_parent.
__global__ void k_l2l(const int* __restrict__ parent, const int* __restrict__ cbits, int nbc, int q,
                      int nrhs, const double* __restrict__ T, const double* __restrict__ gp,
                      double* __restrict__ gc) {
  const int c = blockIdx.x;
  if (c >= nbc) return;
  const double* Tc = T + (int64_t)cbits[c] * q * q;
  const double* g = gp + (int64_t)parent[c] * q * nrhs;
  for (int e = threadIdx.x; e < q * nrhs; e += WG) {
    const int m = e % q, rr = e / q;
    double acc = 0;
    for (int mp = 0; mp < q; ++mp) acc += Tc[m + (int64_t)mp * q] * g[mp + (int64_t)rr * q];
    gc[(int64_t)c * q * nrhs + e] += acc;
  }
}

// Leaf output: y_a = U_i g_i + sum over adjacent leaves of K(|x_a - x_b|) x_b (+ shift at a = b).
__global__ void __launch_bounds__(WG) k_l2p_p2p(const double* __restrict__ pts, const int64_t* __restrict__ leaf_start,
                          const int* __restrict__ nb_start, const int* __restrict__ nbr, int nb, int d,
                          int q, int nrhs, KernelFn kf, const double* __restrict__ ubar,
                          const double* __restrict__ g, const double* __restrict__ x, int64_t ldx,
                          double* __restrict__ y, int64_t ldy, int with_far) {
  const int i = blockIdx.x;
  if (i >= nb) return;
  const int64_t s = leaf_start[i], m = leaf_start[i + 1] - s;
  __shared__ double sp[P2P_TILE * 3];
  __shared__ int64_t sidx[P2P_TILE];
  // one thread per (target point, rhs); loop in chunks so any leaf size works
  for (int64_t base = 0; base < m * nrhs; base += WG) {
    const int64_t e = base + threadIdx.x;
    const bool act = e < m * nrhs;
    const int64_t a = act ? e % m : 0;
    const int rr = act ? (int)(e / m) : 0;
    double xa[3] = {0, 0, 0};
    if (act)
      for (int k = 0; k < d; ++k) xa[k] = pts[(s + a) * d + k];
    double acc = 0;
    if (act && with_far) {
      const double* U = ubar + s * q;
      const double* gi = g + (int64_t)i * q * nrhs + (int64_t)rr * q;
      for (int mm = 0; mm < q; ++mm) acc += U[a + (int64_t)mm * m] * gi[mm];
    }
    for (int t = nb_start[i]; t < nb_start[i + 1]; ++t) {
      const int j = nbr[t];
      const int64_t sj = leaf_start[j], mj = leaf_start[j + 1] - sj;
      for (int64_t b0 = 0; b0 < mj; b0 += P2P_TILE) {
        const int cnt = (int)((mj - b0) < P2P_TILE ? (mj - b0) : P2P_TILE);
        __syncthreads();
        for (int u = threadIdx.x; u < cnt; u += WG) {
          for (int k = 0; k < d; ++k) sp[u * 3 + k] = pts[(sj + b0 + u) * d + k];
          sidx[u] = sj + b0 + u;
        }
        __syncthreads();
        if (act) {
          for (int u = 0; u < cnt; ++u) {
            double r2 = 0;
            for (int k = 0; k < d; ++k) {
              const double df = xa[k] - sp[u * 3 + k];
              r2 += df * df;
            }
            double kv = kappa(kf, sqrt(r2));
            if (sidx[u] == s + a) kv += kf.shift;
            acc += kv * x[sidx[u] + (int64_t)rr * ldx];
          }
        }
      }
    }
    if (act) y[(s + a) + (int64_t)rr * ldy] = acc;
  }
}

// The same product with one wavefront per leaf box (four boxes per
// workgroup), for leaves of a few points: lanes split over (target, source
// subset). A target gets G = 64 / min(64, pow2ceil(m)) lanes, lane sub of a
// target takes the sources sub, sub + G, ... of every neighbour in turn, and
// the G partial sums are added by a butterfly inside the lane group. The
// order of every sum depends on the box sizes only, so each right-hand side
// gets the same result whatever the number of right-hand sides.
// Near-field blocks of the leaves, evaluated once: box i's block is m_i x S_i
// (S_i the points of its neighbour list, in list order), column-major at
// nfoff[i]; nfcol[t] is the first column of neighbour pair t. The entries are
// the ones k_l2p_p2p_w evaluates (kernel plus the shift on the diagonal).
__global__ void __launch_bounds__(WG) k_near_fill(const double* __restrict__ pts, const int64_t* __restrict__ leaf_start,
                                                  const int* __restrict__ nb_start, const int* __restrict__ nbr, int nb,
                                                  int d, KernelFn kf, const int64_t* __restrict__ nfoff,
                                                  const int* __restrict__ nfcol, double* __restrict__ nf) {
  const int lane = threadIdx.x % WAVE;
  const int i = (int)blockIdx.x * (WG / WAVE) + (int)(threadIdx.x / WAVE);
  if (i >= nb) return;
  const int64_t s = leaf_start[i];
  const int m = (int)(leaf_start[i + 1] - s);
  double* B = nf + nfoff[i];
  for (int t = nb_start[i]; t < nb_start[i + 1]; ++t) {
    const int j = nbr[t];
    const int64_t sj = leaf_start[j];
    const int mj = (int)(leaf_start[j + 1] - sj);
    double* Bt = B + (int64_t)nfcol[t] * m;
    for (int e = lane; e < m * mj; e += WAVE) {
      const int a = e % m, u = e / m;
      double r2 = 0;
      for (int k = 0; k < d; ++k) {
        const double df = pts[(s + a) * d + k] - pts[(sj + u) * d + k];
        r2 += df * df;
      }
      double kv = kappa(kf, sqrt(r2));
      if (sj + u == s + a) kv += kf.shift;
      Bt[e] = kv;
    }
  }
}

__global__ void __launch_bounds__(WG) k_l2p_p2p_w(const double* __restrict__ pts, const int64_t* __restrict__ leaf_start,
                                                  const int* __restrict__ nb_start, const int* __restrict__ nbr,
                                                  int nb, int d, int q, int nrhs, KernelFn kf,
                                                  const double* __restrict__ ubar, const double* __restrict__ g,
                                                  const double* __restrict__ x, int64_t ldx, double* __restrict__ y,
                                                  int64_t ldy, int with_far, const double* __restrict__ nf,
                                                  const int64_t* __restrict__ nfoff, const int* __restrict__ nfcol) {
  const int lane = threadIdx.x % WAVE;
  const int i = (int)blockIdx.x * (WG / WAVE) + (int)(threadIdx.x / WAVE);
  if (i >= nb) return;   // whole wavefronts leave together; no barrier below
  const int64_t s = leaf_start[i];
  const int m = (int)(leaf_start[i + 1] - s);
  int mt = 1;
  while (mt < m && mt < WAVE) mt <<= 1;
  const int G = WAVE / mt;          // lanes per target
  const int tp = WAVE / G;          // targets per pass
  const int sub = lane % G;
  const int t0 = nb_start[i], t1 = nb_start[i + 1];
  // with the stored blocks, lane t holds neighbour t's point range and first column (at most 64 neighbours)
  int64_t nsj = 0;
  int nmj = 0, ncol = 0;
  if (nf && lane < t1 - t0) {
    const int j = nbr[t0 + lane];
    nsj = leaf_start[j];
    nmj = (int)(leaf_start[j + 1] - nsj);
    ncol = nfcol[t0 + lane];
  }
  for (int rr = 0; rr < nrhs; ++rr) {
    for (int a0 = 0; a0 < m; a0 += tp) {
      const int a = a0 + lane / G;
      const bool act = a < m;
      double acc = 0;
      if (nf) {   // the stored near-field block; same entries, same order
        const double* B = nf + nfoff[i] + a;
        for (int t = 0; t < t1 - t0; ++t) {   // neighbour t's range and first column, from lane t (all lanes)
          const int64_t sj = __shfl(nsj, t, WAVE);
          const int mj = __shfl(nmj, t, WAVE);
          const int64_t c0 = __shfl(ncol, t, WAVE);
          if (act)
            for (int u = sub; u < mj; u += G) acc += B[(c0 + u) * m] * x[(sj + u) + (int64_t)rr * ldx];
        }
      } else if (act) {
        {
          double xa[3] = {0, 0, 0};
          for (int k = 0; k < d; ++k) xa[k] = pts[(s + a) * d + k];
          for (int t = t0; t < t1; ++t) {
            const int j = nbr[t];
            const int64_t sj = leaf_start[j];
            const int mj = (int)(leaf_start[j + 1] - sj);
            for (int u = sub; u < mj; u += G) {
              double r2 = 0;
              for (int k = 0; k < d; ++k) {
                const double df = xa[k] - pts[(sj + u) * d + k];
                r2 += df * df;
              }
              double kv = kappa(kf, sqrt(r2));
              if (sj + u == s + a) kv += kf.shift;
              acc += kv * x[(sj + u) + (int64_t)rr * ldx];
            }
          }
        }
      }
      for (int o = G / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
      if (act && sub == 0) {
        if (with_far) {
          const double* U = ubar + s * q;
          const double* gi = g + (int64_t)i * q * nrhs + (int64_t)rr * q;
          double far = 0;
          for (int mm = 0; mm < q; ++mm) far += U[a + (int64_t)mm * m] * gi[mm];
          acc += far;
        }
        y[(s + a) + (int64_t)rr * ldy] = acc;
      }
    }
  }
}

// caller order <-> tree order
__global__ void k_perm_gather(const double* __restrict__ src, int64_t lds, const int* __restrict__ perm,
                              int64_t n, int nrhs, double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t t = e % n;
  const int r = (int)(e / n);
  dst[t + r * ldd] = src[(int64_t)perm[t] + r * lds];
}

__global__ void k_perm_scatter(const double* __restrict__ src, int64_t lds, const int* __restrict__ perm,
                               int64_t n, int nrhs, double* __restrict__ dst, int64_t ldd) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n * nrhs) return;
  const int64_t t = e % n;
  const int r = (int)(e / n);
  dst[(int64_t)perm[t] + r * ldd] = src[t + r * lds];
}

}  // namespace ifmm
