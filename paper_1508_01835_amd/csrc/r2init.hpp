// Initial operators of the extended system E (float64):
//  * orthonormal bases by an exact QR of the Chebyshev bases, bottom-up, the
//    R factors folded into K and the transfers (Sec. 3 opening: an SVD after
//    interpolation reduces the rank; here the rank is min(rows, n^d));
//  * sigma_0(E), the largest eigenvalue magnitude of the symmetric E, by a
//    deterministic Lanczos process (Sec. 2.4);
//  * weights Sigma_U, Sigma_V from an SVD of each box's far-field block row /
//    column (Sec. 2.2, footnote on initial weights), top-down so that the
//    parent's far field is included;
//  * rotation to the singular bases and truncation at tau = max(eps, 64u) sigma_0
//    (eq. methods_SVD_rank_spectralnorm), U and V keeping the same count.
#pragma once

#include "svd.hpp"

namespace ifmm {

constexpr int SW_ROWS = 8;       // rows of the intermediate product held in LDS
constexpr int SW_MAXC = 512;     // largest inner dimension (n^d)

// O(ii, jj) = sum_{kb, kc} X(ii, kb) Y(kb, kc) Z(kc, jj) for an a x e output.
template <class FX, class FY, class FZ, class FO>
__device__ inline void sandwich(int a, int b, int c, int e, FX X, FY Y, FZ Z, FO O, double* sh) {
  for (int a0 = 0; a0 < a; a0 += SW_ROWS) {
    const int ra = (a - a0) < SW_ROWS ? (a - a0) : SW_ROWS;
    for (int t = threadIdx.x; t < ra * c; t += WG) {
      const int ii = t % ra, kc = t / ra;
      double s = 0;
      for (int kb = 0; kb < b; ++kb) s += X(a0 + ii, kb) * Y(kb, kc);
      sh[ii + kc * SW_ROWS] = s;
    }
    __syncthreads();
    for (int t = threadIdx.x; t < ra * e; t += WG) {
      const int ii = t % ra, jj = t / ra;
      double s = 0;
      for (int kc = 0; kc < c; ++kc) s += sh[ii + kc * SW_ROWS] * Z(kc, jj);
      O(a0 + ii, jj, s);
    }
    __syncthreads();
  }
}

__device__ inline int find_row(const int* __restrict__ start, int nb, int t) {
  int lo = 0, hi = nb - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (start[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ inline int offset_code(const int* coords, int d, int i, int j) {
  int code = 0, mul = 1;
  for (int k = 0; k < d; ++k) {
    code += (coords[j * d + k] - coords[i * d + k] + 3) * mul;
    mul *= 7;
  }
  return code;
}

// K_pre(i, j) = R_i Kbar(offset) R_j^T for every interaction-list pair of a level.
__global__ void __launch_bounds__(WG) k_kpre(const int* __restrict__ in_start, const int* __restrict__ inter,
                                             const int* __restrict__ coords, int nb, int d, int q,
                                             const double* __restrict__ tab, const double* __restrict__ R,
                                             const int64_t* __restrict__ roff, const int* __restrict__ r,
                                             double* __restrict__ K, const int64_t* __restrict__ koff) {
  __shared__ double sh[SW_ROWS * SW_MAXC];
  const int t = blockIdx.x;
  const int i = find_row(in_start, nb, t);
  const int j = inter[t];
  const int ri = r[i], rj = r[j];
  const double* Ri = R + roff[i];
  const double* Rj = R + roff[j];
  const double* Kb = tab + (int64_t)offset_code(coords, d, i, j) * q * q;
  double* out = K + koff[t];
  sandwich(ri, q, q, rj, [&](int x, int y) { return Ri[x + (int64_t)y * ri]; },
           [&](int x, int y) { return Kb[x + (int64_t)y * q]; },
           [&](int x, int y) { return Rj[y + (int64_t)x * rj]; },
           [&](int x, int y, double v) { out[x + (int64_t)y * ri] = v; }, sh);
}

// The same triple product by one wavefront, for a * c <= SWW: the a x c
// intermediate sits in the wavefront's LDS slice, and both sums run in the same
// order as in sandwich(), so the results are the same bit for bit. A pair of
// small boxes then costs a wavefront instead of a workgroup and its barriers.
constexpr int SWW = 1024;   // LDS doubles per wavefront
template <class FX, class FY, class FZ, class FO>
__device__ inline void wave_sandwich(int a, int b, int c, int e, FX X, FY Y, FZ Z, FO O, double* sh, int lane) {
  for (int t = lane; t < a * c; t += WAVE) {
    const int ii = t % a, kc = t / a;
    double s = 0;
    for (int kb = 0; kb < b; ++kb) s += X(ii, kb) * Y(kb, kc);
    sh[ii + kc * a] = s;
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (int t = lane; t < a * e; t += WAVE) {
    const int ii = t % a, jj = t / a;
    double s = 0;
    for (int kc = 0; kc < c; ++kc) s += sh[ii + kc * a] * Z(kc, jj);
    O(ii, jj, s);
  }
}

// k_kpre with a wavefront per pair (every r_i q <= SWW).
__global__ void __launch_bounds__(WG) k_kpre_w(const int* __restrict__ in_start, const int* __restrict__ inter,
                                               const int* __restrict__ coords, int nb, int d, int q,
                                               const double* __restrict__ tab, const double* __restrict__ R,
                                               const int64_t* __restrict__ roff, const int* __restrict__ r,
                                               double* __restrict__ K, const int64_t* __restrict__ koff, int npairs) {
  __shared__ double sh[(WG / WAVE) * SWW];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int t = blockIdx.x * (WG / WAVE) + wv;
  if (t >= npairs) return;
  const int i = find_row(in_start, nb, t);
  const int j = inter[t];
  const int ri = r[i], rj = r[j];
  const double* Ri = R + roff[i];
  const double* Rj = R + roff[j];
  const double* Kb = tab + (int64_t)offset_code(coords, d, i, j) * q * q;
  double* out = K + koff[t];
  wave_sandwich(ri, q, q, rj, [&](int x, int y) { return Ri[x + (int64_t)y * ri]; },
                [&](int x, int y) { return Kb[x + (int64_t)y * q]; },
                [&](int x, int y) { return Rj[y + (int64_t)x * rj]; },
                [&](int x, int y, double v) { out[x + (int64_t)y * ri] = v; }, sh + wv * SWW, lane);
}

// K_pre by offset tiles on the FP64 matrix cores (q <= 64). A workgroup holds
// targets of one child position, stacked in 16-row blocks of their R_i (one
// wavefront per block: four targets of rank <= 16, two of rank <= 32 or one
// larger), and walks the position's interaction offsets o. Per offset the
// table K~_o is staged in LDS once for all its targets; each wavefront forms
// X = R_i[16 rows] K~_o, passes it through its own LDS slice into the operand
// layout, and multiplies by R_j^T, R_j read straight from memory, j the
// source at offset o. Every entry is summed in a fixed order (over the table
// index in steps of 4, then over the source node), whatever the grouping.
// The kernels are radial, so K~_{-o} = K~_o^T and K_pre(j, i) = K_pre(i, j)^T:
// each unordered pair is formed once, by its smaller box, and stored both ways.
struct KpreWg {
  int start, cnt, rb, pos;   // targets tlist[start .. start + cnt), 16-row blocks per target, child position
};

__global__ void __launch_bounds__(256, 2) k_kpre_tile(const KpreWg* __restrict__ wgs, const int* __restrict__ tlist,
                                                   const int* __restrict__ bo, const int* __restrict__ inter,
                                                   const int* __restrict__ rev, int nofs,
                                                   const int* __restrict__ ocode, int q,
                                                   const double* __restrict__ tab, const double* __restrict__ R,
                                                   const int64_t* __restrict__ roff, const int* __restrict__ r,
                                                   double* __restrict__ K, const int64_t* __restrict__ koff) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  __shared__ double Ks[64][65];       // Ks[k][n] = K~_o[k, n]
  __shared__ double Xs[4][16][65];    // per wavefront: its 16 x q block of X
  const KpreWg g = wgs[blockIdx.x];
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const bool act = w < g.cnt * g.rb;
  const int ti = act ? tlist[g.start + w / g.rb] : 0;
  const int rb = act ? w % g.rb : 0;
  const int ri = act ? r[ti] : 0;
  const int nks = (q + 3) / 4, ncb = (q + 15) / 16;
  // A operand of R_i rows 16 rb .. 16 rb + 15: lane l holds row l % 16, column 4 ks + l / 16
  double af[16];
  {
    const double* Ri = R + roff[ti];
    const int a = 16 * rb + (lane & 15);
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int k = 4 * ks + (lane >> 4);
      af[ks] = (act && a < ri && k < q) ? Ri[a + (int64_t)k * ri] : 0.0;
    }
  }
  const int* codes = ocode + g.pos * nofs;
  for (int o = 0; o < nofs; ++o) {
    const int t = act ? bo[(int64_t)ti * nofs + o] : -1;
    const int j = t >= 0 ? inter[t] : -1;
    const bool need = j > ti;   // the pair's smaller box forms it
    if (!__syncthreads_or(need)) continue;   // also: the previous offset's reads of Ks are done
    const double* Kt = tab + (int64_t)codes[o] * q * q;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
      const int k = e & 63, n = e >> 6;
      Ks[k][n] = (k < q && n < q) ? Kt[k + (int64_t)n * q] : 0.0;
    }
    __syncthreads();
    if (!need) continue;
    v4d x[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) x[cb] = v4d{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int k = 4 * ks + (lane >> 4);
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
        if (ks < nks && cb < ncb)
          x[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[ks], Ks[k][16 * cb + (lane & 15)], x[cb], 0, 0, 0);
    }
    // result lane layout: register e of block cb holds row 4 e + l / 16, column 16 cb + l % 16
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int e = 0; e < 4; ++e) Xs[w][4 * e + (lane >> 4)][16 * cb + (lane & 15)] = x[cb][e];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int rj = r[j];
    const double* Rj = R + roff[j];
    const int nyb = (rj + 15) / 16;
    v4d y[4];
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) y[cb] = v4d{0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < 16; ++ks) {
      const int n = 4 * ks + (lane >> 4);
      const double a = Xs[w][lane & 15][n];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        if (ks < nks && cb < nyb) {
          const int b = 16 * cb + (lane & 15);
          const double bv = (b < rj && n < q) ? Rj[b + (int64_t)n * rj] : 0.0;
          y[cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, y[cb], 0, 0, 0);
        }
      }
    }
    double* out = K + koff[t];
    double* outT = K + koff[rev[t]];   // K_pre(j, i): rj x ri
#pragma unroll
    for (int cb = 0; cb < 4; ++cb) {
      const int b = 16 * cb + (lane & 15);
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int a = 16 * rb + 4 * e + (lane >> 4);
        if (cb < nyb && a < ri && b < rj) {
          out[a + (int64_t)b * ri] = y[cb][e];
          outT[b + (int64_t)a * rj] = y[cb][e];
        }
      }
    }
    // Xs is rewritten only after the next offset's barrier
  }
}

// K(i, j) = WU_i[:, :k_i]^T K_pre(i, j) WV_j[:, :k_j].
__global__ void __launch_bounds__(WG) k_krot(const int* __restrict__ in_start, const int* __restrict__ inter, int nb,
                                             const double* __restrict__ Kpre, const int64_t* __restrict__ kpoff,
                                             const int* __restrict__ r, const double* __restrict__ WU,
                                             const double* __restrict__ WV, const int64_t* __restrict__ woff,
                                             const int* __restrict__ k, double* __restrict__ K,
                                             const int64_t* __restrict__ koff) {
  __shared__ double sh[SW_ROWS * SW_MAXC];
  const int t = blockIdx.x;
  const int i = find_row(in_start, nb, t);
  const int j = inter[t];
  const int ri = r[i], rj = r[j], ki = k[i], kj = k[j];
  const double* A = WU + woff[i];
  const double* B = Kpre + kpoff[t];
  const double* C = WV + woff[j];
  double* out = K + koff[t];
  sandwich(ki, ri, rj, kj, [&](int x, int y) { return A[y + (int64_t)x * ri]; },
           [&](int x, int y) { return B[x + (int64_t)y * ri]; },
           [&](int x, int y) { return C[x + (int64_t)y * rj]; },
           [&](int x, int y, double v) { out[x + (int64_t)y * ki] = v; }, sh);
}

// k_krot with a wavefront per pair (every k_i r_j <= SWW).
__global__ void __launch_bounds__(WG) k_krot_w(const int* __restrict__ in_start, const int* __restrict__ inter, int nb,
                                               const double* __restrict__ Kpre, const int64_t* __restrict__ kpoff,
                                               const int* __restrict__ r, const double* __restrict__ WU,
                                               const double* __restrict__ WV, const int64_t* __restrict__ woff,
                                               const int* __restrict__ k, double* __restrict__ K,
                                               const int64_t* __restrict__ koff, int npairs) {
  __shared__ double sh[(WG / WAVE) * SWW];
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const int t = blockIdx.x * (WG / WAVE) + wv;
  if (t >= npairs) return;
  const int i = find_row(in_start, nb, t);
  const int j = inter[t];
  const int ri = r[i], rj = r[j], ki = k[i], kj = k[j];
  const double* A = WU + woff[i];
  const double* B = Kpre + kpoff[t];
  const double* C = WV + woff[j];
  double* out = K + koff[t];
  wave_sandwich(ki, ri, rj, kj, [&](int x, int y) { return A[y + (int64_t)x * ri]; },
                [&](int x, int y) { return B[x + (int64_t)y * ri]; },
                [&](int x, int y) { return C[x + (int64_t)y * rj]; },
                [&](int x, int y, double v) { out[x + (int64_t)y * ki] = v; }, sh + wv * SWW, lane);
}

// P(i) = W_i[:, :k_i]^T Ppre(i) W_parent[:, :k_parent]; Ppre(i) is r_i x r_p with leading dim pld[i].
__global__ void __launch_bounds__(WG) k_prot(const int* __restrict__ parent, int nb,
                                             const double* __restrict__ Ppre, const int64_t* __restrict__ ppoff,
                                             const int* __restrict__ pld, const int* __restrict__ r,
                                             const int* __restrict__ rpar, const double* __restrict__ W,
                                             const int64_t* __restrict__ woff, const double* __restrict__ Wp,
                                             const int64_t* __restrict__ wpoff, const int* __restrict__ k,
                                             const int* __restrict__ kpar, double* __restrict__ out,
                                             const int64_t* __restrict__ ooff) {
  __shared__ double sh[SW_ROWS * SW_MAXC];
  const int i = blockIdx.x;
  if (i >= nb) return;
  const int p = parent[i];
  const int ri = r[i], rp = rpar[p], ki = k[i], kp = kpar[p];
  const int ld = pld[i];
  const double* A = W + woff[i];
  const double* B = Ppre + ppoff[i];
  const double* C = Wp + wpoff[p];
  double* o = out + ooff[i];
  sandwich(ki, ri, rp, kp, [&](int x, int y) { return A[y + (int64_t)x * ri]; },
           [&](int x, int y) { return B[x + (int64_t)y * ld]; },
           [&](int x, int y) { return C[x + (int64_t)y * rp]; },
           [&](int x, int y, double v) { o[x + (int64_t)y * ki] = v; }, sh);
}

// Rows of M^T for the weights of box i (U side: K_pre(i,j)^T for j in I(i), then
// (PU(i) G_p)^T; V side: K_pre(j,i), then (PV(i) GV_p)^T).
__global__ void __launch_bounds__(WG) k_weight_rows(const int* __restrict__ in_start, const int* __restrict__ inter,
                                                    const int64_t* __restrict__ in_rev_unused, int nb, int side,
                                                    const int* __restrict__ rev, const double* __restrict__ Kpre,
                                                    const int64_t* __restrict__ kpoff, const int* __restrict__ r,
                                                    const int* __restrict__ parent, const double* __restrict__ Ppre,
                                                    const int64_t* __restrict__ ppoff, const int* __restrict__ pld,
                                                    const int* __restrict__ rpar, const double* __restrict__ Gp,
                                                    const int64_t* __restrict__ gpoff, const int* __restrict__ gpcols,
                                                    double* __restrict__ M, const int64_t* __restrict__ moff,
                                                    const int* __restrict__ mrows, int i0) {
  const int i = i0 + (int)blockIdx.x;   // boxes i0 .. nb - 1
  if (i >= nb) return;
  const int ri = r[i];
  const int rows = mrows[i];
  double* out = M + moff[i];   // rows x ri, ld rows
  int row0 = 0;
  for (int t = in_start[i]; t < in_start[i + 1]; ++t) {
    const int j = inter[t];
    const int rj = r[j];
    if (side == 0) {
      const double* B = Kpre + kpoff[t];          // ri x rj
      for (int e = threadIdx.x; e < rj * ri; e += WG) {
        const int a = e % rj, c = e / rj;
        out[(row0 + a) + (int64_t)c * rows] = B[c + (int64_t)a * ri];
      }
    } else {
      const double* B = Kpre + kpoff[rev[t]];     // K_pre(j, i): rj x ri
      for (int e = threadIdx.x; e < rj * ri; e += WG) {
        const int a = e % rj, c = e / rj;
        out[(row0 + a) + (int64_t)c * rows] = B[a + (int64_t)c * rj];
      }
    }
    row0 += rj;
  }
  if (parent) {
    const int p = parent[i];
    const int rp = rpar[p];
    const int gc = gpcols[p];
    const double* Pi = Ppre + ppoff[i];   // ri x rp, ld pld[i]
    const int ld = pld[i];
    const double* G = Gp + gpoff[p];      // rp x gc, ld rp
    for (int e = threadIdx.x; e < gc * ri; e += WG) {
      const int a = e % gc, c = e / gc;
      double s = 0;
      for (int m = 0; m < rp; ++m) s += Pi[c + (int64_t)m * ld] * G[m + (int64_t)a * rp];
      out[(row0 + a) + (int64_t)c * rows] = s;
    }
  }
}

// -------------------------------------------------- E products for sigma_0
// Vector layout: x (n) | for l = L..2: z_l (nb_l * q) | y_l (nb_l * q); entries
// of a box beyond its rank stay zero. E is symmetric (radial kernels), so the
// power iteration applies E twice.
// z-type rows at level l: (V^T x^(l))_i - y_i.
__global__ void k_e_zrows(int nb, int q, const int* __restrict__ r, int leaf,
                          const int64_t* __restrict__ leaf_start, const double* __restrict__ Q,
                          const double* __restrict__ x, const int* __restrict__ ch_start,
                          const double* __restrict__ Ppre, const int64_t* __restrict__ ppoff,
                          const int* __restrict__ pld, const int* __restrict__ rch,
                          const double* __restrict__ ych, const double* __restrict__ yl,
                          double* __restrict__ out) {
  const int i = blockIdx.x;
  if (i >= nb) return;
  const int ri = r[i];
  for (int m = threadIdx.x; m < ri; m += WG) {
    double s = 0;
    if (leaf) {
      const int64_t st = leaf_start[i], mi = leaf_start[i + 1] - st;
      const double* Qi = Q + st * q;
      for (int64_t a = 0; a < mi; ++a) s += Qi[a + (int64_t)m * mi] * x[st + a];
    } else {
      for (int c = ch_start[i]; c < ch_start[i + 1]; ++c) {
        const double* Pc = Ppre + ppoff[c];
        const int ld = pld[c];
        for (int a = 0; a < rch[c]; ++a) s += Pc[a + (int64_t)m * ld] * ych[(int64_t)c * q + a];
      }
    }
    out[(int64_t)i * q + m] = s - yl[(int64_t)i * q + m];
  }
}

// The far-field sum of the y rows without the K_pre blocks: since
// K_pre(i,j) = R_i K~_o R_j^T, sum_j K_pre(i,j) y_j = R_i g_i with
// g = M2L(w), w_j = R_j^T y_j. Both transforms take a wavefront per box,
// a lane per entry (q <= 64).
__global__ void __launch_bounds__(WG) k_e_rty(int nb, int q, const int* __restrict__ r, const double* __restrict__ R,
                                              const int64_t* __restrict__ roff, const double* __restrict__ yl,
                                              double* __restrict__ w) {
  const int lane = threadIdx.x % WAVE;
  const int j = (int)blockIdx.x * (WG / WAVE) + (int)(threadIdx.x / WAVE);
  if (j >= nb || lane >= q) return;
  const int rj = r[j];
  const double* Rj = R + roff[j];
  const double* y = yl + (int64_t)j * q;
  double s = 0;
  for (int a = 0; a < rj; ++a) s += Rj[a + (int64_t)lane * rj] * y[a];
  w[(int64_t)j * q + lane] = s;
}

// y-type rows from the M2L result g: -z_i + R_i g_i + PU(i) z_parent.
__global__ void __launch_bounds__(WG) k_e_yrows_g(int nb, int q, const int* __restrict__ r,
                                                  const double* __restrict__ R, const int64_t* __restrict__ roff,
                                                  const double* __restrict__ g, const double* __restrict__ zl,
                                                  const int* __restrict__ parent, const double* __restrict__ Ppre,
                                                  const int64_t* __restrict__ ppoff, const int* __restrict__ pld,
                                                  const int* __restrict__ rpar, const double* __restrict__ zpar,
                                                  double* __restrict__ out) {
  const int lane = threadIdx.x % WAVE;
  const int i = (int)blockIdx.x * (WG / WAVE) + (int)(threadIdx.x / WAVE);
  if (i >= nb) return;
  const int ri = r[i];
  if (lane >= ri) return;
  const double* Ri = R + roff[i];
  const double* gi = g + (int64_t)i * q;
  double s = -zl[(int64_t)i * q + lane];
  for (int k = 0; k < q; ++k) s += Ri[lane + (int64_t)k * ri] * gi[k];
  if (parent) {
    const int p = parent[i];
    const double* Pi = Ppre + ppoff[i];
    const int ld = pld[i];
    for (int a = 0; a < rpar[p]; ++a) s += Pi[lane + (int64_t)a * ld] * zpar[(int64_t)p * q + a];
  }
  out[(int64_t)i * q + lane] = s;
}

// y-type rows at level l: -z_i + sum_{j in I(i)} K_pre(i,j) y_j + PU(i) z_parent.
__global__ void k_e_yrows(int nb, int q, const int* __restrict__ r, const int* __restrict__ in_start,
                          const int* __restrict__ inter, const double* __restrict__ Kpre,
                          const int64_t* __restrict__ kpoff, const double* __restrict__ zl,
                          const double* __restrict__ yl, const int* __restrict__ parent,
                          const double* __restrict__ Ppre, const int64_t* __restrict__ ppoff,
                          const int* __restrict__ pld, const int* __restrict__ rpar,
                          const double* __restrict__ zpar, double* __restrict__ out) {
  const int i = blockIdx.x;
  if (i >= nb) return;
  const int ri = r[i];
  for (int m = threadIdx.x; m < ri; m += WG) {
    double s = -zl[(int64_t)i * q + m];
    for (int t = in_start[i]; t < in_start[i + 1]; ++t) {
      const int j = inter[t];
      const int rj = r[j];
      const double* B = Kpre + kpoff[t];
      for (int a = 0; a < rj; ++a) s += B[m + (int64_t)a * ri] * yl[(int64_t)j * q + a];
    }
    if (parent) {
      const int p = parent[i];
      const double* Pi = Ppre + ppoff[i];
      const int ld = pld[i];
      for (int a = 0; a < rpar[p]; ++a) s += Pi[m + (int64_t)a * ld] * zpar[(int64_t)p * q + a];
    }
    out[(int64_t)i * q + m] = s;
  }
}

// The same y rows for levels whose ranks are at most 32: each thread takes
// whole blocks of the box's interaction list and accumulates every row of the
// box in registers (all threads busy even when the ranks are small); the
// workgroup adds the per-thread sums with the wavefront reduce-scatter and one
// pass over LDS, in a fixed order.
__global__ void __launch_bounds__(WG) k_e_yrows32(int nb, int q, const int* __restrict__ r,
                                                  const int* __restrict__ in_start, const int* __restrict__ inter,
                                                  const double* __restrict__ Kpre, const int64_t* __restrict__ kpoff,
                                                  const double* __restrict__ zl, const double* __restrict__ yl,
                                                  const int* __restrict__ parent, const double* __restrict__ Ppre,
                                                  const int64_t* __restrict__ ppoff, const int* __restrict__ pld,
                                                  const int* __restrict__ rpar, const double* __restrict__ zpar,
                                                  double* __restrict__ out) {
  __shared__ double part[WG / WAVE][32];
  const int i = blockIdx.x;
  if (i >= nb) return;
  const int ri = r[i];
  double acc[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) acc[m] = 0;
  for (int t = in_start[i] + threadIdx.x; t < in_start[i + 1]; t += WG) {
    const int j = inter[t];
    const int rj = r[j];
    const double* B = Kpre + kpoff[t];
    const double* yj = yl + (int64_t)j * q;
    for (int a = 0; a < rj; ++a) {
      const double y = yj[a];
#pragma unroll
      for (int m = 0; m < 32; ++m)
        if (m < ri) acc[m] += B[m + (int64_t)a * ri] * y;
    }
  }
  if (parent) {
    const int p = parent[i];
    const double* Pi = Ppre + ppoff[i];
    const int ld = pld[i];
    for (int a = threadIdx.x; a < rpar[p]; a += WG) {
      const double z = zpar[(int64_t)p * q + a];
#pragma unroll
      for (int m = 0; m < 32; ++m)
        if (m < ri) acc[m] += Pi[m + (int64_t)a * ld] * z;
    }
  }
  const int lane = threadIdx.x % WAVE, wv = threadIdx.x / WAVE;
  const double rs = wave_sum32_scatter(acc, lane);
  if ((lane & 1) == 0) part[wv][lane >> 1] = rs;
  __syncthreads();
  if ((int)threadIdx.x < ri) {
    double s = -zl[(int64_t)i * q + threadIdx.x];
    for (int w = 0; w < WG / WAVE; ++w) s += part[w][threadIdx.x];
    out[(int64_t)i * q + threadIdx.x] = s;
  }
}

__global__ void k_sumsq_partial(const double* __restrict__ v, int64_t n, double* __restrict__ part) {
  __shared__ double sh[WG / WAVE];
  double s = 0;
  for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) s += v[i] * v[i];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_axpy(double* __restrict__ y, const double* __restrict__ x, int64_t n, double a) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e < n) y[e] += a * x[e];
}

__global__ void k_copy_scaled(double* __restrict__ y, const double* __restrict__ x, int64_t n, double a) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e < n) y[e] = a * x[e];
}

__global__ void k_dot_partial(const double* __restrict__ a, const double* __restrict__ b, int64_t n,
                              double* __restrict__ part) {
  __shared__ double sh[WG / WAVE];
  double s = 0;
  for (int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x; e < n; e += (int64_t)gridDim.x * WG) s += a[e] * b[e];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void k_scale(double* __restrict__ v, int64_t n, double a) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < n) v[i] *= a;
}

__global__ void k_fill(double* __restrict__ v, int64_t n, double a) {
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i < n) v[i] = a;
}

}  // namespace ifmm
