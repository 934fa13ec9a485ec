// Uniform 2^d-tree of the point cloud (Sec. 2.1; Sec. 2.3 for the list
// bounds; Sec. 3 opening for the uniform tree): root = tight bounding cube,
// leaf level L, occupied boxes only, points in Morton order of their leaf.
// Keys and the sort run on the GPU; the box tables, neighbour lists N(i),
// interaction lists I(i) (Sec. 2.2: children of the parent's neighbours that
// are not neighbours) and colours are planned on the host.
#pragma once

#include <algorithm>
#include <unordered_map>

#include "common.hpp"
#include "sort.hpp"

namespace ifmm {

struct HLevel {
  int l = 0, nb = 0;
  std::vector<int> coords;          // nb * d
  std::vector<uint64_t> keys;       // Morton keys at this level
  std::vector<int> parent;          // index at level l-1
  std::vector<int> ch_start, ch;    // children at level l+1 (CSR, Morton order)
  std::vector<int> nb_start, nbr;   // N(i), itself included, Morton order
  std::vector<int> in_start, inter; // I(i), Morton order
  std::vector<int> colour;          // sum_k (c_k mod 3) 3^k
  int ncolour = 1;
  std::vector<std::vector<int>> classes;   // boxes of each colour, Morton order
};

struct HTree {
  int64_t n = 0;
  int d = 0, L = 0;
  double origin[3] = {0, 0, 0}, side = 1.0, inv = 1.0;
  std::vector<int64_t> perm;        // tree position -> caller index
  std::vector<int64_t> leaf_start;  // nb_L + 1 point offsets
  std::vector<HLevel> lev;          // lev[l], l = 0..L (0, 1 unused)
  double box_size(int l) const { return side / (double)(1ll << l); }
};

// ------------------------------------------------------------------ kernels
// Per-block minimum and maximum of every coordinate; a coordinate that is not
// finite turns the block's minimum into NaN so the host rejects the input.
__global__ void k_bbox_partial(const double* __restrict__ p, int64_t n, int d,
                               double* __restrict__ part /* blocks x 2d */) {
  __shared__ double smin[WG], smax[WG];
  for (int k = 0; k < d; ++k) {
    double lo = INFINITY, hi = -INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += (int64_t)gridDim.x * WG) {
      const double x = p[i * d + k];
      if (!isfinite(x)) { lo = NAN; hi = NAN; break; }
      lo = fmin(lo, x);
      hi = fmax(hi, x);
    }
    smin[threadIdx.x] = lo;
    smax[threadIdx.x] = hi;
    __syncthreads();
    for (int s = WG / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        const double a = smin[threadIdx.x], b = smin[threadIdx.x + s];
        const double c = smax[threadIdx.x], e = smax[threadIdx.x + s];
        smin[threadIdx.x] = (a != a || b != b) ? NAN : fmin(a, b);
        smax[threadIdx.x] = (c != c || e != e) ? NAN : fmax(c, e);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      part[blockIdx.x * 2 * d + k] = smin[0];
      part[blockIdx.x * 2 * d + d + k] = smax[0];
    }
    __syncthreads();
  }
}

__device__ inline uint64_t interleave(const int* c, int d, int bits) {
  uint64_t key = 0;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) key |= (uint64_t)((c[k] >> b) & 1) << (b * d + k);
  return key;
}

// Leaf box key of each point: c = clamp(floor((x - origin) * inv * 2^L)).
__global__ void k_point_keys(const double* __restrict__ p, int64_t n, int d, double o0, double o1,
                             double o2, double inv, int L, uint64_t* __restrict__ keys,
                             int* __restrict__ idx) {
#pragma clang fp contract(off)
  const int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (i >= n) return;
  const double o[3] = {o0, o1, o2};
  const int nl = 1 << L;
  int c[3] = {0, 0, 0};
  for (int k = 0; k < d; ++k) {
    const double t = (p[i * d + k] - o[k]) * inv;
    double f = floor(t * (double)nl);
    int ci = f < 0.0 ? 0 : (f > (double)(nl - 1) ? nl - 1 : (int)f);
    c[k] = ci;
  }
  keys[i] = interleave(c, d, L);
  idx[i] = (int)i;
}

__global__ void k_gather_points(const double* __restrict__ p, const int* __restrict__ idx, int64_t n,
                                int d, double* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (t >= n) return;
  const int64_t s = idx[t];
  for (int k = 0; k < d; ++k) out[t * d + k] = p[s * d + k];
}

// ------------------------------------------------------------------ host side
inline void deinterleave(uint64_t key, int d, int bits, int* c) {
  for (int k = 0; k < d; ++k) c[k] = 0;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) c[k] |= (int)((key >> (b * d + k)) & 1ull) << b;
}

inline uint64_t interleave_h(const int* c, int d, int bits) {
  uint64_t key = 0;
  for (int b = 0; b < bits; ++b)
    for (int k = 0; k < d; ++k) key |= (uint64_t)((c[k] >> b) & 1) << (b * d + k);
  return key;
}

// Box lookup by integer coordinates at one level.
struct BoxLookup {
  int d = 0, l = 0;
  std::vector<int> grid;                      // dense when small enough
  std::unordered_map<uint64_t, int> map;      // otherwise
  void build(const HLevel& lv, int dim) {
    d = dim;
    l = lv.l;
    const int64_t cells = 1ll << (l * d);
    if (l * d <= 26) {
      grid.assign((size_t)cells, -1);
      for (int i = 0; i < lv.nb; ++i) grid[(size_t)lv.keys[i]] = i;
    } else {
      map.reserve((size_t)lv.nb * 2);
      for (int i = 0; i < lv.nb; ++i) map[lv.keys[i]] = i;
    }
  }
  int find(const int* c) const {
    const int nl = 1 << l;
    for (int k = 0; k < d; ++k)
      if (c[k] < 0 || c[k] >= nl) return -1;
    const uint64_t key = interleave_h(c, d, l);
    if (!grid.empty()) return grid[(size_t)key];
    auto it = map.find(key);
    return it == map.end() ? -1 : it->second;
  }
};

// Build levels, lists and colours from the sorted leaf keys.
inline void plan_tree(HTree& T, const std::vector<uint64_t>& sorted_keys) {
  const int d = T.d, L = T.L;
  const int64_t n = T.n;
  T.lev.assign(L + 1, HLevel());
  HLevel& leaf = T.lev[L];
  leaf.l = L;
  T.leaf_start.clear();
  for (int64_t i = 0; i < n; ++i)
    if (i == 0 || sorted_keys[i] != sorted_keys[i - 1]) {
      T.leaf_start.push_back(i);
      leaf.keys.push_back(sorted_keys[i]);
    }
  T.leaf_start.push_back(n);
  leaf.nb = (int)leaf.keys.size();
  for (int l = L - 1; l >= 2; --l) {
    HLevel& ch = T.lev[l + 1];
    HLevel& lv = T.lev[l];
    lv.l = l;
    ch.parent.assign(ch.nb, -1);
    for (int i = 0; i < ch.nb; ++i) {
      const uint64_t pk = ch.keys[i] >> d;
      if (lv.keys.empty() || lv.keys.back() != pk) lv.keys.push_back(pk);
      ch.parent[i] = (int)lv.keys.size() - 1;
    }
    lv.nb = (int)lv.keys.size();
    lv.ch_start.assign(lv.nb + 1, 0);
    for (int i = 0; i < ch.nb; ++i) lv.ch_start[ch.parent[i] + 1]++;
    for (int p = 0; p < lv.nb; ++p) lv.ch_start[p + 1] += lv.ch_start[p];
    lv.ch.resize(ch.nb);
    for (int i = 0; i < ch.nb; ++i) lv.ch[i] = i;   // children are contiguous, in order
  }
  for (int l = 2; l <= L; ++l) {
    HLevel& lv = T.lev[l];
    lv.coords.resize((size_t)lv.nb * d);
    for (int i = 0; i < lv.nb; ++i) deinterleave(lv.keys[i], d, l, &lv.coords[(size_t)i * d]);
    lv.colour.resize(lv.nb);
    int nc = 1;
    for (int k = 0; k < d; ++k) nc *= 3;
    lv.ncolour = nc;
    lv.classes.assign(nc, {});
    for (int i = 0; i < lv.nb; ++i) {
      int c = 0, m = 1;
      for (int k = 0; k < d; ++k) { c += (lv.coords[(size_t)i * d + k] % 3) * m; m *= 3; }
      lv.colour[i] = c;
      lv.classes[c].push_back(i);
    }
    BoxLookup look;   // coordinate lookup, used at level 2 (no parent lists)
    if (l == 2) look.build(lv, d);
    int offs1[27][3];
    int no = 0;
    {
      int o[3];
      const int cnt = (d == 1 ? 3 : d == 2 ? 9 : 27);
      for (int e = 0; e < cnt; ++e) {
        int r = e;
        for (int k = 0; k < 3; ++k) { o[k] = k < d ? (r % 3) - 1 : 0; r /= 3; }
        for (int k = 0; k < 3; ++k) offs1[no][k] = o[k];
        ++no;
      }
    }
    lv.nb_start.assign(lv.nb + 1, 0);
    lv.in_start.assign(lv.nb + 1, 0);
    lv.nbr.clear();
    lv.inter.clear();
    if (l > 2) {
      // N(i) and I(i) are the children of the parent's neighbours that are,
      // respectively are not, adjacent to i. The parent's list is in Morton
      // order and children are contiguous in Morton order, so both lists come
      // out sorted.
      const HLevel& pl = T.lev[l - 1];
      lv.nbr.reserve((size_t)lv.nb * no);
      lv.inter.reserve((size_t)lv.nb * (no * (1 << d) - no));
      for (int i = 0; i < lv.nb; ++i) {
        const int* ci = &lv.coords[(size_t)i * d];
        const int p = lv.parent[i];
        for (int t = pl.nb_start[p]; t < pl.nb_start[p + 1]; ++t) {
          const int pn = pl.nbr[t];
          for (int j = pl.ch_start[pn]; j < pl.ch_start[pn + 1]; ++j) {
            const int* cj = &lv.coords[(size_t)j * d];
            bool adj = true;
            for (int k = 0; k < d; ++k) {
              const int dd = cj[k] - ci[k];
              if (dd > 1 || dd < -1) adj = false;
            }
            (adj ? lv.nbr : lv.inter).push_back(j);
          }
        }
        lv.nb_start[i + 1] = (int)lv.nbr.size();
        lv.in_start[i + 1] = (int)lv.inter.size();
      }
      continue;
    }
    std::vector<int> tmp;
    for (int i = 0; i < lv.nb; ++i) {
      const int* ci = &lv.coords[(size_t)i * d];
      tmp.clear();
      for (int e = 0; e < no; ++e) {
        int c[3];
        for (int k = 0; k < d; ++k) c[k] = ci[k] + offs1[e][k];
        const int j = look.find(c);
        if (j >= 0) tmp.push_back(j);
      }
      std::sort(tmp.begin(), tmp.end());
      lv.nbr.insert(lv.nbr.end(), tmp.begin(), tmp.end());
      lv.nb_start[i + 1] = (int)lv.nbr.size();
      tmp.clear();
      int pc[3];
      for (int k = 0; k < d; ++k) pc[k] = ci[k] >> 1;
      for (int e = 0; e < no; ++e) {
        for (int cb = 0; cb < (1 << d); ++cb) {
          int c[3];
          int far = 0;
          for (int k = 0; k < d; ++k) {
            c[k] = 2 * (pc[k] + offs1[e][k]) + ((cb >> k) & 1);
            const int dd = c[k] - ci[k];
            if (dd > 1 || dd < -1) far = 1;
          }
          if (!far) continue;
          const int j = look.find(c);
          if (j >= 0) tmp.push_back(j);
        }
      }
      std::sort(tmp.begin(), tmp.end());
      lv.inter.insert(lv.inter.end(), tmp.begin(), tmp.end());
      lv.in_start[i + 1] = (int)lv.inter.size();
    }
  }
}

inline bool adjacent(const HLevel& lv, int d, int i, int j) {
  for (int k = 0; k < d; ++k) {
    const int dd = lv.coords[(size_t)i * d + k] - lv.coords[(size_t)j * d + k];
    if (dd > 1 || dd < -1) return false;
  }
  return true;
}

// Offset code of j relative to i in [-3,3]^d (7^d table), -1 if farther.
inline int offset7(const HLevel& lv, int d, int i, int j) {
  int code = 0, m = 1;
  for (int k = 0; k < d; ++k) {
    const int dd = lv.coords[(size_t)j * d + k] - lv.coords[(size_t)i * d + k];
    if (dd > 3 || dd < -3) return -1;
    code += (dd + 3) * m;
    m *= 7;
  }
  return code;
}

}  // namespace ifmm
