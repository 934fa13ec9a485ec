// Substitution with the stored factors (Alg. 1: solve for y^(2), then
// substitute back down the tree) as batched matrix-vector products.
//
// Vector store V: one row per unknown of every level (x~ of level L, then the
// x~ of each coarser level = the y of the level below, down to the y^(2) of
// level 2), then the c rows (c = A b(x~_i) of every elimination). The nrhs
// right-hand sides of a row are contiguous, so one pass over a factor block
// serves all of them.
//
//  forward, level L..2, colour classes in order, one launch per class: a
//    workgroup takes 64 rows of H = [A; G] of one elimination; rows of A
//    write c, rows of G subtract from the F rows (x~ of later-coloured and y
//    of earlier-coloured neighbours, disjoint between the eliminations of a
//    class);
//  top: y^(2) = T^-1 b(y^(2));
//  backward, level 2..L, classes in reverse: x~_i = c - W_x x_F.
// The top and backward products are split over column chunks: partial sums,
// then a reduction in a fixed order (deterministic), two launches each. A
// partial-sum workgroup takes 64 rows (a row per lane) and its four wavefronts
// split the chunk's columns, so that the few rows of a box at the fine and
// middle levels still fill the lanes and the columns spread over the chip.
//
// Memory bound: every stored factor element is read once per call. The plan
// (task tables) is uploaded once per factorization; a call only launches.
#pragma once

#include <map>

#include "factor.hpp"

namespace ifmm {

constexpr int SV_KCH = 256;   // widest partial-sum chunk (columns); a launch narrows it to 128 or 64
constexpr int SV_MIN_WG = 1024;   // while it has fewer workgroups than this. Every right-hand-side
                                  // count uses the same chunks, so columns are solved bitwise alike
constexpr int SV_KT = 64;     // chunk widths are multiples of this
constexpr int SV_FKT = 256;   // columns of x staged in LDS at a time by the forward kernel
constexpr int SV_RT = WAVE;   // rows of one partial-sum workgroup (a row per lane)
constexpr int SV_NW = WG / WAVE;   // its wavefronts, which split the columns

struct SvNode {
  int64_t pos;    // V row of the node's first unknown
  int off, dim;   // rows [off, off + dim) of the elimination's F
};

struct FwTask {
  const void* H;
  int64_t ld;
  int m, rows;            // rows = m + f
  int node0, nnode;
  int64_t in_pos, c_pos;  // V rows of x~_i and of c
  int chunk0, pad;        // first workgroup of the task in its launch
};

// out = c + alpha A x, A rows x cols (ld), x gathered through the nodes.
struct BwTask {
  const void* A;
  int64_t ld;
  int rows, cols;
  int node0, nnode;
  int64_t out_pos, c_pos;  // c_pos < 0: c = 0
  int64_t part;            // first partial-sum row
  int chunk0, nrc, nkc, chunk0b;
  int kch;                 // columns of one chunk (a multiple of SV_KT)
  double alpha;
};

// node of a task owning row (column) k; the nodes of a task are in increasing
// off, the first at off 0: binary search for the last node with off <= k
__device__ inline int64_t sv_pos(const SvNode* __restrict__ nodes, int node0, int nnode, int k) {
  int lo = node0, hi = node0 + nnode - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (nodes[mid].off <= k) lo = mid; else hi = mid - 1;
  }
  return nodes[lo].pos + (k - nodes[lo].off);
}

// A workgroup copies its task's nodes into LDS first (one round trip for all
// of them) when there are at most SV_NODE_LDS, so that the searches above run
// in LDS instead of as chains of dependent global loads; otherwise it
// searches the global table. Call before the workgroup's first barrier and
// pass the result to sv_pos_any after it.
constexpr int SV_NODE_LDS = 128;
__device__ inline bool sv_nodes_to_lds(const SvNode* __restrict__ nodes, int node0, int nnode, SvNode* nl) {
  if (nnode > SV_NODE_LDS) return false;
  for (int a = threadIdx.x; a < nnode; a += WG) nl[a] = nodes[node0 + a];
  return true;
}
__device__ inline int64_t sv_pos_any(bool in_lds, const SvNode* nl, const SvNode* __restrict__ nodes, int node0,
                                     int nnode, int k) {
  return in_lds ? sv_pos(nl, 0, nnode, k) : sv_pos(nodes, node0, nnode, k);
}

// A workgroup takes SV_RT rows of H (a row per lane); its wavefronts split
// the m columns (k = w mod SV_NW of each staged block) and their sums are
// added in wavefront order before wavefront 0 writes.
// column-loop unroll: deep for few right-hand sides, shallower where the
// NR accumulators per load already fill the registers
template <int NR>
constexpr int sv_unroll() { return NR >= 8 ? 4 : 16; }

// The column loop is a chain of dependent adds per lane; its loads are
// independent, so it is unrolled deep enough to keep many of them in flight
// (the addition order stays k = w, w + SV_NW, ... whatever the unroll).
template <class T, int NR>
__global__ void __launch_bounds__(WG) k_sv_fwd(const FwTask* __restrict__ ts, const int* __restrict__ wt,
                                               const SvNode* __restrict__ nodes, T* __restrict__ V, int nrhs,
                                               int r0) {
  __shared__ T xb[SV_FKT * NR];
  __shared__ T red[(SV_NW - 1) * SV_RT * NR];
  __shared__ SvNode nl[SV_NODE_LDS];
  const FwTask t = ts[wt[blockIdx.x]];
  const bool nlds = sv_nodes_to_lds(nodes, t.node0, t.nnode, nl);
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int i = ((int)blockIdx.x - t.chunk0) * SV_RT + lane;
  const T* __restrict__ H = static_cast<const T*>(t.H);
  T acc[NR];
  for (int r = 0; r < NR; ++r) acc[r] = 0;
  for (int k0 = 0; k0 < t.m; k0 += SV_FKT) {
    const int kn = min(SV_FKT, t.m - k0);
    __syncthreads();
    for (int e = threadIdx.x; e < kn * NR; e += WG) {
      const int k = e / NR, r = e % NR;
      xb[e] = r0 + r < nrhs ? V[(t.in_pos + k0 + k) * nrhs + r0 + r] : (T)0;
    }
    __syncthreads();
    if (i < t.rows) {
#pragma unroll (sv_unroll<NR>())
      for (int k = w; k < kn; k += SV_NW) {
        const T h = H[i + (int64_t)(k0 + k) * t.ld];
        for (int r = 0; r < NR; ++r) acc[r] += h * xb[k * NR + r];
      }
    }
  }
  if (w > 0)
    for (int r = 0; r < NR; ++r) red[((w - 1) * SV_RT + lane) * NR + r] = acc[r];
  __syncthreads();
  if (w > 0 || i >= t.rows) return;
  for (int v = 0; v < SV_NW - 1; ++v)
    for (int r = 0; r < NR; ++r) acc[r] += red[(v * SV_RT + lane) * NR + r];
  if (i < t.m) {
    for (int r = 0; r < NR; ++r)
      if (r0 + r < nrhs) V[(t.c_pos + i) * nrhs + r0 + r] = acc[r];
    return;
  }
  const int64_t pos = sv_pos_any(nlds, nl, nodes, t.node0, t.nnode, i - t.m);
  for (int r = 0; r < NR; ++r)
    if (r0 + r < nrhs) V[pos * nrhs + r0 + r] -= acc[r];
}

// partial sums of rows rc*SV_RT.. over columns kc*kch..; Part row-major with
// NR. Wavefront w takes the columns k = w (mod SV_NW) of each staged block; the
// wavefronts' sums are added in wavefront order.
// The whole chunk of x (at most SV_KCH columns) is staged at once, so the
// node searches of its columns run side by side, then one unrolled column loop
// (addition order k = kb + w, kb + w + SV_NW, ...).
template <class T, int NR>
__global__ void __launch_bounds__(WG) k_sv_part(const BwTask* __restrict__ ts, const int* __restrict__ wt,
                                                const SvNode* __restrict__ nodes, const T* __restrict__ V, int nrhs,
                                                int r0, T* __restrict__ Part) {
  __shared__ T xb[SV_KCH * NR];
  __shared__ T red[(SV_NW - 1) * SV_RT * NR];
  __shared__ SvNode nl[SV_NODE_LDS];
  const BwTask t = ts[wt[blockIdx.x]];
  const bool nlds = sv_nodes_to_lds(nodes, t.node0, t.nnode, nl);
  __syncthreads();
  const int local = (int)blockIdx.x - t.chunk0;
  const int rc = local % t.nrc, kc = local / t.nrc;
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  const int i = rc * SV_RT + lane;
  const int kb = kc * t.kch, ke = min(t.cols, kb + t.kch);
  const int kn = ke - kb;   // <= t.kch <= SV_KCH
  const T* __restrict__ A = static_cast<const T*>(t.A);
  T acc[NR];
  for (int r = 0; r < NR; ++r) acc[r] = 0;
  for (int k = threadIdx.x; k < kn; k += WG) {
    const int64_t pos = sv_pos_any(nlds, nl, nodes, t.node0, t.nnode, kb + k);
    for (int r = 0; r < NR; ++r) xb[k * NR + r] = r0 + r < nrhs ? V[pos * nrhs + r0 + r] : (T)0;
  }
  __syncthreads();
  if (i < t.rows) {
#pragma unroll (sv_unroll<NR>())
    for (int k = w; k < kn; k += SV_NW) {
      const T a = A[i + (int64_t)(kb + k) * t.ld];
      for (int r = 0; r < NR; ++r) acc[r] += a * xb[k * NR + r];
    }
  }
  if (w > 0)
    for (int r = 0; r < NR; ++r) red[((w - 1) * SV_RT + lane) * NR + r] = acc[r];
  __syncthreads();
  if (w == 0 && i < t.rows) {
    for (int v = 0; v < SV_NW - 1; ++v)
      for (int r = 0; r < NR; ++r) acc[r] += red[(v * SV_RT + lane) * NR + r];
    for (int r = 0; r < NR; ++r) Part[(t.part + (int64_t)kc * t.rows + i) * NR + r] = acc[r];
  }
}

// out = c + alpha * (sum of the partial sums in chunk order)
template <class T, int NR>
__global__ void __launch_bounds__(WG) k_sv_reduce(const BwTask* __restrict__ ts, const int* __restrict__ wt,
                                                  T* __restrict__ V, int nrhs, int r0, const T* __restrict__ Part) {
  const int b = blockIdx.x;
  const BwTask t = ts[wt[b]];
  // the block's WG rows x NR right-hand sides, consecutive threads on consecutive (row, rhs) pairs
  const int i0 = (b - t.chunk0b) * WG;
  for (int e = threadIdx.x; e < WG * NR; e += WG) {
    const int i = i0 + e / NR, r = e % NR;
    if (i >= t.rows || r0 + r >= nrhs) continue;
    T s = 0;
    for (int kc = 0; kc < t.nkc; ++kc) s += Part[(t.part + (int64_t)kc * t.rows + i) * NR + r];
    const T c = t.c_pos >= 0 ? V[(t.c_pos + i) * nrhs + r0 + r] : (T)0;
    V[(t.out_pos + i) * nrhs + r0 + r] = c + (T)t.alpha * s;
  }
}

template <class Ts, class Td>
__global__ void k_sv_perm(const Ts* __restrict__ src, int64_t lds, const int* __restrict__ perm, int64_t n,
                          int nrhs, Td* __restrict__ dst, int64_t ldd, int to_tree) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e >= n * nrhs) return;
  if (to_tree) {   // dst: V rows (row-major over right-hand sides); src: caller order, column-major
    const int64_t t = e / nrhs;
    const int r = (int)(e % nrhs);
    dst[e] = (Td)src[(int64_t)perm[t] + r * lds];
  } else {         // src: V rows; dst: caller order, column-major
    const int64_t t = e % n;
    const int r = (int)(e / n);
    dst[(int64_t)perm[t] + r * ldd] = (Td)src[t * nrhs + r];
  }
}

template <class T>
__global__ void k_sv_zero(T* __restrict__ v, int64_t n) {
  const int64_t e = (int64_t)blockIdx.x * WG + threadIdx.x;
  if (e < n) v[e] = (T)0;
}

template <class T>
struct SolvePlan {
  struct Launch {
    int kind;                 // 0: forward, 1: partial sums + reduction
    int ntasks, nwg, nwg2;
    DevBuf tasks;             // FwTask or BwTask
    DevBuf wt, wt2;           // task of every workgroup (int): of the first kernel, of the reduction
  };
  std::vector<Launch> seq;    // in execution order
  DevBuf nodes;               // SvNode, all launches
  int64_t rows = 0;           // V rows
  int64_t nL = 0;             // rows of the leaf level
  int64_t part_rows = 0;      // largest partial-sum need of one launch
  double factor_elems = 0;    // elements of the stored factors one solve reads
  int64_t launches = 0;
  bool built = false;
  DevBuf V, Part;             // per-call storage (grown on demand)
  // The passes of a solve as replayable HIP graphs, one per right-hand-side
  // count, captured on a stream of their own for the storage (V, Part) they
  // were recorded with; dropped when that storage moves.
  std::map<int, hipGraphExec_t> graphs;
  const void* gV = nullptr;
  const void* gPart = nullptr;
  hipStream_t cap = nullptr;
  void drop_graphs() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    graphs.clear();
  }
  ~SolvePlan() {
    drop_graphs();
    if (cap) (void)hipStreamDestroy(cap);
  }
};

// Task of every workgroup of a backward launch: partial sums (nrc x nkc
// workgroups from chunk0) and reduction (a workgroup per WG rows from chunk0b).
template <class T>
inline void bw_tables(Problem& P, typename SolvePlan<T>::Launch& a, const std::vector<BwTask>& bt) {
  std::vector<int> w((size_t)a.nwg), w2((size_t)a.nwg2);
  for (size_t t = 0; t < bt.size(); ++t) {
    for (int j = 0; j < bt[t].nrc * bt[t].nkc; ++j) w[(size_t)bt[t].chunk0 + j] = (int)t;
    for (int j = 0; j < (int)ceil_div((int64_t)bt[t].rows, WG); ++j) w2[(size_t)bt[t].chunk0b + j] = (int)t;
  }
  P.upload(a.wt, w);
  P.upload(a.wt2, w2);
}

template <class T>
inline SolvePlan<T>& solve_plan(Problem& P, FactorStore<T>& F, SolvePlan<T>& S) {
  if (S.built) return S;
  const int L = P.L;
  // V row bases: level L first, then coarser levels, then the y^(2) rows, then c
  std::vector<int64_t> base(L + 1, 0), M(L + 1, 0);
  for (int l = L; l >= 2; --l) { M[l] = F.sl[l].M; M[l - 1] = F.sl[l].Mup; }
  int64_t r = 0;
  for (int l = L; l >= 1; --l) { base[l] = r; r += M[l]; }
  int64_t cpos = r;
  for (int l = L; l >= 2; --l)
    for (const auto& cf : F.cls[l])
      for (const auto& e : cf.el) cpos += e.m;
  S.rows = cpos;
  S.nL = M[L];
  std::vector<SvNode> nodes;
  std::vector<typename SolvePlan<T>::Launch> fw, bw;
  std::vector<std::vector<BwTask>> bwt;
  int64_t cp = r;
  S.factor_elems = 0;
  S.part_rows = 0;
  auto node_list = [&](const ClassFactors<T>& cf, const ElimDesc& e, int l) {
    const int n0 = (int)nodes.size();
    for (int a = 0; a < e.nF; ++a) {
      const FNode& n = cf.F[e.F0 + a];
      SvNode s{};
      s.pos = n.type == 0 ? base[l] + F.sl[l].xoff[n.box] : base[l - 1] + F.sl[l].yoff[n.box];
      s.off = n.off;
      s.dim = n.dim;
      nodes.push_back(s);
    }
    return n0;
  };
  for (int l = L; l >= 2; --l) {
    for (const auto& cf : F.cls[l]) {
      std::vector<FwTask> ft;
      std::vector<BwTask> bt;
      int wg = 0, wgp = 0, wgr = 0;
      for (const auto& e : cf.el) {
        if (e.m == 0) continue;
        const int n0 = node_list(cf, e, l);
        const T* sol = cf.sol.template as<T>();
        FwTask f{};
        f.H = sol + e.h;
        f.ld = e.m + e.f;
        f.m = e.m;
        f.rows = e.m + e.f;
        f.node0 = n0;
        f.nnode = e.nF;
        f.in_pos = base[l] + F.sl[l].xoff[e.box];
        f.c_pos = cp;
        f.chunk0 = wg;
        wg += (int)ceil_div((int64_t)f.rows, SV_RT);
        ft.push_back(f);
        BwTask b{};
        b.A = sol + e.wx;
        b.ld = e.m;
        b.rows = e.m;
        b.cols = e.f;
        b.node0 = n0;
        b.nnode = e.nF;
        b.out_pos = f.in_pos;
        b.c_pos = cp;
        b.alpha = -1.0;
        b.nrc = (int)ceil_div((int64_t)e.m, SV_RT);
        b.chunk0b = wgr;
        wgr += (int)ceil_div((int64_t)e.m, WG);
        bt.push_back(b);
        cp += e.m;
        S.factor_elems += (double)(e.m + e.f) * e.m + (double)e.m * e.f;
      }
      if (ft.empty()) continue;
      // chunk layout of the backward tasks for a chunk width kch; returns the workgroup count
      auto chunking = [&](std::vector<BwTask>& v, int kch) {
        int64_t pr = 0;
        int nw = 0;
        for (auto& b : v) {
          b.kch = kch;
          b.nkc = std::max(1, (int)ceil_div((int64_t)b.cols, kch));
          b.part = pr;
          pr += (int64_t)b.nkc * b.rows;
          b.chunk0 = nw;
          nw += b.nrc * b.nkc;
        }
        S.part_rows = std::max(S.part_rows, pr);
        return nw;
      };
      // the widest chunk that gives at least SV_MIN_WG workgroups (SV_KT if none does)
      int kch = SV_KCH;
      wgp = chunking(bt, kch);
      while (kch > SV_KT && wgp < SV_MIN_WG) wgp = chunking(bt, kch /= 2);
      typename SolvePlan<T>::Launch a;
      a.kind = 0; a.ntasks = (int)ft.size(); a.nwg = wg; a.nwg2 = 0;
      P.upload(a.tasks, ft);
      {
        std::vector<int> w((size_t)wg);
        for (size_t t = 0; t < ft.size(); ++t)
          for (int j = 0; j < (int)ceil_div((int64_t)ft[t].rows, SV_RT); ++j) w[(size_t)ft[t].chunk0 + j] = (int)t;
        P.upload(a.wt, w);
      }
      fw.push_back(std::move(a));
      typename SolvePlan<T>::Launch b;
      b.kind = 1; b.ntasks = (int)bt.size(); b.nwg = wgp; b.nwg2 = wgr;
      P.upload(b.tasks, bt);
      bw_tables<T>(P, b, bt);
      bw.push_back(std::move(b));
    }
  }
  S.seq.clear();
  for (auto& a : fw) S.seq.push_back(std::move(a));
  if (F.ntop > 0) {
    SvNode s{};
    s.pos = base[1];
    s.off = 0;
    s.dim = F.ntop;
    const int n0 = (int)nodes.size();
    nodes.push_back(s);
    BwTask b{};
    b.A = F.topinv.template as<T>();
    b.ld = F.ntop;
    b.rows = b.cols = F.ntop;
    b.node0 = n0;
    b.nnode = 1;
    b.out_pos = base[1];
    b.c_pos = -1;
    b.alpha = 1.0;
    b.nrc = (int)ceil_div((int64_t)F.ntop, SV_RT);
    b.kch = SV_KCH;
    b.nkc = (int)ceil_div((int64_t)F.ntop, SV_KCH);
    b.part = 0;
    b.chunk0 = 0;
    b.chunk0b = 0;
    typename SolvePlan<T>::Launch a;
    a.kind = 1; a.ntasks = 1; a.nwg = b.nrc * b.nkc; a.nwg2 = (int)ceil_div((int64_t)F.ntop, WG);
    std::vector<BwTask> one(1, b);
    P.upload(a.tasks, one);
    bw_tables<T>(P, a, one);
    S.seq.push_back(std::move(a));
    S.part_rows = std::max(S.part_rows, (int64_t)b.nkc * F.ntop);
    S.factor_elems += (double)F.ntop * F.ntop;
  }
  for (auto it = bw.rbegin(); it != bw.rend(); ++it) S.seq.push_back(std::move(*it));
  P.upload(S.nodes, nodes);
  S.launches = 3;
  for (const auto& a : S.seq) S.launches += a.kind == 0 ? 1 : 2;
  S.built = true;
  return S;
}

template <class T, int NR>
inline void solve_pass(Problem& P, SolvePlan<T>& S, T* V, T* Part, int nrhs, int r0) {
  const SvNode* nodes = S.nodes.template as<SvNode>();
  for (auto& a : S.seq) {
    if (a.kind == 0) {
      hipLaunchKernelGGL((k_sv_fwd<T, NR>), dim3((unsigned)a.nwg), dim3(WG), 0, P.stream,
                         a.tasks.template as<FwTask>(), (const int*)a.wt.template as<int>(), nodes, V, nrhs, r0);
    } else {
      const BwTask* tk = a.tasks.template as<BwTask>();
      hipLaunchKernelGGL((k_sv_part<T, NR>), dim3((unsigned)a.nwg), dim3(WG), 0, P.stream, tk,
                         (const int*)a.wt.template as<int>(), nodes, (const T*)V, nrhs, r0, Part);
      hipLaunchKernelGGL((k_sv_reduce<T, NR>), dim3((unsigned)a.nwg2), dim3(WG), 0, P.stream, tk,
                         (const int*)a.wt2.template as<int>(), V, nrhs, r0, (const T*)Part);
    }
    IFMM_LAUNCH_CHECK();
  }
}

// Elements of the per-call storage of one call: V (S.rows x nrhs) and the
// partial sums (part_rows x the pass width), with the pass width used.
template <class T>
inline int solve_pass_width(int nrhs) {
  constexpr int NRmax = 16;
  const int nr = nrhs >= NRmax ? NRmax : nrhs;
  return nr == 1 ? 1 : nr == 2 ? 2 : nr <= 4 ? 4 : nr <= 8 ? 8 : 16;
}

// The substitution proper, with caller-provided storage V (S.rows * nrhs
// elements) and Part (S.part_rows * solve_pass_width(nrhs) elements). Launches
// only: no allocation, no synchronisation.
// Every pass over the factors (forward, top, backward) for all right-hand sides, on stream st.
template <class T>
inline void solve_passes(Problem& P, SolvePlan<T>& S, T* V, T* Part, int nrhs, hipStream_t st) {
  const hipStream_t keep = P.stream;
  P.stream = st;
  const int nw = solve_pass_width<T>(nrhs);
  for (int r0 = 0; r0 < nrhs; r0 += nw) {
    if (nw == 1) solve_pass<T, 1>(P, S, V, Part, nrhs, r0);
    else if (nw == 2) solve_pass<T, 2>(P, S, V, Part, nrhs, r0);
    else if (nw == 4) solve_pass<T, 4>(P, S, V, Part, nrhs, r0);
    else if (nw == 8) solve_pass<T, 8>(P, S, V, Part, nrhs, r0);
    else solve_pass<T, 16>(P, S, V, Part, nrhs, r0);
  }
  P.stream = keep;
}

// The same as one graph launch on the handle's stream: the hundreds of
// dependent launches of the fine levels are recorded once per right-hand-side
// count and replayed, so the host no longer issues them one by one. The graph
// holds kernel nodes only. IFMM_SOLVE_GRAPH=0 turns replay off.
inline bool solve_graph_on() {
  const char* e = std::getenv("IFMM_SOLVE_GRAPH");
  return !(e && e[0] == '0');
}

template <class T>
inline void solve_passes_graph(Problem& P, SolvePlan<T>& S, T* V, T* Part, int nrhs) {
  if (S.gV != (const void*)V || S.gPart != (const void*)Part) {
    S.drop_graphs();
    S.gV = V;
    S.gPart = Part;
  }
  auto it = S.graphs.find(nrhs);
  if (it == S.graphs.end()) {
    if (!S.cap) IFMM_HIP(hipStreamCreateWithFlags(&S.cap, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    IFMM_HIP(hipStreamBeginCapture(S.cap, hipStreamCaptureModeThreadLocal));
    try {
      solve_passes(P, S, V, Part, nrhs, S.cap);
    } catch (...) {
      (void)hipStreamEndCapture(S.cap, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    IFMM_HIP(hipStreamEndCapture(S.cap, &g));
    hipGraphExec_t ex = nullptr;
    const hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    IFMM_HIP(e);
    it = S.graphs.emplace(nrhs, ex).first;
  }
  IFMM_HIP(hipGraphLaunch(it->second, P.stream));
}

template <class T>
inline void solve_core(Problem& P, SolvePlan<T>& S, const double* b, double* x, int nrhs, int64_t ld, T* V, T* Part,
                       bool graph = false) {
  const int64_t ne = P.n * nrhs;
  hipLaunchKernelGGL((k_sv_perm<double, T>), dim3((unsigned)std::max<int64_t>(1, ceil_div(ne, WG))), dim3(WG), 0,
                     P.stream, b, ld, P.perm.template as<int>(), P.n, nrhs, V, (int64_t)0, 1);
  const int64_t nz = (S.rows - S.nL) * nrhs;
  if (nz > 0)
    hipLaunchKernelGGL(k_sv_zero<T>, dim3((unsigned)ceil_div(nz, WG)), dim3(WG), 0, P.stream, V + S.nL * nrhs, nz);
  IFMM_LAUNCH_CHECK();
  if (graph) solve_passes_graph(P, S, V, Part, nrhs);
  else solve_passes(P, S, V, Part, nrhs, P.stream);
  hipLaunchKernelGGL((k_sv_perm<T, double>), dim3((unsigned)std::max<int64_t>(1, ceil_div(ne, WG))), dim3(WG), 0,
                     P.stream, (const T*)V, (int64_t)0, P.perm.template as<int>(), P.n, nrhs, x, ld, 0);
  IFMM_LAUNCH_CHECK();
}

// x = IFMM^-1 b, b and x in caller order (float64, column-major, ld), nrhs
// columns; per-call storage held by the plan (grown on demand).
template <class T>
inline void solve_impl(Problem& P, FactorStore<T>& F, SolvePlan<T>& S, const double* b, double* x, int nrhs,
                       int64_t ld) {
  solve_plan(P, F, S);
  S.V.reserve(sizeof(T) * (size_t)std::max<int64_t>(S.rows * nrhs, 1), &P.mem);
  S.Part.reserve(sizeof(T) * (size_t)std::max<int64_t>(S.part_rows * solve_pass_width<T>(nrhs), 1), &P.mem);
  P.kset(KF_SOLVE, 2.0 * S.factor_elems * nrhs, S.factor_elems * sizeof(T));
  P.kbegin();
  solve_core(P, S, b, x, nrhs, ld, S.V.template as<T>(), S.Part.template as<T>(), solve_graph_on());
  P.kend();
  P.kset(-1);
}

}  // namespace ifmm
