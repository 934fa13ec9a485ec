// State of one IFMM handle: tree, R1 operators (matvec), the weighted and
// truncated initial operators of E (R2, float64), the factors, timers.
#pragma once

#include <chrono>
#include <memory>

#include "h2.hpp"

namespace ifmm {

// Device copies of one level's tables.
struct LevelDev {
  int nb = 0;
  DevBuf coords, nb_start, nbr, in_start, inter, parent, ch_start, cbits, in_rev;
  int64_t npairs = 0;   // size of the interaction-list CSR
  // M2L by offset tiles: boxes ordered by child position (tord), the
  // interaction pair at every offset of each box (bo, -1: none), group starts
  DevBuf m2l_tord, m2l_bo;
  std::vector<int> m2l_tord_h;
  std::vector<int> m2l_gstart;
};

// Initial operators of one level after QR, weighting and truncation (float64).
//   K   y_i row, y_j column, one block per interaction-list pair (k_i x k_j, ld k_i)
//   PU  y_i row, z_parent column (k_i x k_parent, ld k_i);  PV likewise
//   SU, SV weights (k_i)
//   leaf only: U, V (m_i x k_i, ld m_i)
struct R2Level {
  std::vector<int> k;
  std::vector<int64_t> k_off;      // per pair (CSR-aligned)
  std::vector<int64_t> p_off;      // per box (PU / PV)
  std::vector<int64_t> s_off;      // per box (SU / SV)
  std::vector<int64_t> u_off;      // leaf: per box (U / V)
  DevBuf K, PU, PV, SU, SV, U, V;
};

struct FactorLevelBase;   // defined in factor.hpp (templated on precision)
struct FactorStoreBase {
  virtual ~FactorStoreBase() = default;
};

// Kernel-family timing with HIP events on the handle's stream (enabled by
// IFMM_KTIMING=1, or IFMM_KTIMING=m<hex mask> for the families of the mask
// only): duration, launch count and algorithmic flops / bytes.
// Families 0-8 group the launches of one phase; families 9-14 hold exactly
// one kernel each, every launch timed on its own (per-launch averages);
// family 15 holds the launches of the step-wise pivoted QR; families 16 and
// 17 hold one kernel each again (streaming R-only QR, K_pre products).
enum KFam {
  KF_SCHUR = 0, KF_LU, KF_TRSM, KF_QR, KF_SVD, KF_XFORM, KF_SOLVE, KF_MATVEC, KF_OTHER,
  KF_SVD_ROUND, KF_QR_PANEL, KF_QRCP, KF_SVD_SMALL, KF_ROW_XFORM, KF_COL_XFORM, KF_QRCP_STEP, KF_QR_NARROW,
  KF_KPRE, KF_COUNT
};
static_assert(KF_COUNT <= 24, "the query structure holds 24 families");

// Host wall time by section (diagnostics, IFMM_HOSTPROF=1): where the host
// spends the factorization, waiting on the device included.
struct HostProf {
  static bool on() {
    static const bool v = std::getenv("IFMM_HOSTPROF") != nullptr;
    return v;
  }
  std::vector<std::pair<const char*, double>> acc;
  void add(const char* name, double ms) {
    for (auto& x : acc)
      if (x.first == name) { x.second += ms; return; }
    acc.push_back({name, ms});
  }
  void print(const char* tag) const {
    for (const auto& x : acc) std::fprintf(stderr, "[ifmm-hostprof] %s %-28s %9.2f ms\n", tag, x.first, x.second);
  }
};
struct HostScope {
  HostProf* hp;
  const char* name;
  double t0;
  HostScope(HostProf& h, const char* n) : hp(HostProf::on() ? &h : nullptr), name(n), t0(hp ? now_ms() : 0) {}
  void stop() {
    if (hp) hp->add(name, now_ms() - t0);
    hp = nullptr;
  }
  ~HostScope() { stop(); }
};

struct KTimer {
  bool on = false;
  uint32_t mask = ~0u;        // families that are timed
  bool last_on = false;       // whether the open range was recorded
  struct Rec { int fam; hipEvent_t a, b; double flops, bytes; int64_t launches; bool closed; };
  std::vector<Rec> open;
  std::vector<hipEvent_t> pool;   // events of collected records, reused
  double ms[KF_COUNT] = {}, flops[KF_COUNT] = {}, bytes[KF_COUNT] = {};
  int64_t launches[KF_COUNT] = {};
  ~KTimer() {
    for (auto& r : open) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
    for (auto e : pool) (void)hipEventDestroy(e);
  }
  hipEvent_t event() {
    hipEvent_t e;
    if (!pool.empty()) { e = pool.back(); pool.pop_back(); return e; }
    IFMM_HIP(hipEventCreate(&e));
    return e;
  }
  void begin(hipStream_t s, int fam, double fl, double by, int64_t nl = 1) {
    last_on = on && ((mask >> fam) & 1u);
    if (!last_on) return;
    Rec r{fam, event(), event(), fl, by, nl, false};
    IFMM_HIP(hipEventRecord(r.a, s));
    open.push_back(r);
  }
  void end(hipStream_t s) {
    if (!last_on || open.empty()) return;
    last_on = false;
    IFMM_HIP(hipEventRecord(open.back().b, s));
    open.back().closed = true;
  }
  // Fold completed records into the totals (call after a stream sync).
  void collect() {
    for (auto& r : open) {
      float t = 0;
      if (!r.closed) {   // a range left open is dropped (never queried: that would raise a HIP error)
        pool.push_back(r.a);
        pool.push_back(r.b);
        continue;
      }
      if (hipEventElapsedTime(&t, r.a, r.b) == hipSuccess) {
        ms[r.fam] += t;
        flops[r.fam] += r.flops;
        bytes[r.fam] += r.bytes;
        launches[r.fam] += r.launches;
      } else {
        (void)hipGetLastError();   // not left for the caller's next HIP call to report
      }
      pool.push_back(r.a);
      pool.push_back(r.b);
    }
    open.clear();
  }
  void reset() {
    collect();
    for (int i = 0; i < KF_COUNT; ++i) { ms[i] = flops[i] = bytes[i] = 0; launches[i] = 0; }
  }
};

struct Problem {
  KTimer kt;
  int kcur = -1;              // family charged by the next launches (-1: none)
  double kfl = 0, kby = 0;    // algorithmic flops / bytes still to attribute
  void kset(int fam, double fl = 0, double by = 0) { kcur = fam; kfl = fl; kby = by; }
  void kbegin() {
    if (kt.on && kcur >= 0) { kt.begin(stream, kcur, kfl, kby); kfl = kby = 0; }
  }
  void kend() {
    if (kt.on && kcur >= 0) kt.end(stream);
  }
  // One launch timed on its own in a single-kernel family (not nested in an
  // open kbegin / kend range).
  void kone_begin(int fam, double fl, double by = 0) {
    if (kt.on) kt.begin(stream, fam, fl, by);
  }
  void kone_end() {
    if (kt.on) kt.end(stream);
  }
  // configuration
  int64_t n = 0;
  int d = 0, L = 0, order = 0, q = 0, precision = 64;
  double eps = 0, sigma0 = 0, tau = 0;
  int rank_max = 0;
  KernelFn kf{};
  ChebConst cc{};
  hipStream_t stream = nullptr;
  DevAlloc alloc;                  // the caller's device allocator (null functions: the pool)
  int device = 0;                  // HIP device current at the build
  MemAccount mem;
  Staging stage;
  HostProf hprof;
  bool factorized = false;

  // tree
  HTree T;
  std::vector<LevelDev> ldev;      // by level
  DevBuf pts;                      // tree-ordered points (n x d)
  DevBuf perm;                     // int32: tree position -> caller index
  DevBuf leaf_start;               // int64 (nb_L + 1)

  // R1
  DevBuf ubar;                     // leaf interpolation, per leaf at leaf_start * q
  DevBuf Ttab;                     // 2^d transfers (q x q)
  std::vector<DevBuf> m2l;         // by level: 7^d tables of q x q
  DevBuf m2l_ocode;                // per child position: the codes of its interaction offsets
  DevBuf nf, nfoff, nfcol;         // stored leaf near-field blocks (empty: evaluated in every product)
  int m2l_nofs = 0;                // interaction offsets of a child position: 6^d - 3^d
  std::vector<DevBuf> mv_w, mv_g;  // matvec scratch by level
  int mv_nrhs = 0;
  DevBuf mv_x, mv_y;

  // R2 (float64 initial operators of E)
  std::vector<R2Level> r2;
  double sigma0_estimated = 0;
  int sigma0_iters = 0;

  // factors (precision-specific)
  std::unique_ptr<FactorStoreBase> fac;

  // statistics
  ifmm_stats st{};
  int trace_level = 0;             // level being factorized (IFMM_TRACE output)
  DevBuf trace_buf;
  DevBuf svd_state;                // block-Jacobi SVD: scales and convergence flags
  int* d_info = nullptr;           // device error word (first failing tag)
  DevBuf info_buf;

  void sync() { IFMM_HIP(hipStreamSynchronize(stream)); }

  // The buffer is kept when it is large enough, so a re-upload of a table
  // does not move it: device views taken earlier (LevelView) stay valid.
  template <class T>
  void upload(DevBuf& b, const std::vector<T>& v) {
    const size_t need = v.size() * sizeof(T) + 16;
    if (!b.p || b.bytes < need) b.alloc(need, &mem);
    if (!v.empty()) {
      void* h = stage.get(v.size() * sizeof(T));
      std::memcpy(h, v.data(), v.size() * sizeof(T));
      IFMM_HIP(hipMemcpyAsync(b.p, h, v.size() * sizeof(T), hipMemcpyHostToDevice, stream));
      sync();   // the staging buffer is reused by the next upload
    }
  }
  template <class T>
  void download(std::vector<T>& v, const void* src, size_t count) {
    v.resize(count);
    if (!count) return;
    void* h = stage.get(count * sizeof(T));
    IFMM_HIP(hipMemcpyAsync(h, src, count * sizeof(T), hipMemcpyDeviceToHost, stream));
    sync();
    std::memcpy(v.data(), h, count * sizeof(T));
  }
  // Descriptor arena: launch descriptors are appended to pinned host chunks
  // and copied to matching device chunks on the stream, with no
  // synchronisation. A descriptor stays valid until arena_reset(), which the
  // factorization calls where the stream is idle anyway (start of a colour
  // class, of a merge, of the top system, of every API call).
  struct ArenaChunk {
    DevBuf dev;
    void* host = nullptr;
    size_t bytes = 0;
  };
  std::vector<ArenaChunk> arena;
  size_t arena_cur = 0, arena_off = 0;
  void arena_reset() {
    sync();
    arena_cur = 0;
    arena_off = 0;
  }
  template <class D>
  const D* put(DevBuf& unused, const std::vector<D>& v) {
    (void)unused;
    const size_t bytes = (v.size() * sizeof(D) + 255) & ~size_t(255);
    if (arena.empty() || arena_off + bytes > arena[arena_cur].bytes) {
      if (!arena.empty() && arena_off > 0) { ++arena_cur; arena_off = 0; }
      while (arena_cur < arena.size() && arena[arena_cur].bytes < bytes) ++arena_cur;
      if (arena_cur >= arena.size()) {
        ArenaChunk c;
        c.bytes = std::max<size_t>(bytes, size_t(8) << 20);
        c.dev.alloc(c.bytes, &mem);
        IFMM_HIP(hipHostMalloc(&c.host, c.bytes, hipHostMallocDefault));
        arena.push_back(std::move(c));
        arena_cur = arena.size() - 1;
      }
    }
    ArenaChunk& c = arena[arena_cur];
    char* h = static_cast<char*>(c.host) + arena_off;
    char* d = static_cast<char*>(c.dev.p) + arena_off;
    if (!v.empty()) {
      std::memcpy(h, v.data(), v.size() * sizeof(D));
      IFMM_HIP(hipMemcpyAsync(d, h, v.size() * sizeof(D), hipMemcpyHostToDevice, stream));
    }
    arena_off += bytes;
    return reinterpret_cast<const D*>(d);
  }
  ~Problem() {
    if (stream) (void)hipStreamSynchronize(stream);
    for (auto& c : arena)
      if (c.host) (void)hipHostFree(c.host);
  }
};

// Diagnostics (IFMM_DEBUG=1 in the environment): norm and first values of a
// device array, printed to stderr.
inline bool debug_on() {
  static const bool on = std::getenv("IFMM_DEBUG") != nullptr;
  return on;
}

// Progress lines on stderr (IFMM_PROGRESS set in the environment): one per
// phase of the build and per eliminated level, with the time since the call
// began and the handle's device memory.
inline int progress_level() {
  const char* e = std::getenv("IFMM_PROGRESS");
  return e ? std::max(1, std::atoi(e)) : 0;
}
inline bool progress_on() { return progress_level() > 0; }

// Test switch (IFMM_FORCE_STREAMED set in the environment): the dense kernels
// take the variants meant for large blocks on every size: LU panels streamed
// from memory instead of LDS, the block-Jacobi SVD, the one-workgroup pivoted
// QR and the redirect by batched products. Results agree with the default
// variants to rounding; tests use it to compare those variants with the
// oracle at sizes the oracle runs.
inline bool force_streamed() { return std::getenv("IFMM_FORCE_STREAMED") != nullptr; }

// Per-launch trace of the dense batched kernels (IFMM_TRACE=1): synchronises
// after each launch and prints sizes and duration to stderr.
inline bool trace_on() {
  static const bool on = std::getenv("IFMM_TRACE") != nullptr;
  return on;
}

// IFMM_QR_STATS=1: one line per batched QR launch with the job shapes
inline bool qr_stats_on() {
  static const bool on = std::getenv("IFMM_QR_STATS") != nullptr;
  return on;
}

template <class T>
inline void dbg_dump(Problem& P, const char* name, const void* d, size_t count, size_t show = 6) {
  if (!debug_on() || count == 0) return;
  std::vector<T> h;
  P.download(h, d, count);
  double s = 0;
  size_t nonfinite = 0;
  for (auto v : h) {
    if (!std::isfinite((double)v)) ++nonfinite;
    else s += (double)v * (double)v;
  }
  std::fprintf(stderr, "[ifmm] %s n=%zu norm=%.6e nonfinite=%zu :", name, count, std::sqrt(s), nonfinite);
  for (size_t i = 0; i < count && i < show; ++i) std::fprintf(stderr, " %.6e", (double)h[i]);
  std::fprintf(stderr, "\n");
}

// ------------------------------------------------------------ batched launchers
template <class T>
inline void run_gemm(Problem& P, GemmBatch& gb, DevBuf& scratch) {
  if (gb.v.empty()) return;
  const GemmDesc* d = P.put(scratch, gb.v);
  P.kbegin();
  hipLaunchKernelGGL(k_gemm<T>, dim3(gb.tiles), dim3(WG), 0, P.stream, d, (int)gb.v.size());
  IFMM_LAUNCH_CHECK();
  P.kend();
}

template <class Ts, class Td>
inline void run_copy(Problem& P, CopyBatch<Ts, Td>& cb, DevBuf& scratch) {
  if (cb.v.empty()) return;
  const CopyDesc<Ts, Td>* d = P.put(scratch, cb.v);
  hipLaunchKernelGGL((k_copy<Ts, Td>), dim3((unsigned)cb.v.size()), dim3(WG), 0, P.stream, d,
                     (int)cb.v.size());
  IFMM_LAUNCH_CHECK();
}

template <class T>
inline void run_qr(Problem& P, const std::vector<QrDesc>& v, DevBuf& scratch) {
  if (v.empty()) return;
  const QrDesc* d = P.put(scratch, v);
  P.kbegin();
  hipLaunchKernelGGL(k_qr<T>, dim3((unsigned)v.size()), dim3(WG), 0, P.stream, d);
  IFMM_LAUNCH_CHECK();
  P.kend();
}

template <class T>
inline void run_lu(Problem& P, const std::vector<LuDesc>& v, DevBuf& scratch) {
  if (v.empty()) return;
  const LuDesc* d = P.put(scratch, v);
  hipLaunchKernelGGL(k_lu<T>, dim3((unsigned)v.size()), dim3(WG), 0, P.stream, d, P.d_info);
  IFMM_LAUNCH_CHECK();
}

template <class T>
inline void run_lu_solve(Problem& P, LuSolveBatch& b, DevBuf& scratch) {
  if (b.v.empty()) return;
  const LuSolveDesc* d = P.put(scratch, b.v);
  hipLaunchKernelGGL(k_lu_solve<T>, dim3(b.blocks), dim3(WG), 0, P.stream, d, (int)b.v.size());
  IFMM_LAUNCH_CHECK();
}

}  // namespace ifmm
