// Common infrastructure of the IFMM library: error handling, device memory
// accounting, small host/device helpers.
#pragma once

#include <atomic>
#include <mutex>
#include <map>

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/ifmm.h"

namespace ifmm {

// Failure carried to the C ABI boundary, where it becomes an ifmm_status.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(int code, const std::string& msg) { throw Error(code, msg); }

#define IFMM_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      ::ifmm::fail(e_ == hipErrorOutOfMemory ? IFMM_ERR_OOM : IFMM_ERR_HIP,              \
                   std::string(#call) + ": " + hipGetErrorString(e_) + " at " __FILE__); \
  } while (0)

#define IFMM_CHECK(cond, msg) \
  do {                        \
    if (!(cond)) ::ifmm::fail(IFMM_ERR_INTERNAL, std::string("check failed: ") + (msg)); \
  } while (0)

#define IFMM_LAUNCH_CHECK() IFMM_HIP(hipGetLastError())

// Device memory owned by one handle, with a running total and an optional budget.
struct MemAccount {
  int64_t cur = 0, peak = 0, budget = 0;
  void add(int64_t b) {
    if (budget > 0 && cur + b > budget)
      fail(IFMM_ERR_OOM, "device memory budget exceeded (" + std::to_string(cur + b) + " > " +
                             std::to_string(budget) + " bytes)");
    cur += b;
    if (cur > peak) peak = cur;
  }
  void sub(int64_t b) { cur -= b; }
};

// Host time spent in hipMalloc / hipFree, process totals (diagnostics).
struct AllocClock {
  static inline std::atomic<int64_t> ns_malloc{0}, ns_free{0}, calls{0};
  static int64_t now_ns() {
    return std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
  }
};

// Stream of the API call running on this thread (set by StreamScope at every
// entry point that touches a handle); device blocks freed under it are kept for
// reuse on that stream only.
inline hipStream_t& tls_stream() {
  static thread_local hipStream_t s = nullptr;
  return s;
}
struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(tls_stream()) { tls_stream() = s; }
  ~StreamScope() { tls_stream() = prev; }
};

// Device allocator of the handle whose API call runs on this thread (set by
// AllocScope next to StreamScope); null functions: the library's own pool.
struct DevAlloc {
  void* (*alloc)(size_t, void*) = nullptr;
  void (*free)(void*, size_t, void*) = nullptr;
  void* ctx = nullptr;
};
inline DevAlloc& tls_alloc() {
  static thread_local DevAlloc a;
  return a;
}
struct AllocScope {
  DevAlloc prev;
  explicit AllocScope(const DevAlloc& a) : prev(tls_alloc()) { tls_alloc() = a; }
  ~AllocScope() { tls_alloc() = prev; }
};

// Process-wide cache of device blocks. hipMalloc / hipFree cost about 0.1 ms
// each and serialise host threads, so a build + factorization (hundreds of
// buffers) and batches of problems would spend much of their time there.
// Sizes are rounded to 8 classes per power of two. A freed block is reused
// only by work on the stream that freed it (stream order makes that safe), or
// by any stream once that stream has been synchronised (idle(), called when a
// handle is destroyed). Cached bytes beyond CAP go back to HIP; a failed
// hipMalloc returns every cached block (hipFree waits for the device) and
// tries again.
class DevPool {
 public:
  static DevPool& inst() {
    static DevPool* p = new DevPool();   // never destroyed: blocks outlive static destructors
    return *p;
  }
  static size_t cls(size_t b) {
    if (b <= 4096) return (b + 255) & ~(size_t)255;
    int e = 63 - __builtin_clzll((unsigned long long)b);
    const size_t step = (size_t)1 << (e - 3);
    return (b + step - 1) & ~(step - 1);
  }
  void* get(size_t b, hipStream_t s) {
    const size_t c = cls(b);
    {
      std::lock_guard<std::mutex> g(mu_);
      for (void* tag : {(void*)s, idle_tag()}) {
        auto it = free_.find({tag, c});
        if (it != free_.end() && !it->second.empty()) {
          void* p = it->second.back();
          it->second.pop_back();
          cached_ -= c;
          return p;
        }
      }
    }
    void* p = nullptr;
    const int64_t t0 = AllocClock::now_ns();
    hipError_t e = hipMalloc(&p, c);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      flush();
      e = hipMalloc(&p, c);
    }
    AllocClock::ns_malloc += AllocClock::now_ns() - t0;
    ++AllocClock::calls;
    if (e != hipSuccess) {
      (void)hipGetLastError();
      fail(IFMM_ERR_OOM, "hipMalloc(" + std::to_string(c) + ") failed: " + hipGetErrorString(e));
    }
    return p;
  }
  void put(void* p, size_t b, hipStream_t s) {
    const size_t c = cls(b);
    {
      std::lock_guard<std::mutex> g(mu_);
      if (cached_ + c <= CAP) {
        free_[{(void*)s, c}].push_back(p);
        cached_ += c;
        return;
      }
    }
    const int64_t t0 = AllocClock::now_ns();
    (void)hipFree(p);
    AllocClock::ns_free += AllocClock::now_ns() - t0;
  }
  // tag of blocks that any stream may reuse (freed after a synchronisation)
  static hipStream_t idle_stream() { return reinterpret_cast<hipStream_t>(idle_tag()); }
  // stream s has been synchronised: its cached blocks may serve any stream
  void idle(hipStream_t s) {
    std::lock_guard<std::mutex> g(mu_);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->first.first != (void*)s || it->second.empty()) continue;
      auto& dst = free_[{idle_tag(), it->first.second}];
      dst.insert(dst.end(), it->second.begin(), it->second.end());
      it->second.clear();
    }
  }
  void flush() {
    std::map<std::pair<void*, size_t>, std::vector<void*>> all;
    {
      std::lock_guard<std::mutex> g(mu_);
      all.swap(free_);
      cached_ = 0;
    }
    for (auto& kv : all)
      for (void* p : kv.second) (void)hipFree(p);
  }

 private:
  static constexpr size_t CAP = (size_t)96 << 30;
  static void* idle_tag() { return reinterpret_cast<void*>(1); }
  std::mutex mu_;
  std::map<std::pair<void*, size_t>, std::vector<void*>> free_;
  size_t cached_ = 0;
};

// An owning device buffer. Moves only.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  MemAccount* acct = nullptr;
  DevAlloc from;   // the caller's allocator that gave p (null functions: the pool)
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept { *this = std::move(o); }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p; bytes = o.bytes; acct = o.acct; from = o.from;
      o.p = nullptr; o.bytes = 0; o.acct = nullptr; o.from = DevAlloc();
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b, MemAccount* a) {
    release();
    if (b == 0) b = 256;
    if (a) a->add((int64_t)b);
    const DevAlloc& ca = tls_alloc();
    if (ca.alloc && ca.free) {
      p = ca.alloc(b, ca.ctx);
      if (!p || (reinterpret_cast<uintptr_t>(p) & 255)) {
        if (p) ca.free(p, b, ca.ctx);
        p = nullptr;
        if (a) a->sub((int64_t)b);
        fail(IFMM_ERR_OOM, "the caller's dev_alloc(" + std::to_string(b) + ") gave no 256-byte aligned block");
      }
      from = ca;
    } else {
      try {
        p = DevPool::inst().get(b, tls_stream());
      } catch (...) {
        if (a) a->sub((int64_t)b);
        p = nullptr;
        throw;
      }
      from = DevAlloc();
    }
    bytes = b;
    acct = a;
  }
  void release() {
    if (p) {
      if (from.free) from.free(p, bytes, from.ctx);
      else DevPool::inst().put(p, bytes, tls_stream());
      if (acct) acct->sub((int64_t)bytes);
    }
    p = nullptr;
    bytes = 0;
    acct = nullptr;
    from = DevAlloc();
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
  // Grow (never shrink) to at least b bytes; contents are not kept.
  void reserve(size_t b, MemAccount* a) {
    if (b > bytes) alloc(b + b / 4, a);
  }
};

// Upload a host vector into a device buffer (grow as needed), asynchronously
// from a pinned staging copy owned by the caller's Staging object.
struct Staging {
  void* h = nullptr;
  size_t bytes = 0;
  ~Staging() { if (h) (void)hipHostFree(h); }
  void* get(size_t b) {
    if (b > bytes) {
      if (h) (void)hipHostFree(h);
      size_t nb = b + b / 2 + 4096;
      IFMM_HIP(hipHostMalloc(&h, nb, hipHostMallocDefault));
      bytes = nb;
    }
    return h;
  }
};

inline double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

template <class T> struct Prec;
template <> struct Prec<double> { static constexpr double u = 1.1102230246251565e-16; };
template <> struct Prec<float> { static constexpr double u = 5.9604644775390625e-08; };

}  // namespace ifmm
