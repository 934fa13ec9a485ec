// Allocation-free variant of the solve (ifmm_solve_noalloc in include/ifmm.h)
// for callers that cannot allocate device memory. Its work vectors live in one
// fixed device array per GPU instead of buffers of the handle. The array is
// shared by every call on that GPU and keeps the last call's contents; the
// substitution writes every element it later reads (the leaf rows from b, the
// other rows of V zeroed, each partial sum before its reduction), so nothing
// needs clearing between calls. Calls that overlap on one GPU race on it.
#pragma once

namespace {

// Device storage of ifmm_solve_noalloc: one fixed array per GPU, holding the
// work vector V and the partial sums of one call. Host code never uses the
// array's name as an address: the device address comes from
// hipGetSymbolAddress, taken once per device at the first build on it.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];

std::mutex g_scratch_mu;
std::map<int, void*> g_scratch_addr;   // device -> address of its scratch array

// With `device` current: the address of that device's scratch array.
void* scratch_address(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  if (it != g_scratch_addr.end()) return it->second;
  void* ptr = nullptr;
  IFMM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) fail(IFMM_ERR_HIP, "no device address for the solve scratch array");
  g_scratch_addr[device] = ptr;
  return ptr;
}

// The address recorded for `device` (nullptr if no build ran on it).
void* scratch_lookup(int device) {
  std::lock_guard<std::mutex> g(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  return it == g_scratch_addr.end() ? nullptr : it->second;
}

template <class T>
void solve_noalloc_impl(Problem& P, SolvePlan<T>& S, const double* b, double* x, int nrhs, int64_t ld) {
  if (!S.built) fail(IFMM_ERR_STATE, "the solve plan of the factorization is missing");
  const size_t vbytes = ((sizeof(T) * (size_t)S.rows * nrhs) + 255) & ~size_t(255);
  const size_t need = vbytes + sizeof(T) * (size_t)S.part_rows * solve_pass_width<T>(nrhs);
  if (need > NOALLOC_SCRATCH_BYTES)
    fail(IFMM_ERR_ARG, "ifmm_solve_noalloc needs " + std::to_string(need) + " bytes of scratch for nrhs = " +
                           std::to_string(nrhs) + " (limit " + std::to_string(NOALLOC_SCRATCH_BYTES) + ")");
  char* base = static_cast<char*>(scratch_lookup(P.device));
  if (!base) fail(IFMM_ERR_STATE, "no scratch address for the handle's device");
  solve_core(P, S, b, x, nrhs, ld, reinterpret_cast<T*>(base), reinterpret_cast<T*>(base + vbytes));
}

}  // namespace

extern "C" int ifmm_solve_noalloc(ifmm_handle h, const double* b, double* x, int nrhs, int64_t ld) {
  return guarded([&] {
    if (!h || !b || !x) fail(IFMM_ERR_ARG, "null pointer");
    Problem& P = h->P;
    if (!P.factorized) fail(IFMM_ERR_STATE, "ifmm_solve_noalloc needs a factorized handle");
    if (nrhs < 1 || ld < P.n) fail(IFMM_ERR_ARG, "nrhs must be >= 1 and ld >= n");
    if (P.precision == 64) {
      auto* f = static_cast<Factors<double>*>(P.fac.get());
      solve_noalloc_impl<double>(P, f->S, b, x, nrhs, ld);
    } else {
      auto* f = static_cast<Factors<float>*>(P.fac.get());
      solve_noalloc_impl<float>(P, f->S, b, x, nrhs, ld);
    }
  });
}

