// Stable least-significant-digit radix sort of (64-bit key, int payload)
// pairs on the low `bits` bits of the keys: the Morton order of the points
// (Sec. 2.1: boxes of the tree are contiguous ranges of the sorted points).
//
// Per pass (8-bit digit):
//  1. k_rs_hist: each workgroup counts the digits of its tile of RS_TILE keys
//     (LDS histogram) into cnt[digit * ntiles + tile];
//  2. k_rs_scan: one workgroup turns cnt into exclusive offsets in
//     (digit, tile) order, so a tile's keys of one digit go after those of
//     every earlier tile;
//  3. k_rs_scatter: each workgroup walks its tile in index order, RS_WG keys
//     at a time, and ranks every key among the earlier keys of its digit
//     (wavefront ballots, then per-wavefront counts in LDS). Equal digits
//     keep their order, so the sort is stable.
// No library call; keys/payloads ping-pong between the in and out buffers,
// the result lands in the out buffers.
#pragma once

#include "common.hpp"
#include "linalg.hpp"

namespace ifmm {

constexpr int RS_BITS = 8;
constexpr int RS_BINS = 1 << RS_BITS;
constexpr int RS_WG = 256;                 // threads of the histogram and scatter kernels
constexpr int RS_ITEMS = 16;               // keys per thread of a tile
constexpr int RS_TILE = RS_WG * RS_ITEMS;  // keys of one workgroup
constexpr int RS_WAVES = RS_WG / WAVE;
constexpr int RS_SCAN_WG = 1024;

static_assert(RS_BINS == RS_WG, "one histogram bin per thread");

__global__ void __launch_bounds__(RS_WG) k_rs_hist(const uint64_t* __restrict__ keys, int64_t n, int shift,
                                                   int ntiles, int* __restrict__ cnt) {
  __shared__ int h[RS_BINS];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  for (int j = 0; j < RS_ITEMS; ++j) {
    const int64_t i = base + (int64_t)j * RS_WG + threadIdx.x;
    if (i < n) atomicAdd(&h[(int)((keys[i] >> shift) & (RS_BINS - 1))], 1);
  }
  __syncthreads();
  cnt[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan of m = RS_BINS * ntiles counts in place: thread t scans a
// contiguous segment, the segment totals are scanned in LDS, then every
// segment is rewritten with its offset.
__global__ void __launch_bounds__(RS_SCAN_WG) k_rs_scan(int* __restrict__ cnt, int64_t m) {
  __shared__ int64_t tot[RS_SCAN_WG];
  const int64_t seg = (m + RS_SCAN_WG - 1) / RS_SCAN_WG;
  const int64_t a = (int64_t)threadIdx.x * seg, b = a + seg < m ? a + seg : m;
  int64_t s = 0;
  for (int64_t i = a; i < b; ++i) s += cnt[i];
  tot[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int t = 0; t < RS_SCAN_WG; ++t) {
      const int64_t v = tot[t];
      tot[t] = run;
      run += v;
    }
  }
  __syncthreads();
  int64_t run = tot[threadIdx.x];
  for (int64_t i = a; i < b; ++i) {
    const int v = cnt[i];
    cnt[i] = (int)run;
    run += v;
  }
}

__global__ void __launch_bounds__(RS_WG) k_rs_scatter(const uint64_t* __restrict__ kin, const int* __restrict__ vin,
                                                      int64_t n, int shift, int ntiles, const int* __restrict__ off,
                                                      uint64_t* __restrict__ kout, int* __restrict__ vout) {
  __shared__ int run[RS_BINS];               // keys of each digit placed by earlier steps of this tile
  __shared__ int wc[RS_WAVES][RS_BINS];      // keys of each digit in each wavefront of this step
  const int lane = threadIdx.x % WAVE, w = threadIdx.x / WAVE;
  run[threadIdx.x] = off[(int64_t)threadIdx.x * ntiles + blockIdx.x];
  for (int v = 0; v < RS_WAVES; ++v) wc[v][threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * RS_TILE;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (WAVE - lane));
  for (int j = 0; j < RS_ITEMS; ++j) {
    const int64_t i = base + (int64_t)j * RS_WG + threadIdx.x;   // index order = (step, thread)
    const bool ok = i < n;
    const uint64_t key = ok ? kin[i] : 0;
    const int dg = (int)((key >> shift) & (RS_BINS - 1));
    // lanes of this wavefront holding a key with the same digit
    uint64_t peers = __ballot(ok);
    for (int bt = 0; bt < RS_BITS; ++bt) {
      const uint64_t on = __ballot(ok && ((dg >> bt) & 1));
      peers &= ((dg >> bt) & 1) ? on : ~on;
    }
    const int rank = __popcll(peers & below);
    if (ok && rank == 0) wc[w][dg] = __popcll(peers);   // the first lane of the group counts it
    __syncthreads();
    if (ok) {
      int pos = run[dg] + rank;
      for (int v = 0; v < w; ++v) pos += wc[v][dg];
      kout[pos] = key;
      vout[pos] = vin[i];
    }
    __syncthreads();
    int add = 0;
    for (int v = 0; v < RS_WAVES; ++v) {
      add += wc[v][threadIdx.x];
      wc[v][threadIdx.x] = 0;
    }
    run[threadIdx.x] += add;
    __syncthreads();
  }
}

// Sorts (keys, vals) of length n by the low `bits` bits of the keys, stably.
// kin/vin are clobbered; the sorted pairs are left in kout/vout. cnt must hold
// RS_BINS * ceil(n / RS_TILE) ints.
inline void radix_sort_pairs(hipStream_t st, uint64_t* kin, int* vin, uint64_t* kout, int* vout, int64_t n, int bits,
                             int* cnt) {
  if (n <= 0) return;
  const int ntiles = (int)((n + RS_TILE - 1) / RS_TILE);
  const int passes = bits <= 0 ? 1 : (bits + RS_BITS - 1) / RS_BITS;
  uint64_t* ka = kin;
  int* va = vin;
  uint64_t* kb = kout;
  int* vb = vout;
  for (int p = 0; p < passes; ++p) {
    const int shift = p * RS_BITS;
    hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(RS_WG), 0, st, (const uint64_t*)ka, n, shift, ntiles,
                       cnt);
    hipLaunchKernelGGL(k_rs_scan, dim3(1), dim3(RS_SCAN_WG), 0, st, cnt, (int64_t)RS_BINS * ntiles);
    hipLaunchKernelGGL(k_rs_scatter, dim3((unsigned)ntiles), dim3(RS_WG), 0, st, (const uint64_t*)ka,
                       (const int*)va, n, shift, ntiles, (const int*)cnt, kb, vb);
    IFMM_LAUNCH_CHECK();
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (ka != kout) {   // an even number of passes: the result is in the input buffers
    IFMM_HIP(hipMemcpyAsync(kout, ka, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, st));
    IFMM_HIP(hipMemcpyAsync(vout, va, sizeof(int) * (size_t)n, hipMemcpyDeviceToDevice, st));
  }
}

}  // namespace ifmm
