// Device-wide exclusive scan and stable key-value radix sort, used by the
// device rebuild of the IB operators for moving Lagrangian points.  Both are
// deterministic: integer sums only, and the sort keeps equal keys in their input
// order (least significant digit first, 8-bit digits, one histogram, scan and
// scatter per digit).  The caller provides every buffer (no allocation here).
#pragma once

#include "kernels.hpp"

namespace ibfe {

constexpr int kScanTile = 4096;              // elements per workgroup (kBlock x 16)
constexpr int kScanIPT = kScanTile / kBlock;  // elements per thread
constexpr int kRadixBins = 256;

static_assert(kBlock == 256, "the radix kernels use one thread per digit value");

// Inclusive scan of one value per thread across the workgroup (LDS, Hillis-Steele).
template <typename T>
__device__ __forceinline__ T block_inclusive_scan(T v, T* buf) {
  const int t = threadIdx.x;
  buf[t] = v;
  __syncthreads();
  for (int o = 1; o < kBlock; o <<= 1) {
    const T a = t >= o ? buf[t - o] : T(0);
    __syncthreads();
    buf[t] += a;
    __syncthreads();
  }
  const T r = buf[t];
  __syncthreads();
  return r;
}

// sums[tile] = sum of the tile's elements
template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const T* __restrict__ in, int64_t n, T* __restrict__ sums) {
  __shared__ T buf[kBlock];
  const int64_t t0 = int64_t(blockIdx.x) * kScanTile;
  T s = T(0);
  for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
    const int64_t q = t0 + i;
    if (q < n) s += in[q];
  }
  const T incl = block_inclusive_scan<T>(s, buf);
  if (threadIdx.x == kBlock - 1) sums[blockIdx.x] = incl;
}

// In-place exclusive scan of nb tile sums by one workgroup, kBlock values at a time.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_sums(T* __restrict__ sums, int nb) {
  __shared__ T buf[kBlock];
  T carry = T(0);
  for (int base = 0; base < nb; base += kBlock) {
    const int i = base + int(threadIdx.x);
    const T v = i < nb ? sums[i] : T(0);
    const T incl = block_inclusive_scan<T>(v, buf);
    if (i < nb) sums[i] = carry + incl - v;
    // the last thread's inclusive value is the chunk total: every thread reads it
    if (threadIdx.x == kBlock - 1) buf[0] = incl;
    __syncthreads();
    carry += buf[0];
    __syncthreads();
  }
}

// out = exclusive prefix sums of in (out may alias in): each thread scans its 16
// consecutive elements after the workgroup scan of the per-thread totals.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_scan_tiles(const T* in, T* out, int64_t n, const T* __restrict__ sums) {
  __shared__ T buf[kBlock];
  const int64_t t0 = int64_t(blockIdx.x) * kScanTile + int64_t(threadIdx.x) * kScanIPT;
  T v[kScanIPT];
  T s = T(0);
#pragma unroll
  for (int k = 0; k < kScanIPT; ++k) {
    const int64_t q = t0 + k;
    v[k] = q < n ? in[q] : T(0);
    s += v[k];
  }
  const T incl = block_inclusive_scan<T>(s, buf);
  T run = sums[blockIdx.x] + incl - s;
#pragma unroll
  for (int k = 0; k < kScanIPT; ++k) {
    const int64_t q = t0 + k;
    if (q < n) out[q] = run;
    run += v[k];
  }
}

inline int scan_tiles(int64_t n) { return int((n + kScanTile - 1) / kScanTile); }

// p[0..n) = v (fill kernels instead of memsets, so that a caller may capture them)
__global__ __launch_bounds__(kBlock) void k_fill_f64(double* __restrict__ p, int64_t n, double v) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q < n) p[q] = v;
}
__global__ __launch_bounds__(kBlock) void k_fill_i32(int* __restrict__ p, int64_t n, int v) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q < n) p[q] = v;
}

// Digit histogram of every tile, digit-major: hist[d * nb + tile].
__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                    uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t h[kRadixBins];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t t0 = int64_t(blockIdx.x) * kScanTile;
  for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
    const int64_t q = t0 + i;
    if (q < n) atomicAdd(&h[(keys[q] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[int64_t(threadIdx.x) * nb + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter by one digit: the tile is taken kBlock elements at a time in
// order; within such a chunk an element's rank among equal digits comes from
// wavefront ballots (lanes with the same 8 digit bits) and the counts of the
// lower wavefronts; offs[d * nb + tile] is where the tile's digit d starts.
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin,
                                                       uint32_t* __restrict__ kout, uint32_t* __restrict__ vout,
                                                       int64_t n, int shift, const uint32_t* __restrict__ offs,
                                                       int nb) {
  constexpr int W = kBlock / 64;
  __shared__ uint32_t run[kRadixBins];
  __shared__ uint32_t wc[W][kRadixBins];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  run[t] = offs[int64_t(t) * nb + blockIdx.x];
  const int64_t t0 = int64_t(blockIdx.x) * kScanTile;
  for (int base = 0; base < kScanTile; base += kBlock) {
#pragma unroll
    for (int k = 0; k < W; ++k) wc[k][t] = 0u;
    __syncthreads();
    const int64_t q = t0 + base + t;
    const bool ok = q < n;
    const uint32_t key = ok ? kin[q] : 0u;
    const uint32_t d = (key >> shift) & 0xFFu;
    uint64_t peers = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t bb = __ballot(bit);
      peers &= bit ? bb : ~bb;
    }
    const uint64_t lower = peers & ((uint64_t(1) << lane) - 1u);
    if (ok && lower == 0) wc[w][d] = uint32_t(__popcll(peers));
    __syncthreads();
    if (ok) {
      uint32_t pos = run[d] + uint32_t(__popcll(lower));
      for (int k = 0; k < w; ++k) pos += wc[k][d];
      kout[pos] = key;
      vout[pos] = vin[q];
    }
    __syncthreads();
    uint32_t tot = 0u;
#pragma unroll
    for (int k = 0; k < W; ++k) tot += wc[k][t];
    run[t] += tot;
    __syncthreads();
  }
}

}  // namespace ibfe
