// Step-to-step normalised root-mean-square difference of the velocity (the
// steady-state test of the Poiseuille experiment, Section 3.1):
//   L_d = sqrt(sum_i (u_d,i^{n+1} - u_d,i^n)^2 / N^2) / (max_i u_d,i^n - min_i u_d,i^n)
// per component d over the N nodes of P.
#pragma once

#include <cfloat>

#include "kernels.hpp"

namespace ibfe {

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return v;
}

// partials rows: 0..2 sum of squared differences, 3..5 max of u^n, 6..8 max of -u^n
// (row k of block b at part[k * gridDim.x + b]).
__global__ __launch_bounds__(kBlock) void k_nrmse_part(NodeList nl, const uint8_t* __restrict__ flags,
                                                       uint32_t rowbit, const double* __restrict__ un,
                                                       const double* __restrict__ uo, int64_t stride,
                                                       double* __restrict__ part) {
  double s[3] = {0.0, 0.0, 0.0};
  double mx[6] = {-DBL_MAX, -DBL_MAX, -DBL_MAX, -DBL_MAX, -DBL_MAX, -DBL_MAX};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (!(flags[n] & rowbit)) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double a = uo[d * stride + n], b = un[d * stride + n];
      s[d] += (b - a) * (b - a);
      mx[d] = fmax(mx[d], a);
      mx[3 + d] = fmax(mx[3 + d], -a);
    }
  }
  block_partials<3>(s, part);
  __shared__ double sh[6][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double m = wave_max(mx[k]);
    if (lane == 0) sh[k][wave] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      double m = sh[k][0];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) m = fmax(m, sh[k][w]);
      part[(3 + k) * gridDim.x + blockIdx.x] = m;
    }
  }
}

// out[d] = L_d; a component with max = min gets 0 when it did not change and +inf
// when it did.
__global__ __launch_bounds__(kBlock) void k_fin_nrmse(const double* __restrict__ part, int nb, double nnodes,
                                                      double* __restrict__ out) {
  double tot[3];
  sum_partials<3>(part, nb, tot);
  __shared__ double sh[6][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    double m = -DBL_MAX;
    for (int b = threadIdx.x; b < nb; b += kBlock) m = fmax(m, part[(3 + k) * nb + b]);
    m = wave_max(m);
    if (lane == 0) sh[k][wave] = m;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double hi = sh[d][0], nlo = sh[3 + d][0];
#pragma unroll
    for (int w = 1; w < kWaves; ++w) {
      hi = fmax(hi, sh[d][w]);
      nlo = fmax(nlo, sh[3 + d][w]);
    }
    const double range = hi + nlo;  // max - min
    const double rms = sqrt(tot[d]) / nnodes;
    out[d] = range > 0.0 ? rms / range : (tot[d] == 0.0 ? 0.0 : HUGE_VAL);
  }
}

}  // namespace ibfe
