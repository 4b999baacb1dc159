// Rebuild of the immersed-boundary operators on the device for moving
// Lagrangian points (the points X_i change from step to step; Section 2.3
// defines I, I_F and the force system G = I_F I_F^T for the current positions).
//
// 1. k_ib_stencil: the 4x4x4 support of every point with the weights of Eq. 17
//    (times h^3) and the kernel of Eq. 18, in the layout of the static plan
//    ([64][M] node ids, -1 outside the box), plus one (node, slot) pair per
//    support node (node = N when the node is not free, which sorts last).
// 2. A stable radix sort of the pairs by node (point-major input order, so the
//    points of a node stay in ascending order) gives the spreading lists I_F^T:
//    k_sp_flags / k_sp_fill compact them into (node, ptr, point, weight).
// 3. k_gram_rows: one wavefront per row i of G.  Its candidates are the
//    (point k, w_ij w_kj) products over its free support nodes j, generated in
//    slot order and, per node, in point order; they are sorted by k in LDS
//    (ties keep the generation order) and summed per k in that order.  Run once
//    to count the entries of every row (CSR pointers by a scan) and once to
//    write them.  No floating-point atomics: G is the same on every run.
// 4. k_gram_block_inv: one workgroup per block of kIBBlock consecutive points:
//    the dense diagonal block, its Cholesky factor, the inverse factor and the
//    block inverse L^-T L^-1 rounded to FP32 (the block-Jacobi preconditioner).
#pragma once

#include <cstdint>

#include "kernels.hpp"
#include "plan.hpp"

namespace ibfe {

constexpr int kGramCap = 1024;  // candidate products per row of G held in LDS

// Four-point regularised delta of Eq. 18 (support |r| < 2).
__device__ __forceinline__ double delta4_dev(double r) {
  r = fabs(r);
  if (r <= 1.0) return (3.0 - 2.0 * r + sqrt(1.0 + 4.0 * r - 4.0 * r * r)) / 8.0;
  if (r <= 2.0) return (5.0 - 2.0 * r - sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) / 8.0;
  return 0.0;
}

struct GridGeom {
  double ox, oy, oz, h;
  int nx, ny, nz;   // cells
  int64_t sy, sz;   // node id strides
};

// counters[0]: points without free support, [1]: rows whose candidates exceed
// kGramCap, [2]: n_sp (spreading nodes), [3]: entries of the spreading lists,
// [4]: support nodes outside `band` (refined lattice: the closure of the flagged
// cells minus the hanging nodes; NULL on a uniform grid).
__global__ __launch_bounds__(kBlock) void k_ib_stencil(int M, GridGeom g, const double* __restrict__ X,
                                                       const uint8_t* __restrict__ flags, uint32_t N,
                                                       int32_t* __restrict__ idx, double* __restrict__ w,
                                                       uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                                       int* __restrict__ counters, const uint8_t* __restrict__ band) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= M) return;
  const double o[3] = {g.ox, g.oy, g.oz};
  const int dims[3] = {g.nx, g.ny, g.nz};
  int64_t base[3];
  double wd[3][4];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double xi = X[3 * i + d];
    base[d] = int64_t(floor((xi - o[d]) / g.h)) - 1;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const double xn = o[d] + double(base[d] + a) * g.h;
      wd[d][a] = delta4_dev((xn - xi) / g.h);
    }
  }
  double free2 = 0.0;
  for (int c = 0; c < 4; ++c)
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int s = a + 4 * b + 16 * c;
        const int64_t ii = base[0] + a, jj = base[1] + b, kk = base[2] + c;
        int32_t n = -1;
        double ws = 0.0;
        uint32_t key = N;
        if (ii >= 0 && jj >= 0 && kk >= 0 && ii <= dims[0] && jj <= dims[1] && kk <= dims[2]) {
          n = int32_t(ii + g.sy * jj + g.sz * kk);
          if (band && !band[n]) atomicAdd(&counters[4], 1);
          ws = wd[0][a] * wd[1][b] * wd[2][c];
          if (flags[n] & IBFE_FLAG_F) {
            free2 += ws * ws;
            key = uint32_t(n);
          }
        }
        idx[int64_t(s) * M + i] = n;
        w[int64_t(s) * M + i] = ws;
        keys[int64_t(i) * 64 + s] = key;
        vals[int64_t(i) * 64 + s] = uint32_t(int64_t(i) * 64 + s);
      }
  if (free2 < 1e-12) atomicAdd(&counters[0], 1);
}

// flag[q] = 1 where a new free node starts in the sorted pairs.
__global__ __launch_bounds__(kBlock) void k_sp_flags(int64_t n, const uint32_t* __restrict__ k, uint32_t N,
                                                     int* __restrict__ flag) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= n) return;
  flag[q] = (k[q] < N && (q == 0 || k[q] != k[q - 1])) ? 1 : 0;
}

// Spreading lists from the sorted pairs: node list, CSR pointers, point ids and
// weights; the last valid entry also writes the closing pointer and the counts.
__global__ __launch_bounds__(kBlock) void k_sp_fill(int64_t n, int M, const uint32_t* __restrict__ k,
                                                    const uint32_t* __restrict__ v, uint32_t N,
                                                    const int* __restrict__ flag, const int* __restrict__ pos,
                                                    const double* __restrict__ w, int32_t* __restrict__ sp_node,
                                                    int64_t* __restrict__ sp_ptr, int32_t* __restrict__ sp_pt,
                                                    double* __restrict__ sp_wt, int* __restrict__ counters) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= n || k[q] >= N) return;
  const uint32_t code = v[q];
  const int i = int(code >> 6), s = int(code & 63u);
  sp_pt[q] = i;
  sp_wt[q] = w[int64_t(s) * M + i];
  if (flag[q]) {
    sp_node[pos[q]] = int32_t(k[q]);
    sp_ptr[pos[q]] = q;
  }
  if (q + 1 == n || k[q + 1] >= N) {
    const int nsp = pos[q] + flag[q];
    sp_ptr[nsp] = q + 1;
    counters[2] = nsp;
    counters[3] = int(q + 1);
  }
}

// first position in [0, n) whose key is >= key
__device__ __forceinline__ int64_t lower_bound_u32(const uint32_t* __restrict__ a, int64_t n, uint32_t key) {
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// One wavefront (64 threads, one per support slot) per row of G.  FILL = false:
// cnt[i] = number of distinct columns; FILL = true: write columns, values and
// the diagonal from ptr.
template <bool FILL>
__global__ __launch_bounds__(64) void k_gram_rows(int M, const int32_t* __restrict__ idx,
                                                  const double* __restrict__ w,
                                                  const uint8_t* __restrict__ flags,
                                                  const uint32_t* __restrict__ skeys, int64_t nvalid,
                                                  const int32_t* __restrict__ sp_pt,
                                                  const double* __restrict__ sp_wt, int64_t* __restrict__ cnt,
                                                  const int64_t* __restrict__ ptr, int32_t* __restrict__ col,
                                                  double* __restrict__ val, double* __restrict__ diag,
                                                  int* __restrict__ counters) {
  __shared__ int64_t key[kGramCap];   // k * kGramCap + generation index
  __shared__ double cv[kGramCap];     // candidate products, by generation index
  __shared__ int off[64];
  __shared__ int tot;
  const int i = blockIdx.x;
  const int s = threadIdx.x;
  const int32_t n = idx[int64_t(s) * M + i];
  int64_t lo = 0, hi = 0;
  double wi = 0.0;
  if (n >= 0 && (flags[n] & IBFE_FLAG_F)) {
    wi = w[int64_t(s) * M + i];
    lo = lower_bound_u32(skeys, nvalid, uint32_t(n));
    hi = lower_bound_u32(skeys, nvalid, uint32_t(n) + 1u);
  }
  const int len = int(hi - lo);
  // exclusive prefix of the candidate counts in slot order
  off[s] = len;
  __syncthreads();
  if (s == 0) {
    int acc = 0;
    for (int t = 0; t < 64; ++t) {
      const int l = off[t];
      off[t] = acc;
      acc += l;
    }
    tot = acc;
  }
  __syncthreads();
  const int total = tot;
  if (total > kGramCap) {
    if (s == 0) {
      atomicAdd(&counters[1], 1);
      if (!FILL) cnt[i] = 0;
    }
    return;
  }
  const int my = off[s];
  for (int j = 0; j < len; ++j) {
    const int g = my + j;
    key[g] = int64_t(sp_pt[lo + j]) * kGramCap + g;
    cv[g] = wi * sp_wt[lo + j];
  }
  int P2 = 1;
  while (P2 < total) P2 <<= 1;
  for (int g = total + s; g < P2; g += 64) key[g] = INT64_MAX;
  __syncthreads();
  // bitonic sort of key[0, P2) (the keys are distinct, so ties in k keep the
  // generation order)
  for (int kk = 2; kk <= P2; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int a = s; a < P2; a += 64) {
        const int b = a ^ jj;
        if (b > a) {
          const bool up = (a & kk) == 0;
          const int64_t x = key[a], y = key[b];
          if ((x > y) == up) {
            key[a] = y;
            key[b] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // every thread takes a contiguous range of sorted positions; a column starts
  // where k changes
  const int chunk = (total + 63) / 64;
  const int a0 = min(total, s * chunk), a1 = min(total, a0 + chunk);
  int mine = 0;
  for (int a = a0; a < a1; ++a)
    if (a == 0 || key[a] / kGramCap != key[a - 1] / kGramCap) ++mine;
  off[s] = mine;
  __syncthreads();
  if (s == 0) {
    int acc = 0;
    for (int t = 0; t < 64; ++t) {
      const int l = off[t];
      off[t] = acc;
      acc += l;
    }
    tot = acc;
  }
  __syncthreads();
  if (!FILL) {
    if (s == 0) cnt[i] = tot;
    return;
  }
  const int64_t row0 = ptr[i];
  int rank = off[s];
  for (int a = a0; a < a1; ++a) {
    const int64_t ka = key[a] / kGramCap;
    if (a != 0 && ka == key[a - 1] / kGramCap) continue;
    double acc = 0.0;
    for (int b = a; b < total && key[b] / kGramCap == ka; ++b) acc += cv[key[b] % kGramCap];
    col[row0 + rank] = int32_t(ka);
    val[row0 + rank] = acc;
    if (ka == i) diag[i] = acc;
    ++rank;
  }
}

// One workgroup per diagonal block of G: binv = (L L^T)^-1 = L^-T L^-1 in FP32,
// zero outside the n x n leading part of the last block.  One LDS array holds the
// block: the Cholesky factor L overwrites its lower triangle, the inverse factor
// Li = L^-1 (lower triangular) is kept transposed in the strict upper triangle
// (Li[r][j] at A[j][r], r > j) with its diagonal in dli.
__global__ __launch_bounds__(kBlock) void k_gram_block_inv(int M, const int64_t* __restrict__ ptr,
                                                           const int32_t* __restrict__ col,
                                                           const double* __restrict__ val,
                                                           float* __restrict__ binv) {
  constexpr int B = kIBBlock;
  __shared__ double A[B][B + 1];
  __shared__ double dli[B];
  const int b = blockIdx.x, t = threadIdx.x;
  const int i0 = b * B;
  const int n = min(B, M - i0);
  for (int q = t; q < B * B; q += kBlock) A[q / B][q % B] = 0.0;
  __syncthreads();
  for (int r = t; r < n; r += kBlock)
    for (int64_t q = ptr[i0 + r]; q < ptr[i0 + r + 1]; ++q) {
      const int k = col[q] - i0;
      if (k >= 0 && k <= r) A[r][k] = val[q];  // the lower triangle of the symmetric block
    }
  __syncthreads();
  // Cholesky, column by column: L_jj, then the column below it
  for (int j = 0; j < n; ++j) {
    if (t < 64) {
      // L_jj^2 = A_jj - sum_{k<j} L_jk^2, the sum split over the first wavefront
      double d = 0.0;
      for (int k = t; k < j; k += 64) d += A[j][k] * A[j][k];
      d = wave_sum(d);
      if (t == 0) A[j][j] = sqrt(fmax(A[j][j] - d, 1e-300));
    }
    __syncthreads();
    for (int r = j + 1 + t; r < n; r += kBlock) {
      double v = A[r][j];
      for (int k = 0; k < j; ++k) v -= A[r][k] * A[j][k];
      A[r][j] = v / A[j][j];
    }
    __syncthreads();
  }
  // Li = L^-1, one column per thread (column j of Li goes to row j of the upper part)
  for (int j = t; j < n; j += kBlock) {
    dli[j] = 1.0 / A[j][j];
    for (int r = j + 1; r < n; ++r) {
      double v = -A[r][j] * dli[j];
      for (int k = j + 1; k < r; ++k) v -= A[r][k] * A[j][k];
      A[j][r] = v / A[r][r];
    }
  }
  __syncthreads();
  float* out = binv + size_t(b) * B * B;
  for (int q = t; q < B * B; q += kBlock) {
    const int r = q / B, c = q % B;
    float o = 0.0f;
    if (r < n && c < n) {
      // sum over k >= max(r, c) of Li[k][r] Li[k][c]; Li[k][k] = dli[k], Li[k][m] = A[m][k]
      const int lo = r > c ? r : c;
      const double lr = lo == r ? dli[r] : A[r][lo];
      const double lc = lo == c ? dli[c] : A[c][lo];
      double v = lr * lc;
      for (int k = lo + 1; k < n; ++k) v += A[r][k] * A[c][k];
      o = float(v);
    }
    out[r * B + c] = o;
  }
}

}  // namespace ibfe
