// Block-Jacobi preconditioned CG for the force system G Lambda = b of the BCE-IB
// correction (Section 2.3, Eqs. 20-22), three components at once.  The points
// are taken in blocks of kIBBlock consecutive indices (the generators place
// neighbouring wall points next to each other, so a block holds the strongly
// coupled points of a surface patch); the preconditioner multiplies each block
// of the residual by the inverse of the matching diagonal block of G, built once
// at set-up.  Vectors are 3 planes of `stride` values over the points.
#pragma once

#include "kernels.hpp"
#include "plan.hpp"

namespace ibfe {

// q = G p (three components) and partial p.q.  kIBLanes consecutive lanes share
// a row of the CSR matrix (about 25 entries for wall points 1.5 h apart), each
// taking every kIBLanes-th entry, and are summed by shuffles: short dependent
// chains and kIBLanes times the wavefronts of a row-per-lane walk.
constexpr int kIBLanes = 8;

__global__ __launch_bounds__(kBlock) void k_ibcg_q(int M, const int64_t* __restrict__ ptr,
                                                   const int32_t* __restrict__ col,
                                                   const double* __restrict__ val, int64_t stride,
                                                   const double* __restrict__ p, double* __restrict__ q,
                                                   double* __restrict__ partials, const KScal* sc) {
  if (sc->done) return;
  constexpr int kRows = kBlock / kIBLanes;
  double v[1] = {0.0};
  const int sub = threadIdx.x % kIBLanes;
  for (int r0 = blockIdx.x * kRows; r0 < M; r0 += gridDim.x * kRows) {
    const int row = r0 + int(threadIdx.x) / kIBLanes;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0;
    if (row < M) {
      const int64_t e = ptr[row + 1];
      for (int64_t k = ptr[row] + sub; k < e; k += kIBLanes) {
        const double w = val[k];
        const int c = col[k];
        a0 += w * p[c];
        a1 += w * p[stride + c];
        a2 += w * p[2 * stride + c];
      }
    }
#pragma unroll
    for (int off = kIBLanes / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, 64);
      a1 += __shfl_xor(a1, off, 64);
      a2 += __shfl_xor(a2, off, 64);
    }
    if (row < M && sub == 0) {
      q[row] = a0;
      q[stride + row] = a1;
      q[2 * stride + row] = a2;
      v[0] += p[row] * a0 + p[stride + row] * a1 + p[2 * stride + row] * a2;
    }
  }
  block_partials<1>(v, partials);
}

// r = b - G x (x = 0 with zero_guess); partials r.r, b.b
__global__ __launch_bounds__(kBlock) void k_ibcg_init(NodeList nl, OpCSR<3> op, const double* __restrict__ b,
                                                      double* __restrict__ x, double* __restrict__ r,
                                                      double* __restrict__ partials, int zero_guess) {
  double v[2] = {0.0, 0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    const bool rw = op.row(n);
    double gx[3] = {0.0, 0.0, 0.0};
    if (!zero_guess && rw) op.apply(n, x, gx);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t i = d * op.stride + n;
      if (zero_guess) x[i] = 0.0;
      const double bi = rw ? b[i] : 0.0;
      const double ri = rw ? bi - gx[d] : 0.0;
      r[i] = ri;
      v[0] += ri * ri;
      v[1] += bi * bi;
    }
  }
  block_partials<2>(v, partials);
}

// z = blockdiag(G)^-1 r; partial r.z.  One workgroup per block of points: the
// residual block (3 x kIBBlock) is staged in LDS, thread t < 3 kIBBlock forms
// row t % kIBBlock of component t / kIBBlock from the column-major inverse
// (coalesced reads along the rows).  Grid-stride over the blocks.
__global__ __launch_bounds__(kBlock) void k_ib_bjac(int M, int nblk, const float* __restrict__ binv,
                                                    const double* __restrict__ r, double* __restrict__ z,
                                                    int64_t stride, double* __restrict__ partials,
                                                    const KScal* sc) {
  static_assert(3 * kIBBlock <= kBlock, "one thread per row and component");
  if (sc && sc->done) return;
  __shared__ double rs[3][kIBBlock];
  double v[1] = {0.0};
  const int t = threadIdx.x;
  const int d = t / kIBBlock, i = t % kIBBlock;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int i0 = b * kIBBlock;
    if (t < 3 * kIBBlock) rs[d][i] = (i0 + i < M) ? r[d * stride + i0 + i] : 0.0;
    __syncthreads();
    if (t < 3 * kIBBlock && i0 + i < M) {
      const float* col = binv + size_t(b) * kIBBlock * kIBBlock + i;
      double acc = 0.0;
#pragma unroll 8
      for (int j = 0; j < kIBBlock; ++j) acc += double(col[j * kIBBlock]) * rs[d][j];
      z[d * stride + i0 + i] = acc;
      v[0] += rs[d][i] * acc;
    }
    __syncthreads();
  }
  block_partials<1>(v, partials);
}

// x += alpha p, r -= alpha q; partial r.r
__global__ __launch_bounds__(kBlock) void k_ibcg_xr(NodeList nl, int M, int64_t stride, double* __restrict__ x,
                                                    double* __restrict__ r, const double* __restrict__ p,
                                                    const double* __restrict__ q, double* __restrict__ partials,
                                                    const KScal* sc) {
  if (sc->done) return;
  const double alpha = sc->alpha;
  double v[1] = {0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (n >= M) continue;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int64_t i = d * stride + n;
      x[i] += alpha * p[i];
      const double ri = r[i] - alpha * q[i];
      r[i] = ri;
      v[0] += ri * ri;
    }
  }
  block_partials<1>(v, partials);
}

// p = z + beta p
__global__ __launch_bounds__(kBlock) void k_ibcg_p(NodeList nl, int M, int64_t stride,
                                                   const double* __restrict__ z, double* __restrict__ p,
                                                   const KScal* sc) {
  if (sc->done) return;
  const double beta = sc->beta;
  const int n = chunk_node(nl);
  if (n < 0 || n >= M) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int64_t i = d * stride + n;
    p[i] = z[i] + beta * p[i];
  }
}

}  // namespace ibfe
