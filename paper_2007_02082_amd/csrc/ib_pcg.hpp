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

// kIBLanes consecutive lanes share a row of the CSR matrix of G (about 25 entries
// for wall points 1.5 h apart), each taking every kIBLanes-th entry, summed by
// shuffles: short dependent chains and kIBLanes times the wavefronts of a
// row-per-lane walk.
constexpr int kIBLanes = 8;

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
// residual block (3 x kIBBlock) is staged in LDS and the threads take the
// (component, row) tasks in turn, each forming its row from the column-major
// inverse (coalesced reads along the rows).  Grid-stride over the blocks.
__global__ __launch_bounds__(kBlock) void k_ib_bjac(int M, int nblk, const float* __restrict__ binv,
                                                    const double* __restrict__ r, double* __restrict__ z,
                                                    int64_t stride, double* __restrict__ partials,
                                                    const KScal* sc) {
  if (sc && sc->done) return;
  __shared__ double rs[3][kIBBlock];
  double v[1] = {0.0};
  const int t = threadIdx.x;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int i0 = b * kIBBlock;
    for (int task = t; task < 3 * kIBBlock; task += kBlock) {
      const int d = task / kIBBlock, i = task % kIBBlock;
      rs[d][i] = (i0 + i < M) ? r[d * stride + i0 + i] : 0.0;
    }
    __syncthreads();
    for (int task = t; task < 3 * kIBBlock; task += kBlock) {
      const int d = task / kIBBlock, i = task % kIBBlock;
      if (i0 + i >= M) continue;
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

// ---- fused iteration: four kernels per CG step --------------------------------
// (1) k_ibcg_qp: p_new = z + beta p_old (the search direction, written by its
//     row) and q = G p_new with p_new formed on the fly from z and p_old for the
//     neighbours (p ping-pongs between two buffers, so no row reads a value
//     being overwritten); partial p_new.q;  (2) k_fin_cg_q: alpha;
// (3) k_ib_xr_bjac: x += alpha p_new, r -= alpha q and z = blockdiag(G)^-1 r on
//     each block of points; partials r.r and r.z;  (4) k_fin_ibcg: convergence
//     test on r.r, beta from r.z.

__global__ __launch_bounds__(kBlock) void k_ibcg_qp(int M, const int64_t* __restrict__ ptr,
                                                    const int32_t* __restrict__ col,
                                                    const double* __restrict__ val, int64_t stride,
                                                    const double* __restrict__ z, const double* __restrict__ pold,
                                                    double* __restrict__ pnew, double* __restrict__ q,
                                                    double* __restrict__ partials, const KScal* sc) {
  if (sc->done) return;
  constexpr int kRows = kBlock / kIBLanes;
  const double beta = sc->beta;
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
        a0 += w * (z[c] + beta * pold[c]);
        a1 += w * (z[stride + c] + beta * pold[stride + c]);
        a2 += w * (z[2 * stride + c] + beta * pold[2 * stride + c]);
      }
    }
#pragma unroll
    for (int off = kIBLanes / 2; off > 0; off >>= 1) {
      a0 += __shfl_xor(a0, off, 64);
      a1 += __shfl_xor(a1, off, 64);
      a2 += __shfl_xor(a2, off, 64);
    }
    if (row < M && sub == 0) {
      const double p0 = z[row] + beta * pold[row];
      const double p1 = z[stride + row] + beta * pold[stride + row];
      const double p2 = z[2 * stride + row] + beta * pold[2 * stride + row];
      pnew[row] = p0;
      pnew[stride + row] = p1;
      pnew[2 * stride + row] = p2;
      q[row] = a0;
      q[stride + row] = a1;
      q[2 * stride + row] = a2;
      v[0] += p0 * a0 + p1 * a1 + p2 * a2;
    }
  }
  block_partials<1>(v, partials);
}

__global__ __launch_bounds__(kBlock) void k_ib_xr_bjac(int M, int nblk, const float* __restrict__ binv,
                                                       double* __restrict__ x, double* __restrict__ r,
                                                       const double* __restrict__ p, const double* __restrict__ q,
                                                       double* __restrict__ z, int64_t stride,
                                                       double* __restrict__ partials, const KScal* sc) {
  if (sc->done) return;
  static_assert(kBlock == 2 * kIBBlock, "two threads per row of a point block");
  __shared__ double rs[3][kIBBlock];
  __shared__ double zh[3][kIBBlock];
  const double alpha = sc->alpha;
  double v[2] = {0.0, 0.0};
  const int t = threadIdx.x;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    for (int task = t; task < 3 * kIBBlock; task += kBlock) {
      const int d = task / kIBBlock, i = task % kIBBlock;
      const int gi = b * kIBBlock + i;
      double ri = 0.0;
      if (gi < M) {
        const int64_t k = d * stride + gi;
        x[k] += alpha * p[k];
        ri = r[k] - alpha * q[k];
        r[k] = ri;
        v[0] += ri * ri;
      }
      rs[d][i] = ri;
    }
    __syncthreads();
    {
      // row i of the block inverse, columns j in half h: each entry is loaded once
      // and applied to the three components; the two halves are summed in LDS
      const int i = t % kIBBlock, h = t / kIBBlock;
      const int gi = b * kIBBlock + i;
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
      if (gi < M) {
        const float* colp = binv + size_t(b) * kIBBlock * kIBBlock + i;
        const int j0 = h * (kIBBlock / 2);
#pragma unroll 16
        for (int j = j0; j < j0 + kIBBlock / 2; ++j) {
          const double g = double(colp[j * kIBBlock]);
          a0 += g * rs[0][j];
          a1 += g * rs[1][j];
          a2 += g * rs[2][j];
        }
      }
      if (h == 1) {
        zh[0][i] = a0;
        zh[1][i] = a1;
        zh[2][i] = a2;
      }
      __syncthreads();
      if (h == 0 && gi < M) {
        const double z0 = a0 + zh[0][i], z1 = a1 + zh[1][i], z2 = a2 + zh[2][i];
        z[gi] = z0;
        z[stride + gi] = z1;
        z[2 * stride + gi] = z2;
        v[1] += rs[0][i] * z0 + rs[1][i] * z1 + rs[2][i] * z2;
      }
    }
    __syncthreads();
  }
  block_partials<2>(v, partials);
}

// r.r -> iteration count and convergence test; r.z -> beta (breakdown if r.z <= 0)
__global__ __launch_bounds__(kBlock) void k_fin_ibcg(const double* __restrict__ partials, int nb, KScal* sc) {
  if (sc->done) return;
  double tot[2];
  sum_partials<2>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  const double rr = tot[0], rz = tot[1];
  sc->rr = rr;
  sc->iters += 1;
  if (bad(rr) || bad(rz)) {
    sc->status = 2;
    sc->done = 1;
    return;
  }
  if (rr <= sc->tol2 * sc->bb || sc->iters >= sc->max_iters) {
    sc->done = 1;
    return;
  }
  if (!(rz > 0.0)) {
    sc->status = 1;
    sc->done = 1;
    return;
  }
  sc->beta = rz / sc->rz;
  sc->rz = rz;
}

}  // namespace ibfe
