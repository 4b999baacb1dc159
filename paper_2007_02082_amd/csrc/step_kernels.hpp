// gfx950 kernels for the non-Krylov parts of the step: the advection-diffusion
// stencil of the tentative velocity, right-hand sides, the IB interpolation and
// spreading, inlet data and element-wise updates.
#pragma once

#include "kernels.hpp"

namespace ibfe {

constexpr uint32_t kFlagP = 1u, kFlagF = 2u, kFlagDu = 4u, kFlagPdir = 8u;

// Per-cell entries of the Q1 forms on a cube of side h for a neighbour offset
// with t nonzero components: mass prod_d m(o_d), stiffness
// sum_d k(o_d) prod_{e!=d} m(o_e), with m(0) = h/3, m(1) = h/6, k(0) = 1/h,
// k(1) = -1/h (exact 1-D element integrals).
struct FormCoefs {
  double m[4], k[4], g2[3];
};

inline FormCoefs form_coefs(double h) {
  FormCoefs f{};
  const double m0 = h / 3.0, m1 = h / 6.0, k0 = 1.0 / h, k1 = -1.0 / h;
  for (int t = 0; t <= 3; ++t) {
    // t axes differ (offset +-1), 3 - t axes coincide
    double mv = 1.0;
    for (int a = 0; a < 3; ++a) mv *= (a < t) ? m1 : m0;
    f.m[t] = mv;
    double kv = 0.0;
    for (int d = 0; d < 3; ++d) {
      double term = (d < t) ? k1 : k0;
      for (int a = 0; a < 3; ++a)
        if (a != d) term *= (a < t) ? m1 : m0;
      kv += term;
    }
    f.k[t] = kv;
  }
  for (int c = 0; c <= 2; ++c) {
    double g = 0.5;
    for (int a = 0; a < 2; ++a) g *= (a < c) ? m1 : m0;
    f.g2[c] = g;
  }
  return f;
}

// ---------------------------------------------------------------------------
// tentative-velocity operator A = (rho/dt) M + rho C(u^n) + mu K as a stored
// 27-point stencil per node (rows of P).  The advection part
// C_ij = sum_cells sum_c sum_d u_{c,d} int N_i N_c d_d N_j uses the exact
// 1-D integrals int phi_a phi_b phi_c = h/4 (all equal) or h/12, and
// int phi_a phi_b phi_c' = +-(1/3 if a == b else 1/6) (sign of phi_c').
// ---------------------------------------------------------------------------

__device__ __forceinline__ constexpr double t0c(int a, int b, int c) {
  return (a == b && b == c) ? 0.25 : (1.0 / 12.0);
}
__device__ __forceinline__ constexpr double t1c(int a, int b, int c) {
  return (c == 1 ? 1.0 : -1.0) * (a == b ? (1.0 / 3.0) : (1.0 / 6.0));
}

__global__ __launch_bounds__(kBlock) void k_s1_build(NodeList nl,
                                                     const uint8_t* __restrict__ emask,
                                                     const uint8_t* __restrict__ flags,
                                                     const double* __restrict__ u, int64_t stride,
                                                     int sy, int sz, double h, double cm0, double cm1,
                                                     double cm2, double cm3, double rho,
                                                     double* __restrict__ coef64,
                                                     float* __restrict__ coef32, int st,
                                                     uint32_t rowbit) {
  // st = 2 (with sy, sz of the lattice) builds the coarse-element part of a
  // refined lattice from the coarse cell bits in `emask`
  const int n = chunk_node(nl);
  if (n < 0) return;
  double A[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) A[t] = 0.0;
  const uint32_t e = emask[n];
  if (flags[n] & rowbit) {
    const double cmk[4] = {cm0, cm1, cm2, cm3};
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          const int t = (ox != 0) + (oy != 0) + (oz != 0);
          A[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)] =
              cmk[t] * double(__builtin_popcount(e & compat(ox, oy, oz)));
        }
    const double rh2 = rho * h * h;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (!((e >> s) & 1u)) continue;
      const int li[3] = {1 - (s & 1), 1 - ((s >> 1) & 1), 1 - ((s >> 2) & 1)};
      double a[8][3];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int lc[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        const int off = st * ((lc[0] - li[0]) + sy * (lc[1] - li[1]) + sz * (lc[2] - li[2]));
#pragma unroll
        for (int d = 0; d < 3; ++d) a[c][d] = u[d * stride + n + off];
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int lj[3] = {j & 1, (j >> 1) & 1, (j >> 2) & 1};
        const int ti = (lj[0] - li[0] + 1) + 3 * (lj[1] - li[1] + 1) + 9 * (lj[2] - li[2] + 1);
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          const int lc[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            double w = t1c(li[d], lc[d], lj[d]);
#pragma unroll
            for (int q = 0; q < 3; ++q)
              if (q != d) w *= t0c(li[q], lc[q], lj[q]);
            acc += a[c][d] * w;
          }
        }
        A[ti] += rh2 * acc;
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 27; ++t) {
    coef64[t * stride + n] = A[t];
    if (coef32) coef32[t * stride + n] = float(A[t]);
  }
}

// b_d = (rho/dt)(M u_d) - G_d p on free rows, 0 elsewhere (Eq. 9); the lifting
// of the Dirichlet data, - A g_d, follows in k_s1_lift on the rows next to it.
__global__ __launch_bounds__(kBlock) void k_s1_rhs(NodeList nl,
                                                   const uint8_t* __restrict__ emask,
                                                   const uint8_t* __restrict__ flags,
                                                   const double* __restrict__ u, const double* __restrict__ p,
                                                   double* __restrict__ b,
                                                   int64_t stride, int sy, int sz, double cm0,
                                                   double cm1, double cm2, double cm3, double g20,
                                                   double g21, double g22) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  if (!(flags[n] & kFlagF)) {
#pragma unroll
    for (int d = 0; d < 3; ++d) b[d * stride + n] = 0.0;
    return;
  }
  const uint32_t e = emask[n];
  const double cm[4] = {cm0, cm1, cm2, cm3};
  const double g2[3] = {g20, g21, g22};
  const double gp[3] = {apply_grad<double, 0>(p, n, e, g2, sy, sz),
                        apply_grad<double, 1>(p, n, e, g2, sy, sz),
                        apply_grad<double, 2>(p, n, e, g2, sy, sz)};
#pragma unroll
  for (int d = 0; d < 3; ++d)
    b[d * stride + n] = apply_sym<double>(u + d * stride, n, e, cm, sy, sz) - gp[d];
}

// b_d -= A g_d (stored stencil) on the listed rows: the free rows with an
// inlet-table node among their 27 neighbours, the only rows where g(t^{n+1}),
// zero off the inlet table, contributes.
__global__ __launch_bounds__(kBlock) void k_s1_lift(int nrows, const int32_t* __restrict__ rows,
                                                    const uint8_t* __restrict__ flags,
                                                    const double* __restrict__ coef,
                                                    const double* __restrict__ g, double* __restrict__ b,
                                                    int64_t stride, int sy, int sz) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= nrows) return;
  const int n = rows[q];
  OpStencil<double, 3> A{coef, flags, kFlagF, sy, sz, stride};
  double ag[3];
  A.apply(n, g, ag);
#pragma unroll
  for (int d = 0; d < 3; ++d) b[d * stride + n] -= ag[d];
}

// Explicit advection: b_d = (rho/dt)(M u_d) - (rho C(u^n) u^n)_d - G_d p - A' g_d on
// free rows with A' = (rho/dt) M + mu K; `adv` holds the stencil of rho C(u^n).
__global__ __launch_bounds__(kBlock) void k_s1_rhs_explicit(
    NodeList nl, const uint8_t* __restrict__ emask,
    const uint8_t* __restrict__ flags, const double* __restrict__ adv, const double* __restrict__ u,
    const double* __restrict__ p, const double* __restrict__ g, double* __restrict__ b, int64_t stride, int sy,
    int sz, double cm0, double cm1, double cm2, double cm3, double ca0, double ca1, double ca2, double ca3,
    double g20, double g21, double g22) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  if (!(flags[n] & kFlagF)) {
#pragma unroll
    for (int d = 0; d < 3; ++d) b[d * stride + n] = 0.0;
    return;
  }
  const uint32_t e = emask[n];
  const double cm[4] = {cm0, cm1, cm2, cm3};
  const double ca[4] = {ca0, ca1, ca2, ca3};
  const double g2[3] = {g20, g21, g22};
  const double gp[3] = {apply_grad<double, 0>(p, n, e, g2, sy, sz),
                        apply_grad<double, 1>(p, n, e, g2, sy, sz),
                        apply_grad<double, 2>(p, n, e, g2, sy, sz)};
  OpStencil<double, 3> C{adv, flags, kFlagF, sy, sz, stride};
  double cu[3];
  C.apply(n, u, cu);
#pragma unroll
  for (int d = 0; d < 3; ++d)
    b[d * stride + n] = apply_sym<double>(u + d * stride, n, e, cm, sy, sz) - cu[d] - gp[d] -
                        apply_sym<double>(g + d * stride, n, e, ca, sy, sz);
}

// b = scale * sum_d G_d u_d on rows with (flags & rowbit), 0 elsewhere.
__global__ __launch_bounds__(kBlock) void k_div(NodeList nl,
                                                const uint8_t* __restrict__ emask,
                                                const uint8_t* __restrict__ flags, uint32_t rowbit,
                                                uint32_t exclude, const double* __restrict__ u,
                                                double* __restrict__ b, int64_t stride, int sy, int sz,
                                                double g20, double g21, double g22, double scale) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  const uint32_t f = flags[n];
  if (!(f & rowbit) || (f & exclude)) {
    b[n] = 0.0;
    return;
  }
  const uint32_t e = emask[n];
  const double g2[3] = {g20, g21, g22};
  const double s = apply_grad<double, 0>(u, n, e, g2, sy, sz) +
                   apply_grad<double, 1>(u + stride, n, e, g2, sy, sz) +
                   apply_grad<double, 2>(u + 2 * stride, n, e, g2, sy, sz);
  b[n] = scale * s;
}

// y_d = G_d x on rows with (flags & rowbit), 0 elsewhere.
__global__ __launch_bounds__(kBlock) void k_grad(NodeList nl,
                                                 const uint8_t* __restrict__ emask,
                                                 const uint8_t* __restrict__ flags, uint32_t rowbit,
                                                 const double* __restrict__ x, double* __restrict__ y,
                                                 int64_t stride, int sy, int sz, double g20, double g21,
                                                 double g22) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  if (!(flags[n] & rowbit)) {
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d * stride + n] = 0.0;
    return;
  }
  const uint32_t e = emask[n];
  const double g2[3] = {g20, g21, g22};
  y[n] = apply_grad<double, 0>(x, n, e, g2, sy, sz);
  y[stride + n] = apply_grad<double, 1>(x, n, e, g2, sy, sz);
  y[2 * stride + n] = apply_grad<double, 2>(x, n, e, g2, sy, sz);
}

// Plain apply of a symmetric form or the stored stencil (verification hooks).
template <typename T, int NC, class Op>
__global__ __launch_bounds__(kBlock) void k_apply(NodeList nl, Op op,
                                                  const T* __restrict__ x, T* __restrict__ y) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  T v[NC];
  const bool rw = op.row(n);
  if (rw) op.apply(n, x, v);
#pragma unroll
  for (int d = 0; d < NC; ++d) y[d * op.stride + n] = rw ? v[d] : T(0);
}

// ---------------------------------------------------------------------------
// immersed boundary
// ---------------------------------------------------------------------------

// b_d[i] = U_B[i][d] - sum_s w[s][i] u_d[idx[s][i]]   (Eq. 23 with h^3 D = w)
// Eight lanes per point: lane g * 8 + p of a wavefront sums slots 8 g .. 8 g + 7 of
// point 8 w + p (w the wavefront's point group), so the lanes of one slot group
// read 8 consecutive points of the slot-major stencil; the eight partial sums of a
// point are added across the lanes in a fixed order.  Grid: ceil(M / 8) wavefronts.
__global__ __launch_bounds__(kBlock) void k_ib_interp(int M, const int32_t* __restrict__ idx,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ UB,
                                                      const double* __restrict__ u, int64_t stride,
                                                      double* __restrict__ b, int64_t bstride,
                                                      int with_ub) {
  const int lane = threadIdx.x & 63;
  const int g = lane >> 3, p = lane & 7;
  const int i = (blockIdx.x * kWaves + int(threadIdx.x >> 6)) * 8 + p;
  const bool ok = i < M;
  double acc[3] = {0.0, 0.0, 0.0};
  if (ok) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int s = 8 * g + k;
      const int n = idx[int64_t(s) * M + i];
      if (n < 0) continue;
      const double ws = w[int64_t(s) * M + i];
#pragma unroll
      for (int d = 0; d < 3; ++d) acc[d] += ws * u[d * stride + n];
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int off = 8; off < 64; off <<= 1) acc[d] += __shfl_xor(acc[d], off, 64);
  if (ok && g == 0) {
#pragma unroll
    for (int d = 0; d < 3; ++d) b[d * bstride + i] = (with_ub ? UB[3 * i + d] : 0.0) - acc[d];
  }
}

// u_d[node] += sum_{points} w lam_d[point] over free support nodes (I_F^T lam),
// one thread per node: deterministic, no atomics.
__global__ __launch_bounds__(kBlock) void k_ib_spread(int nnodes, const int32_t* __restrict__ node,
                                                      const int64_t* __restrict__ ptr,
                                                      const int32_t* __restrict__ pt,
                                                      const double* __restrict__ w,
                                                      const double* __restrict__ lam, int64_t lstride,
                                                      double* __restrict__ u, int64_t stride) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= nnodes) return;
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t k = ptr[q]; k < ptr[q + 1]; ++k) {
    const double wk = w[k];
    const int i = pt[k];
#pragma unroll
    for (int d = 0; d < 3; ++d) acc[d] += wk * lam[d * lstride + i];
  }
  const int n = node[q];
#pragma unroll
  for (int d = 0; d < 3; ++d) u[d * stride + n] += acc[d];
}

// ---------------------------------------------------------------------------
// inlet data and element-wise updates
// ---------------------------------------------------------------------------

// cos(k w t) and sin(k w t) for k = 1..K, evaluated on the host in FP64.
struct Harmonics {
  double c[16], s[16];
  int K;
};

// g_d[id_q] = W_0 + sum_k (Re W_k cos(k w t) - Im W_k sin(k w t)) at table node q.
__global__ __launch_bounds__(kBlock) void k_inlet(int n, const int64_t* __restrict__ ids,
                                                  const double* __restrict__ shape, Harmonics hm,
                                                  double* __restrict__ g, int64_t stride) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= n) return;
  const int64_t blk = int64_t(n) * 3;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double v = shape[3 * q + d];
    for (int k = 1; k <= hm.K; ++k) {
      v += shape[(2 * k - 1) * blk + 3 * q + d] * hm.c[k - 1];
      v -= shape[(2 * k) * blk + 3 * q + d] * hm.s[k - 1];
    }
    g[d * stride + ids[q]] = v;
  }
}

// y = (flags & bit) ? x : 0, nc planes
template <typename TI, typename TO>
__global__ __launch_bounds__(kBlock) void k_masked_copy(NodeList nl,
                                                        const uint8_t* __restrict__ flags, uint32_t bit,
                                                        const TI* __restrict__ x, TO* __restrict__ y,
                                                        int nc, int64_t stride) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  const bool on = flags[n] & bit;
  for (int d = 0; d < nc; ++d) y[d * stride + n] = on ? TO(x[d * stride + n]) : TO(0);
}

// z = a x + b y over all chunk nodes, nc planes
__global__ __launch_bounds__(kBlock) void k_axpby(NodeList nl, double a,
                                                  const double* __restrict__ x, double b,
                                                  const double* __restrict__ y, double* __restrict__ z,
                                                  int nc, int64_t stride) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  for (int d = 0; d < nc; ++d) {
    const int64_t i = d * stride + n;
    z[i] = a * x[i] + b * y[i];
  }
}

// x = 0 on every chunk node (nc planes); positions outside the chunks are never
// written and stay zero from the allocation
template <typename T>
__global__ __launch_bounds__(kBlock) void k_zero(NodeList nl,
                                                 T* __restrict__ x, int nc, int64_t stride) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  for (int d = 0; d < nc; ++d) x[d * stride + n] = T(0);
}

// x = a fixed pseudo-random value in [-1, 1) on rows (a hash of the node id), 0
// elsewhere: a start vector with every spectral component present
__global__ __launch_bounds__(kBlock) void k_fill_hash(NodeList nl, const uint8_t* __restrict__ flags,
                                                      uint32_t rowbit, double* __restrict__ x) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  uint32_t h = uint32_t(n) * 2654435761u;
  h ^= h >> 16;
  h *= 2246822519u;
  h ^= h >> 13;
  x[n] = (flags[n] & rowbit) ? double(h) * (2.0 / 4294967296.0) - 1.0 : 0.0;
}

// x += TO(d) on rows (mixed precision update of an FP64 iterate by an FP32 correction)
template <typename TD>
__global__ __launch_bounds__(kBlock) void k_add_correction(NodeList nl,
                                                           const uint8_t* __restrict__ flags,
                                                           uint32_t bit, const TD* __restrict__ dx,
                                                           double* __restrict__ x, int nc,
                                                           int64_t stride) {
  const int n = chunk_node(nl);
  if (n < 0 || !(flags[n] & bit)) return;
  for (int d = 0; d < nc; ++d) x[d * stride + n] += double(dx[d * stride + n]);
}

// compact (canonical order) <-> dense
__global__ __launch_bounds__(kBlock) void k_scatter(int64_t n, const int64_t* __restrict__ ids,
                                                    const double* __restrict__ comp,
                                                    double* __restrict__ dense, int nc,
                                                    int64_t stride) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= n) return;
  for (int d = 0; d < nc; ++d) dense[d * stride + ids[q]] = comp[d * n + q];
}
__global__ __launch_bounds__(kBlock) void k_gather(int64_t n, const int64_t* __restrict__ ids,
                                                   const double* __restrict__ dense,
                                                   double* __restrict__ comp, int nc, int64_t stride) {
  const int64_t q = int64_t(blockIdx.x) * kBlock + threadIdx.x;
  if (q >= n) return;
  for (int d = 0; d < nc; ++d) comp[d * n + q] = dense[d * stride + ids[q]];
}

// Per-slot partial sums over nodes of outlet-less parts (slot >= 0), then a
// one-block finalize that stores means[s] = sum_s / count_s.
__global__ __launch_bounds__(kBlock) void k_slot_sum(NodeList nl,
                                                     const int8_t* __restrict__ slot,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ partials) {
  double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    const int s = slot[n];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (s == k) v[k] += x[n];
  }
  block_partials<8>(v, partials);
}
__global__ __launch_bounds__(kBlock) void k_fin_slot(const double* __restrict__ partials, int nb,
                                                     int nslots, const double* __restrict__ count,
                                                     double* __restrict__ means) {
  double tot[8];
  sum_partials<8>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  for (int k = 0; k < nslots; ++k) means[k] = tot[k] / count[k];
}
__global__ __launch_bounds__(kBlock) void k_slot_sub(NodeList nl,
                                                     const int8_t* __restrict__ slot,
                                                     double* __restrict__ x,
                                                     const double* __restrict__ means) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  const int s = slot[n];
  if (s >= 0) x[n] -= means[s];
}

}  // namespace ibfe
