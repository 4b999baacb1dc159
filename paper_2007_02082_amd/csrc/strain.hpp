// Strain-rate viscous form on the masked uniform grid.
//
// The viscous stress of the momentum equation (Section 2.1) in the form
// 2 mu (eps(u), eps(v)), eps(u) = (grad u + grad u^T)/2, equals the
// component-wise mu (grad u, grad v) plus the cross blocks
//   mu X_dc,   (X_dc)_{n, n+o} = sum over the kept cells shared by n and n + o of
//              int d_c N_n d_d N_{n+o}
// between test component d and trial component c.  On a cube of side h the
// entry is a product of 1-D integrals: int phi_i' phi_j = s_i / 2 (s_0 = -1,
// s_1 = +1) in the direction of the test derivative, int phi_i phi_j' = s_j / 2
// in the direction of the trial derivative, int phi_i' phi_j' = s_i s_j / h when
// both derivatives share a direction, and the 1-D mass h/3 or h/6 in the rest.
// With the cell bits of emask (bit s = sx + 2 sy + 4 sz: the cell on side s of
// the node), the node's local coordinate in cell s is 1 - s along each axis, so
// every sign is a function of o and of the side bits, and the sums over shared
// cells are popcounts of emask & compat(o) restricted to sides.
#pragma once

#include "composite.hpp"

namespace ibfe {

// sum over the cells in S of (1 - 2 s_a) (1 - 2 s_b) for axes a != b
__device__ __forceinline__ int side_pair_sum(uint32_t S, int a, int b) {
  const uint32_t a0 = S & side_mask(a, -1), a1 = S & side_mask(a, 1);
  const uint32_t b0 = side_mask(b, -1);
  return __builtin_popcount(a0 & b0) - __builtin_popcount(a0 & ~b0) - __builtin_popcount(a1 & b0) +
         __builtin_popcount(a1 & ~b0);
}

// y_d += mu sum_c sum_o w_dc(o) x_c(n + o) over the 27 neighbours (the cross
// blocks X_dc of the strain-rate form, including d = c); with STENCIL also
// y_d += coef_t(n) x_d(n + o), the stored stencil of plane t (one pass over the
// neighbours: each value of x is loaded once).  With FULL every cell around the
// node is kept: the cell sets are then compile-time constants and the weights
// fold to constants times h.
template <typename T, bool FULL, bool STENCIL>
__device__ __forceinline__ void strain_cross_body(const T* __restrict__ x, int64_t stride, int n, uint32_t e,
                                                  T mu, T h, int sy, int sz, const T* __restrict__ coef,
                                                  T (&y)[3], int st) {
  const T m3 = h / T(3), m6 = h / T(6);
#pragma unroll
  for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        const uint32_t S = FULL ? compat(ox, oy, oz) : e & compat(ox, oy, oz);
        if (!STENCIL && S == 0u) continue;
        const int o[3] = {ox, oy, oz};
        const int m = n + st * ox + sy * oy + sz * oz;
        const T xv[3] = {x[m], x[stride + m], x[2 * stride + m]};
        if (STENCIL) {
          const T w0 = coef[((ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)) * stride + n];
#pragma unroll
          for (int d = 0; d < 3; ++d) y[d] += w0 * xv[d];
        }
        const int cnt = __builtin_popcount(S);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          T acc = T(0);
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            T w;
            if (c == d) {
              // int d_d N_n d_d N_{n+o}: (s s' / h) times the 1-D masses across
              T mm = T(1);
#pragma unroll
              for (int f = 0; f < 3; ++f)
                if (f != d) mm *= o[f] != 0 ? m6 : m3;
              w = T(o[d] != 0 ? -cnt : cnt) * mm / h;
            } else {
              const int f = 3 - c - d;  // the remaining axis
              int sum;
              if (o[c] != 0 && o[d] != 0) {
                sum = -o[c] * o[d] * cnt;
              } else if (o[c] != 0) {
                sum = -o[c] * (__builtin_popcount(S & side_mask(d, -1)) - __builtin_popcount(S & side_mask(d, 1)));
              } else if (o[d] != 0) {
                sum = o[d] * (__builtin_popcount(S & side_mask(c, -1)) - __builtin_popcount(S & side_mask(c, 1)));
              } else {
                sum = side_pair_sum(S, c, d);
              }
              w = T(sum) * (o[f] != 0 ? m6 : m3) / T(4);
            }
            acc += w * xv[c];
          }
          y[d] += mu * acc;
        }
      }
}

// st = 2 with doubled sy, sz and the coarse h: the unrefined cells of a refined
// lattice (corners at even lattice positions).
template <typename T, bool STENCIL>
__device__ __forceinline__ void apply_strain_cross(const T* __restrict__ x, int64_t stride, int n, uint32_t e,
                                                   T mu, T h, int sy, int sz, const T* __restrict__ coef,
                                                   T (&y)[3], int st = 1) {
  if (__all(e == 0xFFu))
    strain_cross_body<T, true, STENCIL>(x, stride, n, e, mu, h, sy, sz, coef, y, st);
  else
    strain_cross_body<T, false, STENCIL>(x, stride, n, e, mu, h, sy, sz, coef, y, st);
}

// The stored tentative-velocity stencil (identical for the three components)
// plus the strain-rate cross blocks; Jacobi diagonal of the stored stencil (a
// preconditioner only: the block diagonals mu X_dd are left out of it).
template <typename T>
struct OpStencilStrain {
  static constexpr int kNC = 3;
  OpStencil<T, 3> base;
  const uint8_t* emask;
  T mu, h;
  int64_t stride;
  __device__ __forceinline__ bool row(int n) const { return base.row(n); }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[3]) const {
    y[0] = y[1] = y[2] = T(0);
    apply_strain_cross<T, true>(x, stride, n, emask[n], mu, h, base.sy, base.sz, base.coef, y);
  }
  __device__ __forceinline__ T inv_diag(int n) const { return base.inv_diag(n); }
};

// (rho/dt) M + mu K (identical components, explicit advection) plus the
// strain-rate cross blocks: symmetric positive definite, so CG applies.
template <typename T>
struct OpSymStrain {
  static constexpr int kNC = 3;
  OpSym<T, 3> base;
  const uint8_t* emask;
  T mu, h;
  int64_t stride;
  __device__ __forceinline__ bool row(int n) const { return base.row(n); }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[3]) const {
    base.apply(n, x, y);
    apply_strain_cross<T, false>(x, stride, n, emask[n], mu, h, base.sy, base.sz, nullptr, y);
  }
  __device__ __forceinline__ T inv_diag(int n) const { return base.inv_diag(n); }
};

// The composite tentative-velocity operator (the stored 54-plane stencil, or
// the matrix-free form with the same member names) plus the strain-rate cross
// blocks of the fine cells (stride 1, h/2) and of the unrefined cells (stride
// 2, h); the hanging constraint enters through the element rows as for
// OpCStencil.
template <typename T, class Base = OpCStencil<T, 3>>
struct OpCStencilStrain {
  static constexpr int kNC = 3;
  Base base;
  const uint8_t* emask;
  T mu, hf, hc;
  int64_t stride;
  const T* yh;  // the hanging rows (base.yh), filled before every apply
  __device__ __forceinline__ bool row(int n) const { return base.row(n); }
  __device__ __forceinline__ void elem(int n, const T* __restrict__ x, T (&y)[3]) const {
    base.elem(n, x, y);
    apply_strain_cross<T, false>(x, stride, n, emask[n], mu, hf, base.sy, base.sz, nullptr, y, 1);
    const uint32_t m = base.cmask[n];
    if (__any(m != 0u))
      apply_strain_cross<T, false>(x, stride, n, m, mu, hc, 2 * base.sy, 2 * base.sz, nullptr, y, 2);
  }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[3]) const {
    elem(n, x, y);
    if (base.flags[n] & kFlagPar) add_children<T, 3>(base.ch, base.pw, base.yh, n, y);
  }
  __device__ __forceinline__ T inv_diag(int n) const { return base.inv_diag(n); }
};

// The composite symmetric (rho/dt) M + mu K (explicit advection) plus the
// strain-rate cross blocks of the fine and the unrefined cells: symmetric
// positive definite on the constrained space, so CG applies.
template <typename T>
struct OpCSymStrain {
  static constexpr int kNC = 3;
  OpCSym<T, 3> base;
  T mu, hf, hc;
  int64_t stride;
  const T* yh;  // the hanging rows (base.yh), filled before every apply
  __device__ __forceinline__ bool row(int n) const { return base.row(n); }
  __device__ __forceinline__ void elem(int n, const T* __restrict__ x, T (&y)[3]) const {
    base.elem(n, x, y);
    apply_strain_cross<T, false>(x, base.stride, n, base.emask[n], mu, hf, base.sy, base.sz, nullptr, y, 1);
    const uint32_t m = base.cmask[n];
    if (__any(m != 0u))
      apply_strain_cross<T, false>(x, base.stride, n, m, mu, hc, 2 * base.sy, 2 * base.sz, nullptr, y, 2);
  }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[3]) const {
    elem(n, x, y);
    if (base.flags[n] & kFlagPar) add_children<T, 3>(base.ch, base.pw, base.yh, n, y);
  }
  __device__ __forceinline__ T inv_diag(int n) const { return base.inv_diag(n); }
};

// Right-hand side of the tentative velocity with the strain-rate form on the
// refined lattice: the element rows of Rhs (S1RhsElem or S1RhsExplicitElem)
// minus mu sum_c (X_dc g_c) (the cross blocks of the fine and the unrefined
// cells applied to the Dirichlet data).
template <typename Rhs>
struct S1RhsStrainElem {
  static constexpr int kNO = 3;
  Rhs base;
  const uint8_t* emask;
  const uint8_t* cmask;
  double mu, hf, hc;
  int sy, sz;
  int64_t stride;
  __device__ __forceinline__ void elem(int n, double (&y)[3]) const {
    base.elem(n, y);
    double ys[3] = {0.0, 0.0, 0.0};
    apply_strain_cross<double, false>(base.g, stride, n, emask[n], mu, hf, sy, sz, nullptr, ys, 1);
    const uint32_t m = cmask[n];
    if (__any(m != 0u))
      apply_strain_cross<double, false>(base.g, stride, n, m, mu, hc, 2 * sy, 2 * sz, nullptr, ys, 2);
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] -= ys[d];
  }
};

// b_d -= mu sum_c (X_dc g_c) on the listed rows (the strain-rate part of the
// lifting of the Dirichlet data in the tentative-velocity right-hand side; the
// free rows with an inlet-table node among their neighbours).
__global__ __launch_bounds__(kBlock) void k_strain_lift(int nrows, const int32_t* __restrict__ rows,
                                                        const uint8_t* __restrict__ emask,
                                                        const double* __restrict__ g, double* __restrict__ b,
                                                        int64_t stride, double mu, double h, int sy, int sz) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= nrows) return;
  const int n = rows[q];
  double y[3] = {0.0, 0.0, 0.0};
  apply_strain_cross<double, false>(g, stride, n, emask[n], mu, h, sy, sz, nullptr, y);
#pragma unroll
  for (int d = 0; d < 3; ++d) b[d * stride + n] -= y[d];
}

}  // namespace ibfe
