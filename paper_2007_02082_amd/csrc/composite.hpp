// gfx950 kernels of the 2:1 locally refined lattice.
//
// Every field lives on the fine lattice (spacing h/2) with the dense padded
// layout of the uniform grid.  The element part of an operator row at node n
// is the uniform matrix-free stencil over the fine elements around n (cell bits
// `emask`, neighbours at lattice offsets +-1) plus the same stencil with the
// coarse element entries over the unrefined cells around n (cell bits `cmask`,
// set on all-even nodes only, neighbours at offsets +-2).  The hanging-node
// constraint u_h = mean of its 2 or 4 parents turns every form A into C^T A C:
//   1. fill   x[h] = mean of x over the parents of h          (x -> C x)
//   2. rows   yh[k] = element row of hanging node h_k on C x  (A C x at h)
//   3. apply  y[n] = element row of n + sum_k w_k yh[k] over the hanging
//             children k of n (the C^T gather), on the rows of P.
// Steps 1 and 2 are small launches over the hanging list; step 3 is the
// chunked row kernel (Krylov kernels call it through the operator's apply).
#pragma once

#include "step_kernels.hpp"

namespace ibfe {

constexpr uint32_t kFlagHang = 32u;  // hanging lattice node
constexpr uint32_t kFlagPar = 64u;   // node of P with hanging children

// Hanging children of parent nodes: CSR by parent slot.
struct Children {
  const int32_t* slot;   // per lattice node (read on parents only)
  const int32_t* ptr;
  const int32_t* child;  // hanging index
  int nh;
};

template <typename T, int NC>
__device__ __forceinline__ void add_children(const Children& ch, const T* __restrict__ w,
                                             const T* __restrict__ yh, int n, T (&y)[NC]) {
  const int s = ch.slot[n];
  for (int q = ch.ptr[s]; q < ch.ptr[s + 1]; ++q) {
    const int k = ch.child[q];
    const T wq = w[q];
#pragma unroll
    for (int d = 0; d < NC; ++d) y[d] += wq * yh[d * ch.nh + k];
  }
}

// alpha M + beta K on the composite mesh: per-cell entries cf (fine, h/2) and
// cc (coarse, h); rows with (flags & rowbit); Jacobi diagonal = the lumped
// constrained diagonal (the hanging children's diagonals added to the parents
// with their weights).
template <typename T, int NC>
struct OpCSym {
  static constexpr int kNC = NC;
  const uint8_t* emask;
  const uint8_t* cmask;
  const uint8_t* flags;
  uint32_t rowbit;
  int sy, sz;
  int64_t stride;
  T cf[4], cc[4];
  const T* dinv;
  Children ch;
  const T* pw;
  const T* yh;
  __device__ __forceinline__ bool row(int n) const { return flags[n] & rowbit; }
  __device__ __forceinline__ void elem(int n, const T* __restrict__ x, T (&y)[NC]) const {
    const uint32_t e = emask[n], m = cmask[n];
    const bool anyf = __any(e != 0u), anyc = __any(m != 0u);
    const T f4[4] = {cf[0], cf[1], cf[2], cf[3]};
    const T c4[4] = {cc[0], cc[1], cc[2], cc[3]};
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      T v = T(0);
      if (anyf) v = apply_sym<T>(x + d * stride, n, e, f4, sy, sz, 1);
      if (anyc) v += apply_sym<T>(x + d * stride, n, m, c4, 2 * sy, 2 * sz, 2);
      y[d] = v;
    }
  }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[NC]) const {
    elem(n, x, y);
    if (flags[n] & kFlagPar) add_children<T, NC>(ch, pw, yh, n, y);
  }
  __device__ __forceinline__ T inv_diag(int n) const { return dinv[n]; }
};

// Stored stencil of the tentative-velocity operator on the composite mesh:
// planes 0..26 hold the fine-element part (offsets +-1), planes 27..53 the
// coarse-element part (offsets +-2), t = (ox+1) + 3 (oy+1) + 9 (oz+1).
template <typename T, int NC>
struct OpCStencil {
  static constexpr int kNC = NC;
  const T* coef;
  const uint8_t* cmask;
  const uint8_t* flags;
  uint32_t rowbit;
  int sy, sz;
  int64_t stride;
  Children ch;
  const T* pw;
  const T* yh;
  __device__ __forceinline__ bool row(int n) const { return flags[n] & rowbit; }
  __device__ __forceinline__ void elem(int n, const T* __restrict__ x, T (&y)[NC]) const {
#pragma unroll
    for (int d = 0; d < NC; ++d) y[d] = T(0);
#pragma unroll
    for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
      for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
        for (int ox = -1; ox <= 1; ++ox) {
          const int t = (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1);
          const T w = coef[t * stride + n];
          const int m = n + ox + sy * oy + sz * oz;
#pragma unroll
          for (int d = 0; d < NC; ++d) y[d] += w * x[d * stride + m];
        }
    if (cmask[n]) {
#pragma unroll
      for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
        for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
          for (int ox = -1; ox <= 1; ++ox) {
            const int t = 27 + (ox + 1) + 3 * (oy + 1) + 9 * (oz + 1);
            const T w = coef[t * stride + n];
            const int m = n + 2 * (ox + sy * oy + sz * oz);
#pragma unroll
            for (int d = 0; d < NC; ++d) y[d] += w * x[d * stride + m];
          }
    }
  }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[NC]) const {
    elem(n, x, y);
    if (flags[n] & kFlagPar) add_children<T, NC>(ch, pw, yh, n, y);
  }
  __device__ __forceinline__ T inv_diag(int n) const {
    return T(1) / (coef[13 * stride + n] + coef[40 * stride + n]);
  }
};

// Element rows of an operator on a fixed input vector (the functor form used
// by the hanging-row and row kernels).
template <typename T, class Op>
struct OpElem {
  static constexpr int kNO = Op::kNC;
  Op op;
  const T* x;
  __device__ __forceinline__ void elem(int n, T (&y)[kNO]) const { op.elem(n, x, y); }
};

// sum_d G_d u_d (weak divergence) on the composite mesh.
struct DivElem {
  static constexpr int kNO = 1;
  const uint8_t* emask;
  const uint8_t* cmask;
  const double* u;
  int64_t stride;
  int sy, sz;
  double gf[3], gc[3];
  __device__ __forceinline__ void elem(int n, double (&y)[1]) const {
    const uint32_t e = emask[n], m = cmask[n];
    double s = 0.0;
    if (e) {
      const double g[3] = {gf[0], gf[1], gf[2]};
      s += apply_grad<double, 0>(u, n, e, g, sy, sz) + apply_grad<double, 1>(u + stride, n, e, g, sy, sz) +
           apply_grad<double, 2>(u + 2 * stride, n, e, g, sy, sz);
    }
    if (m) {
      const double g[3] = {gc[0], gc[1], gc[2]};
      s += apply_grad<double, 0>(u, n, m, g, 2 * sy, 2 * sz, 2) +
           apply_grad<double, 1>(u + stride, n, m, g, 2 * sy, 2 * sz, 2) +
           apply_grad<double, 2>(u + 2 * stride, n, m, g, 2 * sy, 2 * sz, 2);
    }
    y[0] = s;
  }
};

// (G_1 x, G_2 x, G_3 x) on the composite mesh.
struct GradElem {
  static constexpr int kNO = 3;
  const uint8_t* emask;
  const uint8_t* cmask;
  const double* x;
  int sy, sz;
  double gf[3], gc[3];
  __device__ __forceinline__ void elem(int n, double (&y)[3]) const {
    const uint32_t e = emask[n], m = cmask[n];
    y[0] = y[1] = y[2] = 0.0;
    if (e) {
      const double g[3] = {gf[0], gf[1], gf[2]};
      y[0] += apply_grad<double, 0>(x, n, e, g, sy, sz);
      y[1] += apply_grad<double, 1>(x, n, e, g, sy, sz);
      y[2] += apply_grad<double, 2>(x, n, e, g, sy, sz);
    }
    if (m) {
      const double g[3] = {gc[0], gc[1], gc[2]};
      y[0] += apply_grad<double, 0>(x, n, m, g, 2 * sy, 2 * sz, 2);
      y[1] += apply_grad<double, 1>(x, n, m, g, 2 * sy, 2 * sz, 2);
      y[2] += apply_grad<double, 2>(x, n, m, g, 2 * sy, 2 * sz, 2);
    }
  }
};

// (rho/dt) M u_d - G_d p - A g_d (right-hand side of the tentative velocity,
// Eq. 9 with the Dirichlet lifting) on the composite mesh.
// g vanishes off the inlet table, so A g is formed only inside the lattice box
// [lo, hi] (the inlet-table nodes' bounding box widened by 4 lattice steps: a
// coarse element reaches 2 steps, a hanging child's parents 2 more).
template <class AOp = OpCStencil<double, 3>>
struct S1RhsElemT {
  static constexpr int kNO = 3;
  OpCSym<double, 3> mass;     // (rho/dt) M
  AOp A;                      // advection-diffusion operator (stored or matrix-free)
  GradElem grad;              // on p
  const double* u;
  const double* g;
  int lo[3], hi[3];
  __device__ __forceinline__ void elem(int n, double (&y)[3]) const {
    double mu_[3], gp[3], ag[3] = {0.0, 0.0, 0.0};
    mass.elem(n, u, mu_);
    grad.elem(n, gp);
    const int k = n / A.sz, j = (n - k * A.sz) / A.sy, i = n - k * A.sz - j * A.sy;
    if (i >= lo[0] && i <= hi[0] && j >= lo[1] && j <= hi[1] && k >= lo[2] && k <= hi[2]) A.elem(n, g, ag);
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = mu_[d] - gp[d] - ag[d];
  }
};
using S1RhsElem = S1RhsElemT<>;

// Explicit advection on the composite mesh:
// (rho/dt) M u_d - rho C(u^n) u_d - G_d p - A' g_d with A' = (rho/dt) M + mu K.
struct S1RhsExplicitElem {
  static constexpr int kNO = 3;
  OpCSym<double, 3> mass;     // (rho/dt) M
  OpCStencil<double, 3> adv;  // stored rho C(u^n)
  OpCSym<double, 3> aprime;   // (rho/dt) M + mu K
  GradElem grad;              // on p
  const double* u;
  const double* g;
  __device__ __forceinline__ void elem(int n, double (&y)[3]) const {
    double mu_[3], cu[3], gp[3], ag[3];
    mass.elem(n, u, mu_);
    adv.elem(n, u, cu);
    grad.elem(n, gp);
    aprime.elem(n, g, ag);
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = mu_[d] - cu[d] - gp[d] - ag[d];
  }
};

// extra[d][n] = coarse-element part of the row of n plus its hanging children
// (the row terms the z-blocked fine walk does not see), at the listed nodes.
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_comp_extra(int nn, const int32_t* __restrict__ ids, OpCSym<T, NC> op,
                                                       const T* __restrict__ x, T* __restrict__ extra,
                                                       const KScal* sc) {
  if (sc && sc->done) return;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nn) return;
  const int n = ids[k];
  T y[NC];
#pragma unroll
  for (int d = 0; d < NC; ++d) y[d] = T(0);
  const uint32_t m = op.cmask[n];
  if (m) {
    const T c4[4] = {op.cc[0], op.cc[1], op.cc[2], op.cc[3]};
#pragma unroll
    for (int d = 0; d < NC; ++d) y[d] = apply_sym<T>(x + d * op.stride, n, m, c4, 2 * op.sy, 2 * op.sz, 2);
  }
  if (op.flags[n] & kFlagPar) add_children<T, NC>(op.ch, op.pw, op.yh, n, y);
#pragma unroll
  for (int d = 0; d < NC; ++d) extra[d * op.stride + n] = y[d];
}

// x[h] = mean of x over the 2 or 4 parents of hanging node h (nc planes).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_hang_fill(int nh, const int32_t* __restrict__ hang_ids,
                                                      const int32_t* __restrict__ hang_par,
                                                      T* __restrict__ x, int nc, int64_t stride,
                                                      const KScal* sc) {
  if (sc && sc->done) return;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nh) return;
  const int n = hang_ids[k];
  const int p0 = hang_par[k], p1 = hang_par[nh + k], p2 = hang_par[2 * nh + k], p3 = hang_par[3 * nh + k];
  for (int d = 0; d < nc; ++d) {
    const T* xd = x + d * stride;
    const T v = p2 < 0 ? T(0.5) * (xd[p0] + xd[p1]) : T(0.25) * ((xd[p0] + xd[p1]) + (xd[p2] + xd[p3]));
    x[d * stride + n] = v;
  }
}

// yh[d][k] = element row of hanging node k (the input must already be filled).
template <typename T, class F>
__global__ __launch_bounds__(kBlock) void k_hang_elem(int nh, const int32_t* __restrict__ hang_ids, F f,
                                                      T* __restrict__ yh, const KScal* sc) {
  if (sc && sc->done) return;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nh) return;
  T y[F::kNO];
  f.elem(hang_ids[k], y);
#pragma unroll
  for (int d = 0; d < F::kNO; ++d) yh[d * nh + k] = y[d];
}

// out[d][n] = scale * (element row + hanging children) on rows (flags & rowbit,
// none of `exclude`), 0 elsewhere.
template <typename T, class F>
__global__ __launch_bounds__(kBlock) void k_comp_rows(NodeList nl, F f,
                                                      const uint8_t* __restrict__ flags, uint32_t rowbit,
                                                      uint32_t exclude, T scale, Children ch,
                                                      const T* __restrict__ pw, const T* __restrict__ yh,
                                                      T* __restrict__ out, int64_t stride) {
  constexpr int NO = F::kNO;
  const int n = chunk_node(nl);
  if (n < 0) return;
  const uint32_t fl = flags[n];
  const bool rw = (fl & rowbit) && !(fl & exclude);
  T y[NO];
  if (rw) {
    f.elem(n, y);
    if (fl & kFlagPar) add_children<T, NO>(ch, pw, yh, n, y);
  }
#pragma unroll
  for (int d = 0; d < NO; ++d) out[d * stride + n] = rw ? T(scale * y[d]) : T(0);
}

// Chebyshev-Jacobi step on the chunk list for any operator (NC planes):
//   d <- c1 d + c2 D^-1 (b - A x_in), x_out = x_in + d on rows, 0 elsewhere;
// with DOT the partial sums of b . x_out.
template <typename T, class Op, bool DOT>
__global__ __launch_bounds__(kBlock) void k_cheb_gen(NodeList nl, Op op,
                                                     const T* __restrict__ x_in, const T* __restrict__ b,
                                                     T* __restrict__ d, T* __restrict__ x_out, T c1, T c2,
                                                     double* __restrict__ partials, const KScal* sc) {
  if (sc && sc->done) return;
  constexpr int NC = Op::kNC;
  double dot[1] = {0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    const bool rw = op.row(n);
    T y[NC];
    if (rw) op.apply(n, x_in, y);
    const T di = rw ? op.inv_diag(n) : T(0);
#pragma unroll
    for (int q = 0; q < NC; ++q) {
      const int64_t i = q * op.stride + n;
      if (rw) {
        const T dold = (c1 != T(0)) ? d[i] : T(0);
        const T dn = c1 * dold + c2 * di * (b[i] - y[q]);
        const T xn = x_in[i] + dn;
        d[i] = dn;
        x_out[i] = xn;
        if (DOT) dot[0] += double(b[i]) * double(xn);
      } else {
        d[i] = T(0);
        x_out[i] = T(0);
      }
    }
  }
  if (DOT) block_partials<1>(dot, partials);
}

// x = d = c2 D^-1 b on rows (Chebyshev step from x = 0), 0 elsewhere.
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_cheb0_gen(NodeList nl, Op op,
                                                      const T* __restrict__ b, T* __restrict__ d,
                                                      T* __restrict__ x, T c2, const KScal* sc) {
  if (sc && sc->done) return;
  const int n = chunk_node(nl);
  if (n < 0) return;
  const bool rw = op.row(n);
  const T di = rw ? op.inv_diag(n) : T(0);
#pragma unroll
  for (int q = 0; q < Op::kNC; ++q) {
    const int64_t i = q * op.stride + n;
    const T v = rw ? T(c2 * b[i] * di) : T(0);
    d[i] = v;
    x[i] = v;
  }
}

// r = b - A x on rows, 0 elsewhere (multigrid residual on the composite level).
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_resid_gen(NodeList nl, Op op,
                                                      const T* __restrict__ x, const T* __restrict__ b,
                                                      T* __restrict__ r, const KScal* sc) {
  if (sc && sc->done) return;
  const int n = chunk_node(nl);
  if (n < 0) return;
  const bool rw = op.row(n);
  T y[Op::kNC];
  if (rw) op.apply(n, x, y);
#pragma unroll
  for (int q = 0; q < Op::kNC; ++q) {
    const int64_t i = q * op.stride + n;
    r[i] = rw ? T(b[i] - y[q]) : T(0);
  }
}

}  // namespace ibfe
