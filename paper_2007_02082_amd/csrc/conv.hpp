// Matrix-free tentative-velocity operator A = (rho/dt) M + rho C(u^n) + mu K
// (Section 2.2, Eq. 9) on the masked uniform grid and on the 2:1 refined lattice.
//
// The row of node n is formed on the fly from the cell bits around n and the
// advecting velocity w = u^n at the 27 neighbours: the constant per-cell
// entries of alpha M + beta K times the number of kept cells a neighbour shares
// with n, plus the Galerkin convection
//   C_nj = sum_{kept cells} sum_d sum_c w_d(c) int N_n N_c d_d N_j.
// On a cube of side h the integral is h^2 times a product of 1-D integrals over
// [0, 1]: int l_a l_c l_j = 1/4 when a = c = j, else 1/12; int l_a l_c l_j' =
// sign(l_j') (1/3 if a = c, else 1/6).  Where all 8 cells around n are kept
// (every lane of the wavefront), the sum over the cells factorises per axis and
// the 27 entries follow from three 1-D passes over the 3 x 3 x 3 block of each
// component of w (about 330 operations per row).  Elsewhere each kept cell is
// taken on its own: per direction d the sum over its 8 corners is contracted
// along d with the derivative weights (1/3, 1/6), then along the two other axes
// with the 2 x 2 triple-mass weights (24 multiply-adds per cell and direction).
// Nothing is stored between applies; the 27 neighbour values of each field are
// loaded from nine row bases.
#pragma once

#include "strain.hpp"
#include "zblock.hpp"

namespace ibfe {

// A[t] = c[type(o_t)] * (kept cells of e shared with the neighbour at offset o_t),
// t = (ox+1) + 3 (oy+1) + 9 (oz+1): the symmetric alpha M + beta K part.
template <typename T>
__device__ __forceinline__ void sym_row(uint32_t e, const T (&c)[4], T (&A)[27]) {
#pragma unroll
  for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        const int type = (ox != 0) + (oy != 0) + (oz != 0);
        A[(ox + 1) + 3 * (oy + 1) + 9 * (oz + 1)] = c[type] * T(__builtin_popcount(e & compat(ox, oy, oz)));
      }
}

// the 1-D weights in the operator's precision
template <typename T>
__device__ __forceinline__ constexpr T mass3(int li, int c, int j) {
  return (li == c && c == j) ? T(0.25) : T(1) / T(12);
}
template <typename T>
__device__ __forceinline__ constexpr T deriv2(int li, int c) {
  return li == c ? T(1) / T(3) : T(1) / T(6);
}

// The 27 values of x around n (offset t = (ox+1) + 3 (oy+1) + 9 (oz+1), x
// offsets of st lattice steps): nine row bases, the x neighbours as immediate
// offsets of each.
template <typename T>
__device__ __forceinline__ void load27(const T* __restrict__ x, int n, int sy, int sz, int st, T (&v)[27]) {
#pragma unroll
  for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy) {
      const T* row = x + (n + oy * sy + oz * sz);
      const int b = 3 * (oy + 1) + 9 * (oz + 1);
      v[b] = row[-st];
      v[b + 1] = row[0];
      v[b + 2] = row[st];
    }
}

// A[t] += rh2 * C_{n, n+o_t} over the cells of e, from the neighbour values
// wd of component d of w.
template <typename T>
__device__ __forceinline__ void conv_cells_dir(const T (&wd)[27], int d, uint32_t e, T rh2, T (&A)[27]) {
  const int q1 = (d + 1) % 3, q2 = (d + 2) % 3;
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    if (!((e >> s) & 1u)) continue;
    // local coordinate of n in cell s (the cell on side s of n)
    const int li[3] = {1 - (s & 1), 1 - ((s >> 1) & 1), 1 - ((s >> 2) & 1)};
    // corner c of the cell is the neighbour at offset lc - li
    auto wc = [&](int c) -> T {
      return wd[((c & 1) - li[0] + 1) + 3 * (((c >> 1) & 1) - li[1] + 1) + 9 * (((c >> 2) & 1) - li[2] + 1)];
    };
    // along d: v[i1][i2] = sum_{c_d} w_d * (1/3 or 1/6)
    T v[2][2];
#pragma unroll
    for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2) {
        const int c0 = (i1 << q1) | (i2 << q2), c1 = c0 | (1 << d);
        v[i1][i2] = wc(c0) * deriv2<T>(li[d], 0) + wc(c1) * deriv2<T>(li[d], 1);
      }
    // along q1, then q2: P[j1][j2]
    T u[2][2];
#pragma unroll
    for (int j1 = 0; j1 < 2; ++j1)
#pragma unroll
      for (int i2 = 0; i2 < 2; ++i2)
        u[j1][i2] = v[0][i2] * mass3<T>(li[q1], 0, j1) + v[1][i2] * mass3<T>(li[q1], 1, j1);
#pragma unroll
    for (int j1 = 0; j1 < 2; ++j1)
#pragma unroll
      for (int j2 = 0; j2 < 2; ++j2) {
        const T pv = rh2 * (u[j1][0] * mass3<T>(li[q2], 0, j2) + u[j1][1] * mass3<T>(li[q2], 1, j2));
#pragma unroll
        for (int jd = 0; jd < 2; ++jd) {
          int lj[3];
          lj[d] = jd;
          lj[q1] = j1;
          lj[q2] = j2;
          const int t = (lj[0] - li[0] + 1) + 3 * (lj[1] - li[1] + 1) + 9 * (lj[2] - li[2] + 1);
          A[t] += jd ? pv : -pv;
        }
      }
  }
}

// All 8 cells kept: the sum over the cells factorises per axis.  Summed over
// the two cells on either side of n, the 1-D weights between a velocity offset
// q and a trial offset j (rows q = -1, 0, 1; columns j) are
//   mass  (1/12) [[1, 1, 0], [1, 6, 1], [0, 1, 1]],
//   deriv (1/6)  [[-1, 1, 0], [-2, 0, 2], [0, -1, 1]],
// so C = sum_d (W_x (x) W_y (x) W_z) w_d with W = deriv along d and mass across:
// three 1-D passes (in place) over the 3 x 3 x 3 block per direction, the
// scale 1/864 and rho h^2 applied once at the end.
template <int AX>
__device__ __forceinline__ constexpr int line_idx(int l, int k) {
  return AX == 0 ? k + 3 * (l % 3) + 9 * (l / 3) : AX == 1 ? (l % 3) + 3 * k + 9 * (l / 3) : (l % 3) + 3 * (l / 3) + 9 * k;
}
template <typename T, int AX>
__device__ __forceinline__ void pass_mass(T (&v)[27]) {
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const T a = v[line_idx<AX>(l, 0)], b = v[line_idx<AX>(l, 1)], c = v[line_idx<AX>(l, 2)];
    v[line_idx<AX>(l, 0)] = a + b;
    v[line_idx<AX>(l, 1)] = T(6) * b + (a + c);
    v[line_idx<AX>(l, 2)] = b + c;
  }
}
template <typename T, int AX>
__device__ __forceinline__ void pass_deriv(T (&v)[27]) {
#pragma unroll
  for (int l = 0; l < 9; ++l) {
    const T a = v[line_idx<AX>(l, 0)], b = v[line_idx<AX>(l, 1)], c = v[line_idx<AX>(l, 2)];
    v[line_idx<AX>(l, 0)] = -(T(2) * b + a);
    v[line_idx<AX>(l, 1)] = a - c;
    v[line_idx<AX>(l, 2)] = T(2) * b + c;
  }
}

// Full row of A at n over the cells e: symmetric part plus convection, w read
// one component at a time (27 values live).
template <typename T>
__device__ __forceinline__ void advdiff_row(const T* __restrict__ w, int64_t stride, int n, uint32_t e,
                                            const T (&c)[4], T rh2, int sy, int sz, int st, T (&A)[27]) {
  if (__all(e == 0xFFu)) {
    sym_row<T>(0xFFu, c, A);
    T s[27], b[27];
    load27<T>(w + stride, n, sy, sz, st, s);      // w_y: mass z, deriv y
    pass_mass<T, 2>(s);
    pass_deriv<T, 1>(s);
    load27<T>(w + 2 * stride, n, sy, sz, st, b);  // w_z: deriv z, mass y
    pass_deriv<T, 2>(b);
    pass_mass<T, 1>(b);
#pragma unroll
    for (int t = 0; t < 27; ++t) s[t] += b[t];
    pass_mass<T, 0>(s);                           // both: mass x
    load27<T>(w, n, sy, sz, st, b);               // w_x: mass z, mass y, deriv x
    pass_mass<T, 2>(b);
    pass_mass<T, 1>(b);
    pass_deriv<T, 0>(b);
    const T k = rh2 * (T(1) / T(864));
#pragma unroll
    for (int t = 0; t < 27; ++t) A[t] += k * (s[t] + b[t]);
  } else {
    sym_row<T>(e, c, A);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T wd[27];
      load27<T>(w + d * stride, n, sy, sz, st, wd);
      conv_cells_dir<T>(wd, d, e, rh2, A);
    }
  }
}

template <typename T, int NC>
__device__ __forceinline__ void row_apply(const T (&A)[27], const T* __restrict__ x, int64_t stride, int n,
                                          int sy, int sz, int st, T (&y)[NC]) {
#pragma unroll
  for (int d = 0; d < NC; ++d) {
    T v[27];
    load27<T>(x + d * stride, n, sy, sz, st, v);
    T acc = y[d];
#pragma unroll
    for (int t = 0; t < 27; ++t) acc += A[t] * v[t];
    y[d] = acc;
  }
}

// The operator on the uniform grid (rows with flags & rowbit); the three
// components share it.  w holds u^n in the operator's precision, dinv the
// inverse Jacobi diagonal of the rows.
template <typename T>
struct OpConv {
  static constexpr int kNC = 3;
  const uint8_t* emask;
  const uint8_t* flags;
  uint32_t rowbit;
  int sy, sz;
  int64_t stride;
  T c[4];
  T rh2;
  const T* w;
  const T* dinv;
  __device__ __forceinline__ bool row(int n) const { return flags[n] & rowbit; }
  __device__ __forceinline__ void coefs(int n, T (&A)[27]) const {
    const T cc[4] = {c[0], c[1], c[2], c[3]};
    advdiff_row<T>(w, stride, n, emask[n], cc, rh2, sy, sz, 1, A);
  }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[3]) const {
    T A[27];
    coefs(n, A);
    y[0] = y[1] = y[2] = T(0);
    row_apply<T, 3>(A, x, stride, n, sy, sz, 1, y);
  }
  __device__ __forceinline__ T inv_diag(int n) const { return dinv[n]; }
};

// The operator on the refined lattice: fine cells (emask, spacing h/2,
// neighbours at +-1) plus unrefined cells (cmask on all-even nodes, spacing h,
// neighbours at +-2), and the hanging constraint C^T A C through the hanging
// rows yh as for the stored stencil (the member names match OpCStencil, so the
// strain-rate wrapper takes either).
template <typename T>
struct OpCConv {
  static constexpr int kNC = 3;
  const uint8_t* emask;
  const uint8_t* cmask;
  const uint8_t* flags;
  uint32_t rowbit;
  int sy, sz;
  int64_t stride;
  T cf[4], cc[4];
  T rh2f, rh2c;
  const T* w;
  const T* dinv;
  Children ch;
  const T* pw;
  const T* yh;
  // with extra: the coarse-cell part and the hanging children of the rows flagged
  // kFlagExtra (about 7 % of them) precomputed there by k_conv_extra before the
  // apply, so the other rows' wavefronts skip them; without: both in the row
  const T* extra = nullptr;
  __device__ __forceinline__ bool row(int n) const { return flags[n] & rowbit; }
  __device__ __forceinline__ void elem(int n, const T* __restrict__ x, T (&y)[3]) const {
    y[0] = y[1] = y[2] = T(0);
    const uint32_t e = emask[n], m = cmask[n];
    if (__any(e != 0u)) {
      T A[27];
      const T c4[4] = {cf[0], cf[1], cf[2], cf[3]};
      advdiff_row<T>(w, stride, n, e, c4, rh2f, sy, sz, 1, A);
      row_apply<T, 3>(A, x, stride, n, sy, sz, 1, y);
    }
    if (!extra && __any(m != 0u)) coarse(n, m, x, y);
  }
  __device__ __forceinline__ void coarse(int n, uint32_t m, const T* __restrict__ x, T (&y)[3]) const {
    T A[27];
    const T c4[4] = {cc[0], cc[1], cc[2], cc[3]};
    advdiff_row<T>(w, stride, n, m, c4, rh2c, 2 * sy, 2 * sz, 2, A);
    row_apply<T, 3>(A, x, stride, n, 2 * sy, 2 * sz, 2, y);
  }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[3]) const {
    elem(n, x, y);
    if (extra) {
      if (flags[n] & kFlagExtra) {
#pragma unroll
        for (int d = 0; d < 3; ++d) y[d] += extra[d * stride + n];
      }
    } else if (flags[n] & kFlagPar) {
      add_children<T, 3>(ch, pw, yh, n, y);
    }
  }
  __device__ __forceinline__ T inv_diag(int n) const { return dinv[n]; }
};

// extra[d][n] = coarse-cell part of the row of n plus its hanging children's rows
// (yh, filled before) at the listed nodes (those flagged kFlagExtra).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_conv_extra(int nn, const int32_t* __restrict__ ids, OpCConv<T> op,
                                                       const T* __restrict__ x, T* __restrict__ extra,
                                                       const KScal* sc) {
  if (sc && sc->done) return;
  const int k = blockIdx.x * kBlock + threadIdx.x;
  if (k >= nn) return;
  const int n = ids[k];
  T y[3] = {T(0), T(0), T(0)};
  const uint32_t m = op.cmask[n];
  if (m) op.coarse(n, m, x, y);
  if (op.flags[n] & kFlagPar) add_children<T, 3>(op.ch, op.pw, op.yh, n, y);
#pragma unroll
  for (int d = 0; d < 3; ++d) extra[d * op.stride + n] = y[d];
}

// The matrix-free operator plus the strain-rate cross blocks (uniform grid);
// the Jacobi diagonal leaves the block diagonals mu X_dd out, as for the stored
// stencil.
template <typename T>
struct OpConvStrain {
  static constexpr int kNC = 3;
  OpConv<T> base;
  T mu, h;
  int64_t stride;
  __device__ __forceinline__ bool row(int n) const { return base.row(n); }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[3]) const {
    base.apply(n, x, y);
    apply_strain_cross<T, false>(x, stride, n, base.emask[n], mu, h, base.sy, base.sz, nullptr, y);
  }
  __device__ __forceinline__ T inv_diag(int n) const { return base.inv_diag(n); }
};

// Once per step: the advecting velocity u^n copied into the buffers the
// operators read (FP64, and FP32 when w32 is set; every node of P and every
// hanging node, Dirichlet nodes included; fixed buffers, where u itself
// alternates between two, so captured solver graphs stay valid), and the
// inverse Jacobi diagonal of the rows (FP64, and its FP32 rounding when dinv32
// is set) from u^n.
template <class Op64>
__global__ __launch_bounds__(kBlock) void k_conv_prep(NodeList nl, Op64 op, const double* __restrict__ u,
                                                      double* __restrict__ w64, float* __restrict__ w32,
                                                      double* __restrict__ dinv64, float* __restrict__ dinv32) {
  const int n = chunk_node(nl);
  // inactive lattice nodes: no kept cell has them as a corner, so no row reads them
  if (n < 0 || !(op.op.flags[n] & (kFlagP | kFlagHang))) return;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double v = u[d * op.stride + n];
    w64[d * op.stride + n] = v;
    if (w32) w32[d * op.stride + n] = float(v);
  }
  double inv = 0.0;
  if (op.row(n)) {
    double dg = 0.0;
    op.diag_entry(n, dg);
    inv = 1.0 / dg;
  }
  dinv64[n] = inv;
  if (dinv32) dinv32[n] = float(inv);
}

// Convection diagonal C_nn / (rho h^2) over the cells of e: per kept cell and
// direction d, the 8 corner values of w_d with the weights of the trial node n
// itself (the sign of its derivative is + when n is the cell's upper corner
// along d).
template <typename T>
__device__ __forceinline__ T conv_diag(const T* __restrict__ w, int64_t stride, int n, uint32_t e, int sy,
                                       int sz, int st) {
  T acc = T(0);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T wd[27];
    load27<T>(w + d * stride, n, sy, sz, st, wd);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (!((e >> s) & 1u)) continue;
      const int li[3] = {1 - (s & 1), 1 - ((s >> 1) & 1), 1 - ((s >> 2) & 1)};
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int lc[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        T wt = (li[d] == 1 ? T(1) : T(-1)) * deriv2<T>(li[d], lc[d]);
#pragma unroll
        for (int q = 0; q < 3; ++q)
          if (q != d) wt *= mass3<T>(li[q], lc[q], li[q]);
        acc += wt * wd[(lc[0] - li[0] + 1) + 3 * (lc[1] - li[1] + 1) + 9 * (lc[2] - li[2] + 1)];
      }
    }
  }
  return acc;
}

// Diagonal entries of the rows (fine plus coarse part on a refined lattice).
template <typename T>
struct ConvDiag {
  OpConv<T> op;
  int64_t stride;
  __device__ __forceinline__ bool row(int n) const { return op.row(n); }
  __device__ __forceinline__ void diag_entry(int n, double& dg) const {
    const uint32_t e = op.emask[n];
    dg = double(op.c[0] * T(__builtin_popcount(e)) +
                op.rh2 * conv_diag<T>(op.w, op.stride, n, e, op.sy, op.sz, 1));
  }
};
template <typename T>
struct CConvDiag {
  OpCConv<T> op;
  int64_t stride;
  __device__ __forceinline__ bool row(int n) const { return op.row(n); }
  __device__ __forceinline__ void diag_entry(int n, double& dg) const {
    const uint32_t e = op.emask[n], m = op.cmask[n];
    T s = op.cf[0] * T(__builtin_popcount(e)) + op.rh2f * conv_diag<T>(op.w, op.stride, n, e, op.sy, op.sz, 1);
    if (m) s += op.cc[0] * T(__builtin_popcount(m)) +
                op.rh2c * conv_diag<T>(op.w, op.stride, n, m, 2 * op.sy, 2 * op.sz, 2);
    dg = double(s);
  }
};

// b_d -= (A g)_d on the listed rows (the lifting of the Dirichlet data, zero off
// the inlet table): the rows of `rows` only, the operator's own row formula.
template <class Op>
__global__ __launch_bounds__(kBlock) void k_lift_rows(int nrows, const int32_t* __restrict__ rows, Op A,
                                                      const double* __restrict__ g, double* __restrict__ b) {
  const int q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= nrows) return;
  const int n = rows[q];
  double ag[3];
  A.apply(n, g, ag);
#pragma unroll
  for (int d = 0; d < 3; ++d) b[d * A.stride + n] -= ag[d];
}

// The FP32 apply of the refined lattice (fine part only: the flagged rows' extra
// terms come precomputed) fits in 128 VGPRs with a few spills: four waves per
// SIMD instead of three, 170 -> 162 us on the refined aneurysm.  The uniform
// grid's needs 145; squeezed into 128 it spills 27 registers and runs at half
// the speed, so it keeps three.
template <>
struct ApplyWaves<OpCConv<float>> {
  static constexpr int value = 4;
};

}  // namespace ibfe
