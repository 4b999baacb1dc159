// Z-blocked matrix-free apply of the symmetric masked Q1 forms (alpha M + beta K).
//
// A wavefront owns one "column item": 64 in-plane positions (ascending, mostly
// runs of consecutive x, where some plane of the item holds a kept cell) and
// walks them up through the item's planes (at most kZB).  A 3-plane sliding window of the 3x3 (y, x) neighbour
// rows stays in registers, so each output node costs 9 coalesced row loads
// instead of 27 gathers, and the y/z row addresses are shared by the x shifts.
// When every lane of the wavefront sits in the interior (all 8 cells kept) the
// constant 27-point stencil is used; otherwise the per-neighbour kept-cell
// counts are evaluated.  The per-node result is handed to an epilogue (CG
// product with dot, residual, Chebyshev smoothing step).
#pragma once

#include "kernels.hpp"

namespace ibfe {

constexpr int kZB = 8;

// Node whose operator row has terms beyond the fine cells of its emask (on a
// refined lattice: unrefined cells around it, or hanging children); their sum
// is precomputed into op.extra before the walk.
constexpr uint32_t kFlagExtra = 128u;

// Symmetric masked operator of one grid level.
template <typename T>
struct ZOp {
  const uint8_t* emask;
  const uint8_t* flags;
  uint32_t rowbit;
  int sy, sz, nplanes;
  T c[4];
  int zb;             // planes per column item (<= kZB)
  const int* lanes;   // 64 in-plane positions per item, -1 = none
  // refined lattice: inverse Jacobi diagonal per node (else c[0] x kept cells)
  // and the precomputed extra terms of kFlagExtra rows (planes of the field stride)
  const T* dinv = nullptr;
  const T* extra = nullptr;
  // the cell bits and flags of the walked positions in walk order (item, plane,
  // lane: one coalesced 64-byte load per plane), or nullptr to read them from
  // the lattice arrays
  const uint8_t* em_im = nullptr;
  const uint8_t* fl_im = nullptr;
};

// Walk order: position (item it, plane k of the item, lane) has index
// (it * zb + k) * 64 + lane.  Vectors that the walks read and write only at the
// walked node itself can live in this order (dense, whole cache lines) instead
// of on the lattice, where a vessel's columns fill part of each line.

// Walk the column items of this block.  The 3-plane window slides through a ring of kZBPF + 3 planes: the row loads of
// the plane kZBPF + 1 steps ahead are issued before the current output is formed,
// so each wavefront keeps 9 (kZBPF + 1) row loads in flight while computing, and
// the window takes 9 (kZBPF + 3) registers instead of 9 (kZB + 2) (more waves per
// SIMD to hide the memory latency).
constexpr int kZBPF = 2;

// A wavefront walks its item once per component (planes of `stride`): the cell
// bits and flags of the item stay in its caches.  (Spreading the (item,
// component) pairs over different wavefronts was measured slower: 32 -> 35 us
// for the pulsatile mass step.)
// epi(component, node, lane_ok, row, emask, Ax, x_centre, extra_row, walk-order index).
// zb_walk_range walks the items [cr.c0, cr.c1); zb_walk, this block's share of
// all nitems items.
template <typename T, int NC, class Epi>
__device__ __forceinline__ void zb_walk_range(const int* __restrict__ items, ChunkRange cr, const ZOp<T>& op,
                                              const T* __restrict__ x0, int64_t stride, Epi& epi,
                                              const T* __restrict__ extra0 = nullptr) {
  constexpr int R = kZBPF + 3;
  const int lane = threadIdx.x & 63;
  const int sy = op.sy, sz = op.sz;
  const T c[4] = {op.c[0], op.c[1], op.c[2], op.c[3]};
  for (int it = cr.c0 + int(threadIdx.x >> 6); it < cr.c1; it += kWaves)
#pragma unroll
  for (int comp = 0; comp < NC; ++comp) {
    const T* __restrict__ x = x0 + comp * stride;
    const T* __restrict__ extra = extra0 ? extra0 + comp * stride : nullptr;
    const int pb = items[it];
    const int inplane = op.lanes[it * 64 + lane];
    const bool lane_ok = inplane >= 0;
    const int k0 = pb * op.zb;
    const int kend = min(op.zb, op.nplanes - k0);
    const int base = k0 * sz + (lane_ok ? inplane : 0);
    const int imb = (it * op.zb) * 64 + lane;
    // cell bits and flags of plane k at emp[k * estep], flp[k * estep]
    const uint8_t* __restrict__ emp = op.em_im ? op.em_im + imb : op.emask + base;
    const uint8_t* __restrict__ flp = op.fl_im ? op.fl_im + imb : op.flags + base;
    const int estep = op.em_im ? 64 : sz;
    // plane j of the item is grid plane k0 - 1 + j (j = 0 .. kend + 1), kept in
    // slot j % R; the cell bits and flags of output plane k in slot k % R
    T w[R][9];
    uint32_t em[R], fl[R];
#pragma unroll
    for (int j = 0; j < kZBPF + 2; ++j)
      if (j < kend + 2) load_plane(x, base + (j - 1) * sz, sy, w[j % R]);
#pragma unroll
    for (int k = 0; k <= kZBPF; ++k)
      if (k < kend) {
        em[k % R] = emp[k * estep];
        fl[k % R] = flp[k * estep];
      }
#pragma unroll
    for (int k = 0; k < kZB; ++k) {
      if (k >= kend) break;
      // prefetch: plane j = k + kZBPF + 2 replaces plane k - 1 (no longer needed)
      const int j = k + kZBPF + 2;
      if (j < kZB + 2 && j < kend + 2) load_plane(x, base + (j - 1) * sz, sy, w[j % R]);
      const int kn = k + kZBPF + 1;
      if (kn < kZB && kn < kend) {
        em[kn % R] = emp[kn * estep];
        fl[kn % R] = flp[kn * estep];
      }
      const int node = base + k * sz;
      const uint32_t e = em[k % R];
      const bool rw = lane_ok && (fl[k % R] & op.rowbit);
      // the constant stencil when every row lane has all 8 cells (non-row lanes'
      // results are discarded by the epilogues)
      const bool interior = __all((!rw) || e == 0xFFu);
      T y = window_apply<T>(w[k % R], w[(k + 1) % R], w[(k + 2) % R], e, interior, c);
      if (extra != nullptr && rw && (fl[k % R] & kFlagExtra)) y += extra[node];
      epi(comp, node, lane_ok, rw, e, y, w[(k + 1) % R][4], (fl[k % R] & kFlagExtra) != 0u, imb + 64 * k);
    }
  }
}

template <typename T, int NC, class Epi>
__device__ __forceinline__ void zb_walk(const int* __restrict__ items, int nitems, const ZOp<T>& op,
                                        const T* __restrict__ x0, int64_t stride, Epi& epi,
                                        const T* __restrict__ extra0 = nullptr) {
  zb_walk_range<T, NC>(items, block_chunks(nitems), op, x0, stride, epi, extra0);
}

// q = A p on rows (0 elsewhere), partial p.q; NC identical components.
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_cg_q_zb(const int* __restrict__ items, int nitems, ZOp<T> op,
                                                    int64_t stride, const T* __restrict__ p,
                                                    T* __restrict__ q, double* __restrict__ partials,
                                                    const KScal* sc) {
  if (sc->done) return;
  double dot[1] = {0.0};
  auto epi = [&](int d, int node, bool ok, bool rw, uint32_t, T y, T xc, bool, int) {
    const T qv = rw ? y : T(0);
    if (ok) q[d * stride + node] = qv;
    dot[0] += double(xc) * double(qv);
  };
  zb_walk<T, NC>(items, nitems, op, p, stride, epi, op.extra);
  block_partials<1>(dot, partials);
}

// Refinement residual in FP64 on the z-blocked walk, NC identical components:
// r32 = TR(b - A x) on rows (0 elsewhere) and the partial sums of r.r and b.b.
// With IMO, r32 is stored in walk order (planes of imstride).
template <typename TR, int NC, bool IMO = false>
__global__ __launch_bounds__(kBlock) void k_zb_residual(const int* __restrict__ items, int nitems, ZOp<double> op,
                                                        const double* __restrict__ b, const double* __restrict__ x,
                                                        TR* __restrict__ r32, int64_t stride,
                                                        double* __restrict__ partials, int64_t imstride = 0) {
  double v[2] = {0.0, 0.0};
  auto epi = [&](int q, int node, bool ok, bool rw, uint32_t, double y, double, bool, int im) {
    if (!ok) return;
    const int64_t i = q * stride + node;
    const double bi = rw ? b[i] : 0.0;
    const double ri = rw ? bi - y : 0.0;
    r32[IMO ? int64_t(q * int(imstride) + im) : i] = TR(ri);
    v[0] += ri * ri;
    v[1] += bi * bi;
  };
  zb_walk<double, NC>(items, nitems, op, x, stride, epi, op.extra);
  block_partials<2>(v, partials);
}

// r = b - A x on rows, 0 elsewhere (multigrid residual).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_zb_resid(const int* __restrict__ items, int nitems, ZOp<T> op,
                                                     const T* __restrict__ x, const T* __restrict__ b,
                                                     T* __restrict__ r, const KScal* sc) {
  if (sc->done) return;
  auto epi = [&](int, int node, bool ok, bool rw, uint32_t, T y, T, bool, int) {
    if (ok) r[node] = rw ? T(b[node] - y) : T(0);
  };
  zb_walk<T, 1>(items, nitems, op, x, 0, epi, op.extra);
}

// Chebyshev-Jacobi step on rows, NC identical components (planes of `stride`):
//   d <- c1 d + c2 D^-1 (b - A x_in),  x_out = x_in + d;  0 off rows.
// With DOT, also the partial sum of b . x_out (the preconditioned residual dot).
// With IMV, b and d are in walk order (planes of imstride; d is neither read nor
// written off the rows), x_in and x_out on the lattice.
template <typename T, bool DOT, int NC, bool IMV = false>
__device__ __forceinline__ void zb_cheb_body(const int* __restrict__ items, ChunkRange cr, const ZOp<T>& op,
                                             const T* __restrict__ x_in, const T* __restrict__ b,
                                             T* __restrict__ d, T* __restrict__ x_out, T c1, T c2,
                                             double (&dot)[1], int64_t stride, int zero_off_rows,
                                             int64_t imstride = 0) {
  const T c0 = op.c[0];
  auto epi = [&](int q, int node, bool ok, bool rw, uint32_t e, T y, T xc, bool xrow, int im) {
    if (!ok) return;
    const int64_t i = q * stride + node;
    const int64_t iv = IMV ? int64_t(q * int(imstride) + im) : i;
    if (rw) {
      // the stored diagonal only where the row has terms beyond its fine cells:
      // elsewhere it is c0 times the number of kept fine cells
      const T dinv = (op.dinv && xrow) ? op.dinv[node] : T(1) / (c0 * T(__builtin_popcount(e)));
      const T dold = (c1 != T(0)) ? d[iv] : T(0);
      const T bi = b[iv];
      const T dn = c1 * dold + c2 * dinv * (bi - y);
      const T xn = xc + dn;
      d[iv] = dn;
      x_out[i] = xn;
      if (DOT) dot[0] += double(bi) * double(xn);
    } else if (zero_off_rows) {
      if (!IMV) d[i] = T(0);
      x_out[i] = T(0);
    }
  };
  zb_walk_range<T, NC>(items, cr, op, x_in, stride, epi, op.extra);
}

// Chebyshev start from x = 0 in walk order: d = x = c2 D^-1 b on the rows of the
// walked positions (b, d in walk order, x on the lattice, 0 off the rows), with
// the diagonal the walk uses.
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_cheb0_im(const int* __restrict__ items, int nitems, ZOp<T> op,
                                                     const T* __restrict__ b, T* __restrict__ d,
                                                     T* __restrict__ x, T c2, int64_t stride, int64_t imstride) {
  const int lane = threadIdx.x & 63;
  const T c0 = op.c[0];
  const ChunkRange cr = block_chunks(nitems);
  for (int it = cr.c0 + int(threadIdx.x >> 6); it < cr.c1; it += kWaves) {
    const int inplane = op.lanes[it * 64 + lane];
    if (inplane < 0) continue;
    const int k0 = items[it] * op.zb;
    const int kend = min(op.zb, op.nplanes - k0);
    const int64_t imb = int64_t(it) * op.zb * 64 + lane;
    for (int k = 0; k < kend; ++k) {
      const int node = (k0 + k) * op.sz + inplane;
      const int64_t im = imb + 64 * k;
      const uint32_t e = op.em_im ? op.em_im[im] : op.emask[node];
      const uint32_t f = op.fl_im ? op.fl_im[im] : op.flags[node];
      const bool rw = f & op.rowbit;
      const T dinv = !rw ? T(0)
                         : (op.dinv && (f & kFlagExtra)) ? op.dinv[node] : T(1) / (c0 * T(__builtin_popcount(e)));
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const T v = rw ? T(c2 * b[q * imstride + im] * dinv) : T(0);
        if (rw) d[q * imstride + im] = v;
        x[q * stride + node] = v;
      }
    }
  }
}

template <typename T, bool DOT, int NC = 1, bool IMV = false>
__global__ __launch_bounds__(kBlock) void k_zb_cheb(const int* __restrict__ items, int nitems, ZOp<T> op,
                                                    const T* __restrict__ x_in, const T* __restrict__ b,
                                                    T* __restrict__ d, T* __restrict__ x_out, T c1, T c2,
                                                    double* __restrict__ partials, const KScal* sc,
                                                    int64_t stride = 0, int zero_off_rows = 1,
                                                    int64_t imstride = 0) {
  // zero_off_rows = 0: d and x_out already hold 0 off rows (written by an earlier
  // step of the same sequence), so only the rows are stored
  if (sc && sc->done) return;
  double dot[1] = {0.0};
  zb_cheb_body<T, DOT, NC, IMV>(items, block_chunks(nitems), op, x_in, b, d, x_out, c1, c2, dot, stride,
                                zero_off_rows, imstride);
  if (DOT) block_partials<1>(dot, partials);
}

// Chebyshev step k of the consistent-mass correction for several requests at
// once (one launch over the column items of all of them).  Request r owns the
// logical blocks [off[r], off[r+1]) and splits its items over them as its own
// launch would; a request whose sequence is shorter than k returns at once.
// Buffer buf0 holds the iterate after the odd steps' inputs: step k reads buf0
// when k is odd and writes buf1, and the other way round when k is even.
constexpr int kMaxBatch = 16;
template <typename T>
struct ChebJob {
  const int* items;
  int nitems, nblocks, iters;
  ZOp<T> op;
  const T* b;
  T* d;
  T* buf0;
  T* buf1;
  int64_t stride, imstride;  // b and d in walk order
};
template <typename T>
struct ChebBatch {
  ChebJob<T> job[kMaxBatch];
  int off[kMaxBatch + 1];
  int njobs;
};
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_zb_cheb_batch(ChebBatch<T> B, int k, T c1, T c2) {
  const int L = xcd_block();
  int r = 0;
  while (r + 1 < B.njobs && L >= B.off[r + 1]) ++r;
  const ChebJob<T>& J = B.job[r];
  if (k >= J.iters) return;
  const int lb = L - B.off[r];
  const int per = J.nitems / J.nblocks, rem = J.nitems % J.nblocks;
  const int c0 = lb * per + (lb < rem ? lb : rem);
  const ChunkRange cr{c0, c0 + per + (lb < rem ? 1 : 0)};
  double dot[1] = {0.0};
  const T* x_in = (k & 1) ? J.buf0 : J.buf1;
  T* x_out = (k & 1) ? J.buf1 : J.buf0;
  zb_cheb_body<T, false, NC, true>(J.items, cr, J.op, x_in, J.b, J.d, x_out, c1, c2, dot, J.stride, k == 1 ? 1 : 0,
                                   J.imstride);
}

// ---------------------------------------------------------------------------
// Consistent-mass correction with a tensor-product preconditioner (the
// velocity correction M_FF delta = (G Phi)_F of Sections 2.2 and 2.4).
//
// On a uniform grid the Q1 mass stencil is the product over the three axes of
// (1, 4, 1) h/6; scaled by its diagonal, each axis contributes the symbol
// 1 + cos(th)/2 in [1/2, 3/2], which is where the Jacobi interval [1/8, 27/8]
// comes from.  The preconditioner P = D^-1/2 T D^-1/2, with T the product over
// the axes of the three-point stencil (-1/4, 1, -1/4) restricted to the free
// rows (a principal submatrix of a positive definite product stencil, hence
// itself positive definite), gives each axis the symbol
// (1 + cos/2)(1 - cos/2) = 1 - cos^2/4 in [3/4, 1]: the interior spectrum of
// P M lies in [27/64, 1] (condition 2.4 instead of 27).  Rows at the vessel wall
// move it outward.  On a refined lattice T is block diagonal: the stride-1
// product stencil among the rows with fine cells only, the stride-2 one among
// the rows with coarse cells or hanging children (kFlagExtra).
//
// One Chebyshev step is two passes: w = D^-1/2 (b - M x) on the lattice (the mass
// walk), then d = c1 d + c2 D^-1/2 T w, x += d (a walk with the constant
// product stencil over w).  x is updated in place: the second pass reads x only
// at the node itself.
// ---------------------------------------------------------------------------

// weight of the one-dimensional three-point stencil (-t, 1, -t)
constexpr double kTensorT = 0.25;

// w = D^-1/2 b on the rows of the walked positions, 0 at the others; on a
// refined lattice the kFlagExtra rows go to wx and w holds 0 there.  With IMV,
// b is in walk order.
template <typename T, int NC, bool IMV>
__global__ __launch_bounds__(kBlock) void k_tm_scale(const int* __restrict__ items, int nitems, ZOp<T> op,
                                                     const T* __restrict__ b, T* __restrict__ w,
                                                     T* __restrict__ wx, int64_t stride, int64_t imstride) {
  const int lane = threadIdx.x & 63;
  const T c0 = op.c[0];
  const ChunkRange cr = block_chunks(nitems);
  for (int it = cr.c0 + int(threadIdx.x >> 6); it < cr.c1; it += kWaves) {
    const int inplane = op.lanes[it * 64 + lane];
    if (inplane < 0) continue;
    const int k0 = items[it] * op.zb;
    const int kend = min(op.zb, op.nplanes - k0);
    const int64_t imb = int64_t(it) * op.zb * 64 + lane;
    for (int k = 0; k < kend; ++k) {
      const int node = (k0 + k) * op.sz + inplane;
      const int64_t im = imb + 64 * k;
      const uint32_t e = op.em_im ? op.em_im[im] : op.emask[node];
      const uint32_t f = op.fl_im ? op.fl_im[im] : op.flags[node];
      const bool rw = f & op.rowbit;
      const bool xr = wx != nullptr && (f & kFlagExtra);
      const T sd = !rw ? T(0)
                       : sqrt((op.dinv && (f & kFlagExtra)) ? op.dinv[node]
                                                            : T(1) / (c0 * T(__builtin_popcount(e))));
#pragma unroll
      for (int q = 0; q < NC; ++q) {
        const int64_t i = q * stride + node;
        const T v = rw ? sd * b[IMV ? q * imstride + im : i] : T(0);
        if (xr) {
          if (rw) wx[i] = v;
          w[i] = T(0);
        } else {
          w[i] = v;
        }
      }
    }
  }
}

// w = D^-1/2 (b - M x) on the rows (the mass walk; on a refined lattice with the
// extra terms of op.extra), 0 at the other walked positions; kFlagExtra rows into
// wx as in k_tm_scale.
template <typename T, int NC, bool IMV>
__global__ __launch_bounds__(kBlock) void k_tm_resid(const int* __restrict__ items, int nitems, ZOp<T> op,
                                                     const T* __restrict__ x, const T* __restrict__ b,
                                                     T* __restrict__ w, T* __restrict__ wx, int64_t stride,
                                                     int64_t imstride) {
  const T c0 = op.c[0];
  auto epi = [&](int q, int node, bool ok, bool rw, uint32_t e, T y, T, bool xrow, int im) {
    if (!ok) return;
    const int64_t i = q * stride + node;
    T v = T(0);
    if (rw) {
      const T dinv = (op.dinv && xrow) ? op.dinv[node] : T(1) / (c0 * T(__builtin_popcount(e)));
      v = sqrt(dinv) * (b[IMV ? int64_t(q * int(imstride) + im) : i] - y);
    }
    if (wx != nullptr && xrow) {
      if (rw) wx[i] = v;
      w[i] = T(0);
    } else {
      w[i] = v;
    }
  };
  zb_walk<T, NC>(items, nitems, op, x, stride, epi, op.extra);
}

// The stride-2 product stencil on the kFlagExtra rows of a refined lattice (the
// listed nodes xn; lattice planes sy, sz, nplanes): zx = sum over o in
// {-1,0,1}^3 of (-t)^{|o|} wx[n + 2o], neighbours outside the lattice dropped.
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_tm_extra(int nxn, const int32_t* __restrict__ xn,
                                                     const uint8_t* __restrict__ flags, uint32_t rowbit,
                                                     const T* __restrict__ wx, T* __restrict__ zx, T tw, int sy,
                                                     int sz, int nplanes, int64_t stride) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nxn) return;
  const int n = xn[t];
  if (!(flags[n] & rowbit)) return;
  const int ix = n % sy, iy = (n % sz) / sy, iz = n / sz;
  const int ny = sz / sy;
  const T wt[3] = {-tw, T(1), -tw};
  T acc[NC];
#pragma unroll
  for (int q = 0; q < NC; ++q) acc[q] = T(0);
  for (int oz = -1; oz <= 1; ++oz) {
    const int jz = iz + 2 * oz;
    if (jz < 0 || jz >= nplanes) continue;
    for (int oy = -1; oy <= 1; ++oy) {
      const int jy = iy + 2 * oy;
      if (jy < 0 || jy >= ny) continue;
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        const int jx = ix + 2 * ox;
        if (jx < 0 || jx >= sy) continue;
        const int m = jz * sz + jy * sy + jx;
        const T wgt = wt[oz + 1] * wt[oy + 1] * wt[ox + 1];
#pragma unroll
        for (int q = 0; q < NC; ++q) acc[q] += wgt * wx[q * stride + m];
      }
    }
  }
#pragma unroll
  for (int q = 0; q < NC; ++q) zx[q * stride + n] = acc[q];
}

// d = c1 d + c2 D^-1/2 (T w), x += d on the rows (FIRST: d = x = c2 D^-1/2 T w, and
// x = 0 at the other walked positions).  The stride-1 product stencil is walked
// like the mass apply, with the constant weights and the window entries whose x
// or y neighbour lies outside the lattice set to 0; on a refined lattice the
// kFlagExtra rows take their sum from zx.  op.c[0] is the mass cell diagonal.
// With IMV, d is in walk order.
template <typename T, int NC, bool IMV, bool FIRST>
__global__ __launch_bounds__(kBlock) void k_tm_cheb(const int* __restrict__ items, int nitems, ZOp<T> op,
                                                    const T* __restrict__ w0, const T* __restrict__ zx,
                                                    T* __restrict__ d, T* __restrict__ x, T c1, T c2, T tw,
                                                    int64_t stride, int64_t imstride) {
  constexpr int R = kZBPF + 3;
  const int lane = threadIdx.x & 63;
  const int sy = op.sy, sz = op.sz;
  const int ny = sz / sy;
  const T c0 = op.c[0];
  // per neighbour class (centre, face, edge, corner), in the form window_apply
  // takes for its constant stencil
  const T ct[4] = {T(0.125), -tw * T(0.25), tw * tw * T(0.5), -tw * tw * tw};
  const ChunkRange cr = block_chunks(nitems);
  for (int it = cr.c0 + int(threadIdx.x >> 6); it < cr.c1; it += kWaves)
#pragma unroll
  for (int comp = 0; comp < NC; ++comp) {
    const T* __restrict__ w = w0 + comp * stride;
    const int pb = items[it];
    const int inplane = op.lanes[it * 64 + lane];
    const bool lane_ok = inplane >= 0;
    const int ip = lane_ok ? inplane : 0;
    const int ix = ip % sy, iy = ip / sy;
    // window entry (y + 1) * 3 + (x + 1) of offsets x, y in {-1, 0, 1}
    uint32_t vm = 0x1FFu;
    if (ix == 0) vm &= ~0x49u;
    if (ix == sy - 1) vm &= ~0x124u;
    if (iy == 0) vm &= ~0x7u;
    if (iy == ny - 1) vm &= ~0x1C0u;
    const int k0 = pb * op.zb;
    const int kend = min(op.zb, op.nplanes - k0);
    const int base = k0 * sz + ip;
    const int imb = (it * op.zb) * 64 + lane;
    const uint8_t* __restrict__ emp = op.em_im ? op.em_im + imb : op.emask + base;
    const uint8_t* __restrict__ flp = op.fl_im ? op.fl_im + imb : op.flags + base;
    const int estep = op.em_im ? 64 : sz;
    T wr[R][9];
    uint32_t em[R], fl[R];
    // plane load with the entries outside the lattice set to 0
    auto ldm = [&](int node, T(&dst)[9]) {
      load_plane(w, node, sy, dst);
#pragma unroll
      for (int q = 0; q < 9; ++q)
        if (!((vm >> q) & 1u)) dst[q] = T(0);
    };
#pragma unroll
    for (int j = 0; j < kZBPF + 2; ++j)
      if (j < kend + 2) ldm(base + (j - 1) * sz, wr[j % R]);
#pragma unroll
    for (int k = 0; k <= kZBPF; ++k)
      if (k < kend) {
        em[k % R] = emp[k * estep];
        fl[k % R] = flp[k * estep];
      }
#pragma unroll
    for (int k = 0; k < kZB; ++k) {
      if (k >= kend) break;
      const int j = k + kZBPF + 2;
      if (j < kZB + 2 && j < kend + 2) ldm(base + (j - 1) * sz, wr[j % R]);
      const int kn = k + kZBPF + 1;
      if (kn < kZB && kn < kend) {
        em[kn % R] = emp[kn * estep];
        fl[kn % R] = flp[kn * estep];
      }
      const T y = window_apply<T>(wr[k % R], wr[(k + 1) % R], wr[(k + 2) % R], 0xFFu, true, ct);
      if (!lane_ok) continue;
      const int node = base + k * sz;
      const int64_t i = comp * stride + node;
      const int64_t iv = IMV ? int64_t(comp * imstride + imb + 64 * k) : i;
      const uint32_t f = fl[k % R];
      if (f & op.rowbit) {
        const bool xrow = (f & kFlagExtra) != 0u;
        const T dinv = (op.dinv && xrow) ? op.dinv[node] : T(1) / (c0 * T(__builtin_popcount(em[k % R])));
        const T z = sqrt(dinv) * ((zx != nullptr && xrow) ? zx[i] : y);
        const T dn = FIRST ? c2 * z : c1 * d[iv] + c2 * z;
        d[iv] = dn;
        x[i] = FIRST ? dn : x[i] + dn;
      } else if (FIRST) {
        x[i] = T(0);
      }
    }
  }
}

}  // namespace ibfe
