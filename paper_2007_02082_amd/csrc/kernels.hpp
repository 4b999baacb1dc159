// gfx950 kernels of the IPCS + BCE-IB step on the masked Q1 grid.
//
// Data layout: every nodal field is a dense array over all grid nodes (id
// n = i + sy j + sz k), offset by a zero halo so that the 27 neighbours of any
// node are addressable without bounds checks; base pointers passed to kernels
// point at node 0.  Work is distributed over a node list (NodeList): either
// 64-node chunks that contain at least one active node (a wavefront owns one
// chunk, so every load and store of a chunk is one coalesced 256/512-byte
// transaction), or, where the active nodes fill their chunks sparsely (thin
// vessels on a large box), the active nodes themselves, 64 per wavefront in
// ascending order.  Multi-component fields are `nc` planes of `stride` values.
//
// Matrix-free Q1 operators on a uniform grid: within one cube the entry
// between nodes i and j = i + o depends only on o, and the assembled entry is
// that value times the number of kept cells that contain both nodes.  With
// emask(i) = bits of the 8 cells around node i (bit s = sx + 2 sy + 4 sz for
// the cell (i-1+sx, j-1+sy, k-1+sz)), the cells shared with i + o are
// emask & X(ox) & Y(oy) & Z(oz), X(+1) = cells with sx = 1, X(-1) with sx = 0.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ibfe {

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// ---------------------------------------------------------------------------
// launch geometry
// ---------------------------------------------------------------------------

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own
// L2).  Remap so that XCD x runs a contiguous range of logical blocks: a
// block's neighbour rows are then mostly reused from that XCD's L2.
__device__ __forceinline__ int xcd_block() {
  const int B = gridDim.x, b = blockIdx.x;
  const int xcd = b & 7, idx = b >> 3;
  const int per = B >> 3, rem = B & 7;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Nodes of a launch, one 64-lane group per wavefront trip.  With per_lane = 0
// group c is the chunk ids[c] (node = 64 ids[c] + lane); with per_lane = 1 it
// is ids[64 c .. 64 c + 63], ascending, the last group padded with a node that
// is in no set (flags 0, no cells, no floating slot).  Every kernel treats such
// a node as a non-row; padding lanes only ever store zeros there.
struct NodeList {
  const int* ids = nullptr;
  int n = 0;
  int per_lane = 0;
  __device__ __forceinline__ int node(int c) const {
    const int l = int(threadIdx.x & 63);
    const int v = ids[per_lane ? c * 64 + l : c];
    return per_lane ? v : v * 64 + l;
  }
};

// Contiguous range of chunks [c0, c1) owned by this block; each wavefront
// walks it with stride kWaves (one 64-node chunk per wavefront per trip).
struct ChunkRange {
  int c0, c1;
};
__device__ __forceinline__ ChunkRange block_chunks(int nchunks) {
  const int b = xcd_block(), B = gridDim.x;
  const int per = nchunks / B, rem = nchunks % B;
  const int c0 = b * per + (b < rem ? b : rem);
  return {c0, c0 + per + (b < rem ? 1 : 0)};
}

// Node of the one-node-per-thread kernels (grid = ceil(nl.n / kWaves)), or -1.
__device__ __forceinline__ int chunk_node(const NodeList& nl) {
  const int c = xcd_block() * kWaves + int(threadIdx.x >> 6);
  if (c >= nl.n) return -1;
  return nl.node(c);
}

// ---------------------------------------------------------------------------
// deterministic FP64 reductions: every reducing kernel writes one partial per
// block (plain stores; the kernel boundary publishes them) and a one-block
// finalize kernel sums them in a fixed order.  No atomics, no fences.
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return v;
}

// Block sum of K values; thread 0 stores partials[k * gridDim.x + blockIdx.x].
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], double* __restrict__ partials) {
  __shared__ double sh[K][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = wave_sum(v[k]);
    if (lane == 0) sh[k][wave] = s;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) s += sh[k][w];
      partials[k * gridDim.x + blockIdx.x] = s;
    }
  }
}

// One-block sum of K rows of nb partials (fixed order); result valid in thread 0.
template <int K>
__device__ __forceinline__ void sum_partials(const double* __restrict__ partials, int nb,
                                             double (&tot)[K]) {
  __shared__ double sh[K][kWaves];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int b = threadIdx.x; b < nb; b += kBlock) s += partials[k * nb + b];
    s = wave_sum(s);
    if (lane == 0) sh[k][wave] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) t += sh[k][w];
    tot[k] = t;
  }
}

// ---------------------------------------------------------------------------
// stencil coefficient helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ constexpr uint32_t side_mask(int axis, int o) {
  // cells whose side along `axis` is compatible with neighbour offset o
  return o == 0 ? 0xFFu
                 : (axis == 0 ? (o > 0 ? 0xAAu : 0x55u)
                              : axis == 1 ? (o > 0 ? 0xCCu : 0x33u) : (o > 0 ? 0xF0u : 0x0Fu));
}
__device__ __forceinline__ constexpr uint32_t compat(int ox, int oy, int oz) {
  return side_mask(0, ox) & side_mask(1, oy) & side_mask(2, oz);
}

// 3x3 window of one plane around `node`; neighbours at x offsets +-st and row
// offsets +-sy (st = 2 with doubled sy, sz addresses the coarse elements of a
// refined lattice).
template <typename T>
__device__ __forceinline__ void load_plane(const T* __restrict__ x, int node, int sy, T (&w)[9],
                                           int st = 1) {
#pragma unroll
  for (int y = -1; y <= 1; ++y) {
    const T* row = x + (node + y * sy);
    w[(y + 1) * 3 + 0] = row[-st];
    w[(y + 1) * 3 + 1] = row[0];
    w[(y + 1) * 3 + 2] = row[st];
  }
}

// y = sum_o cw(o) x(o) over the window planes lo (z-1), mid (z), hi (z+1), with
// cw(o) = c[t(o)] * (number of kept cells shared by the node and node + o).
// The counts are formed from the 8 cell bits as floating-point sums: a corner
// neighbour lies in one cell, an edge neighbour in two, a face neighbour in four.
template <typename T>
__device__ __forceinline__ T window_apply(const T (&lo)[9], const T (&mid)[9], const T (&hi)[9],
                                          uint32_t e, bool interior, const T (&c)[4]) {
  const T* pl[3] = {lo, mid, hi};
  // W(i, j, k): window value at offset (i-1, j-1, k-1)
#define W_(i, j, k) pl[k][(j) * 3 + (i)]
  if (interior) {
    T s[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int z = 0; z < 3; ++z)
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        const int ox = k % 3 - 1, oy = k / 3 - 1, oz = z - 1;
        const int t = (ox != 0) + (oy != 0) + (oz != 0);
        s[t] += pl[z][k];
      }
    return c[0] * T(8) * s[0] + c[1] * T(4) * s[1] + c[2] * T(2) * s[2] + c[3] * s[3];
  }
  T b[2][2][2];  // b[sz][sy][sx]: cell (i-1+sx, j-1+sy, k-1+sz) kept
#pragma unroll
  for (int q = 0; q < 8; ++q) b[q >> 2][(q >> 1) & 1][q & 1] = T((e >> q) & 1u);
  T n = T(0), a3 = T(0), a2 = T(0);
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    const int sx = q & 1, sy = (q >> 1) & 1, sz = q >> 2;
    n += b[sz][sy][sx];
    a3 += b[sz][sy][sx] * W_(2 * sx, 2 * sy, 2 * sz);
  }
#pragma unroll
  for (int u = 0; u < 2; ++u)
#pragma unroll
    for (int v = 0; v < 2; ++v) {
      a2 += (b[0][v][u] + b[1][v][u]) * W_(2 * u, 2 * v, 1);   // edge (ox, oy, 0)
      a2 += (b[v][0][u] + b[v][1][u]) * W_(2 * u, 1, 2 * v);   // edge (ox, 0, oz)
      a2 += (b[v][u][0] + b[v][u][1]) * W_(1, 2 * u, 2 * v);   // edge (0, oy, oz)
    }
  T acc = c[0] * n * W_(1, 1, 1) + c[2] * a2 + c[3] * a3;
  if (c[1] != T(0)) {  // face neighbours (zero per-cell entry for the stiffness)
    T a1 = T(0);
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      a1 += (b[0][0][u] + b[0][1][u] + b[1][0][u] + b[1][1][u]) * W_(2 * u, 1, 1);
      a1 += (b[0][u][0] + b[0][u][1] + b[1][u][0] + b[1][u][1]) * W_(1, 2 * u, 1);
      a1 += (b[u][0][0] + b[u][0][1] + b[u][1][0] + b[u][1][1]) * W_(1, 1, 2 * u);
    }
    acc += c[1] * a1;
  }
#undef W_
  return acc;
}

// y = sum_o c[|ox|+|oy|+|oz|] * (kept cells shared with node n + o) * x[n + o]
// (symmetric operators alpha M + beta K: c[t] = per-cell entry for offset type t).
template <typename T>
__device__ __forceinline__ T apply_sym(const T* __restrict__ x, int n, uint32_t e,
                                       const T (&c)[4], int sy, int sz, int st = 1) {
  T w0[9], w1[9], w2[9];
  load_plane(x, n - sz, sy, w0, st);
  load_plane(x, n, sy, w1, st);
  load_plane(x, n + sz, sy, w2, st);
  return window_apply<T>(w0, w1, w2, e, __all(e == 0xFFu), c);
}

// Weak gradient G_d x at node n: entry(o) = sum over shared kept cells of
// (1/2)(+-1) * prod_{e != d} m(o_e), m(0) = h/3, m(1) = h/6; the sign is that
// of o_d, or for o_d = 0 +1 on cells below the node (s_d = 0), -1 above.
// g2[c] = (1/2) (h/3)^(2-c) (h/6)^c with c = nonzeros among the two other axes.
template <typename T, int D>
__device__ __forceinline__ T apply_grad(const T* __restrict__ x, int n, uint32_t e,
                                        const T (&g2)[3], int sy, int sz, int st = 1) {
  T acc = T(0);
#pragma unroll
  for (int oz = -1; oz <= 1; ++oz)
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy)
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        const int o[3] = {ox, oy, oz};
        const int cnt_other = (D != 0 && ox != 0) + (D != 1 && oy != 0) + (D != 2 && oz != 0);
        const uint32_t cm = e & compat(ox, oy, oz);
        int mult;
        if (o[D] != 0) {
          mult = o[D] * __builtin_popcount(cm);
        } else {
          mult = __builtin_popcount(cm & side_mask(D, -1)) - __builtin_popcount(cm & side_mask(D, 1));
        }
        acc += g2[cnt_other] * T(mult) * x[n + st * ox + sy * oy + sz * oz];
      }
  return acc;
}

// ---------------------------------------------------------------------------
// operators used inside the Krylov kernels
// ---------------------------------------------------------------------------

// alpha M + beta K restricted to rows with (flags & rowbit); nc identical
// components.  diag = c[0] * popcount(emask).
template <typename T, int NC>
struct OpSym {
  static constexpr int kNC = NC;
  const uint8_t* emask;
  const uint8_t* flags;
  uint32_t rowbit;
  int sy, sz;
  int64_t stride;
  T c[4];
  __device__ __forceinline__ bool row(int n) const { return flags[n] & rowbit; }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[NC]) const {
    const uint32_t e = emask[n];
    T cc[4] = {c[0], c[1], c[2], c[3]};
#pragma unroll
    for (int d = 0; d < NC; ++d) y[d] = apply_sym<T>(x + d * stride, n, e, cc, sy, sz);
  }
  __device__ __forceinline__ T inv_diag(int n) const {
    return T(1) / (c[0] * T(__builtin_popcount(uint32_t(emask[n]))));
  }
};

// Stored 27-point stencil (advection-diffusion operator of the tentative
// velocity), coefficient plane t = (ox+1) + 3 (oy+1) + 9 (oz+1).
template <typename T, int NC>
struct OpStencil {
  static constexpr int kNC = NC;
  const T* coef;  // [27][stride]
  const uint8_t* flags;
  uint32_t rowbit;
  int sy, sz;
  int64_t stride;
  __device__ __forceinline__ bool row(int n) const { return flags[n] & rowbit; }
  __device__ __forceinline__ void apply(int n, const T* __restrict__ x, T (&y)[NC]) const {
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
  }
  __device__ __forceinline__ T inv_diag(int n) const { return T(1) / coef[13 * stride + n]; }
  // the same product with the loads staged: the 27 coefficients, then the 27
  // neighbour values of one component at a time, each batch issued before any
  // use (more loads in flight per wavefront for the FP64 refinement residual)
  __device__ __forceinline__ void apply_staged(int n, const T* __restrict__ x, T (&y)[NC]) const {
    T w[27];
#pragma unroll
    for (int t = 0; t < 27; ++t) w[t] = coef[t * stride + n];
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      T v[27];
#pragma unroll
      for (int t = 0; t < 27; ++t) v[t] = x[d * stride + n + (t % 3 - 1) + sy * ((t / 3) % 3 - 1) + sz * (t / 9 - 1)];
      T acc = T(0);
#pragma unroll
      for (int t = 0; t < 27; ++t) acc += w[t] * v[t];
      y[d] = acc;
    }
  }
};

// CSR matrix (the IB Gram matrix) over rows [0, nrows), NC right-hand sides.
template <int NC>
struct OpCSR {
  static constexpr int kNC = NC;
  const int64_t* ptr;
  const int32_t* col;
  const double* val;
  const double* diag;
  int nrows;
  int64_t stride;
  __device__ __forceinline__ bool row(int n) const { return n < nrows; }
  __device__ __forceinline__ void apply(int n, const double* __restrict__ x, double (&y)[NC]) const {
#pragma unroll
    for (int d = 0; d < NC; ++d) y[d] = 0.0;
    for (int64_t q = ptr[n]; q < ptr[n + 1]; ++q) {
      const double w = val[q];
      const int c = col[q];
#pragma unroll
      for (int d = 0; d < NC; ++d) y[d] += w * x[d * stride + c];
    }
  }
  __device__ __forceinline__ double inv_diag(int n) const { return 1.0 / diag[n]; }
};

// ---------------------------------------------------------------------------
// Krylov scalar state (device resident; updated by one-block finalize kernels
// so that no host round trip is needed between kernels)
// ---------------------------------------------------------------------------

struct KScal {
  double rz, rr, bb, alpha, beta, tol2;        // CG
  double rho, rho_old, omega, ts, tt, rv;      // BiCGStab (alpha shared)
  int32_t done, iters, max_iters, status;      // status: 0 ok, 1 breakdown, 2 non-finite
  // testing aid (BiCGStab only): report a breakdown once the iteration count reaches
  // brk_at (> 0), then clear it; set from the host, never by the init kernels
  int32_t brk_at, pad_;
};

__device__ __forceinline__ bool bad(double v) { return !(v == v) || v - v != 0.0; }

// ---------------------------------------------------------------------------
// CG (Jacobi preconditioned): x, r, p, q are NC-plane vectors
// ---------------------------------------------------------------------------

// r = b - A x (x = 0 if zero_guess); p = D^-1 r; partials: r.p, r.r, b.b
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_cg_init(NodeList nl,
                                                    Op op, const T* __restrict__ b, T* __restrict__ x,
                                                    T* __restrict__ r, T* __restrict__ p,
                                                    double* __restrict__ partials, int zero_guess) {
  constexpr int NC = Op::kNC;
  double v[3] = {0.0, 0.0, 0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    const bool rw = op.row(n);
    T ax[NC];
    if (!zero_guess && rw) op.apply(n, x, ax);
    const T di = rw ? op.inv_diag(n) : T(0);
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      const int64_t i = d * op.stride + n;
      if (zero_guess) x[i] = T(0);
      const T bi = rw ? b[i] : T(0);
      const T ri = rw ? (zero_guess ? bi : T(bi - ax[d])) : T(0);
      const T zi = ri * di;
      r[i] = ri;
      p[i] = zi;
      v[0] += double(ri) * double(zi);
      v[1] += double(ri) * double(ri);
      v[2] += double(bi) * double(bi);
    }
  }
  block_partials<3>(v, partials);
}

__global__ __launch_bounds__(kBlock) void k_fin_cg_init(const double* __restrict__ partials, int nb,
                                                        KScal* sc, double tol2, int max_iters) {
  double tot[3];
  sum_partials<3>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  sc->tol2 = tol2;
  sc->max_iters = max_iters;
  sc->rz = tot[0];
  sc->rr = tot[1];
  sc->bb = tot[2];
  sc->iters = 0;
  sc->status = 0;
  sc->done = (tot[1] <= tol2 * tot[2]) ? 1 : 0;
  if (bad(tot[0]) || bad(tot[1]) || bad(tot[2])) {
    sc->status = 2;
    sc->done = 1;
  }
}

// q = A p; partial p.q
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_cg_q(NodeList nl, Op op,
                                                 const T* __restrict__ p, T* __restrict__ q,
                                                 double* __restrict__ partials, const KScal* sc) {
  if (sc->done) return;
  constexpr int NC = Op::kNC;
  double v[1] = {0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    T y[NC];
    const bool rw = op.row(n);
    if (rw) op.apply(n, p, y);
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      const int64_t i = d * op.stride + n;
      const T qi = rw ? y[d] : T(0);
      q[i] = qi;
      v[0] += double(p[i]) * double(qi);
    }
  }
  block_partials<1>(v, partials);
}

// alpha = rz / p.q
__global__ __launch_bounds__(kBlock) void k_fin_cg_q(const double* __restrict__ partials, int nb,
                                                     KScal* sc) {
  if (sc->done) return;
  double tot[1];
  sum_partials<1>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  const double pq = tot[0];
  if (!(pq > 0.0) || bad(pq)) {
    sc->status = bad(pq) ? 2 : 1;
    sc->done = 1;
    sc->alpha = 0.0;
  } else {
    sc->alpha = sc->rz / pq;
  }
}

// x += alpha p; r -= alpha q; partials r.D^-1 r, r.r
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_cg_xr(NodeList nl, Op op,
                                                  T* __restrict__ x, T* __restrict__ r,
                                                  const T* __restrict__ p, const T* __restrict__ q,
                                                  double* __restrict__ partials, const KScal* sc) {
  if (sc->done) return;
  constexpr int NC = Op::kNC;
  const T alpha = T(sc->alpha);
  double v[2] = {0.0, 0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (op.row(n)) {
      const T di = op.inv_diag(n);
#pragma unroll
      for (int d = 0; d < NC; ++d) {
        const int64_t i = d * op.stride + n;
        x[i] += alpha * p[i];
        const T ri = r[i] - alpha * q[i];
        r[i] = ri;
        v[0] += double(ri) * double(ri * di);
        v[1] += double(ri) * double(ri);
      }
    }
  }
  block_partials<2>(v, partials);
}

// beta = rz_new / rz; convergence test on |r|^2 <= tol2 |b|^2
__global__ __launch_bounds__(kBlock) void k_fin_cg_xr(const double* __restrict__ partials, int nb,
                                                      KScal* sc) {
  if (sc->done) return;
  double tot[2];
  sum_partials<2>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  const double rz_new = tot[0];
  sc->beta = rz_new / sc->rz;
  sc->rz = rz_new;
  sc->rr = tot[1];
  sc->iters += 1;
  if (bad(rz_new) || bad(tot[1])) {
    sc->status = 2;
    sc->done = 1;
  } else if (tot[1] <= sc->tol2 * sc->bb || sc->iters >= sc->max_iters) {
    sc->done = 1;
  }
}

// p = D^-1 r + beta p
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_cg_p(NodeList nl, Op op,
                                                 const T* __restrict__ r, T* __restrict__ p,
                                                 const KScal* sc) {
  if (sc->done) return;
  constexpr int NC = Op::kNC;
  const T beta = T(sc->beta);
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (op.row(n)) {
      const T di = op.inv_diag(n);
#pragma unroll
      for (int d = 0; d < NC; ++d) {
        const int64_t i = d * op.stride + n;
        p[i] = r[i] * di + beta * p[i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// BiCGStab (right Jacobi preconditioning), NC-plane vectors.  x, b and the
// preconditioned directions phat, shat (read at the neighbours by the applies)
// live on the lattice.  With a per-lane node list the other vectors (r, rhat,
// p, v, s, t), touched only at the row itself, are kept in node-list order:
// component d of the node of lane l of chunk c at d * 64 nl.n + 64 c + l (dense,
// whole cache lines where a vessel's rows fill part of each lattice line); with
// a list of lattice chunks they stay on the lattice (measured: the chunk order
// made the uniform cylinder's apply slower, 78 -> 94 us).
// ---------------------------------------------------------------------------

__device__ __forceinline__ int64_t nl_index(const NodeList& nl, int c, int d, int n, int64_t stride) {
  return nl.per_lane ? int64_t(d) * (int64_t(nl.n) * 64) + int64_t(c) * 64 + int(threadIdx.x & 63)
                     : int64_t(d) * stride + n;
}

// r = b - A x, rhat = r, p = v = 0; partials r.r, b.b
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_bi_init(NodeList nl, Op op,
                                                    const T* __restrict__ b, const T* __restrict__ x,
                                                    T* __restrict__ r, T* __restrict__ rhat,
                                                    T* __restrict__ p, T* __restrict__ v,
                                                    double* __restrict__ partials, int zero_guess) {
  // zero_guess: x = 0, so r = b without an apply
  constexpr int NC = Op::kNC;
  double s[2] = {0.0, 0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    const bool rw = op.row(n);
    T ax[NC];
#pragma unroll
    for (int d = 0; d < NC; ++d) ax[d] = T(0);
    if (rw && !zero_guess) op.apply(n, x, ax);
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      const int64_t i = d * op.stride + n;
      const int64_t q = nl_index(nl, c, d, n, op.stride);
      const T bi = rw ? b[i] : T(0);
      const T ri = rw ? T(bi - ax[d]) : T(0);
      r[q] = ri;
      rhat[q] = ri;
      p[q] = T(0);
      v[q] = T(0);
      s[0] += double(ri) * double(ri);
      s[1] += double(bi) * double(bi);
    }
  }
  block_partials<2>(s, partials);
}

__global__ __launch_bounds__(kBlock) void k_fin_bi_init(const double* __restrict__ partials, int nb,
                                                        KScal* sc, double tol2, int max_iters) {
  double tot[2];
  sum_partials<2>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  sc->tol2 = tol2;
  sc->max_iters = max_iters;
  sc->rho = tot[0];
  sc->rr = tot[0];
  sc->bb = tot[1];
  sc->rho_old = 1.0;
  sc->alpha = 1.0;
  sc->omega = 1.0;
  sc->iters = 0;
  sc->status = 0;
  sc->done = (tot[0] <= tol2 * tot[1]) ? 1 : 0;
  if (bad(tot[0]) || bad(tot[1])) {
    sc->status = 2;
    sc->done = 1;
  }
}

// p = r + beta (p - omega v), phat = D^-1 p
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_bi_p(NodeList nl, Op op,
                                                 const T* __restrict__ r, T* __restrict__ p,
                                                 const T* __restrict__ v, T* __restrict__ phat,
                                                 const KScal* sc) {
  if (sc->done) return;
  constexpr int NC = Op::kNC;
  const T beta = T((sc->rho / sc->rho_old) * (sc->alpha / sc->omega));
  const T omega = T(sc->omega);
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (op.row(n)) {
      const T di = op.inv_diag(n);
#pragma unroll
      for (int d = 0; d < NC; ++d) {
        const int64_t q = nl_index(nl, c, d, n, op.stride);
        const T pi = r[q] + beta * (p[q] - omega * v[q]);
        p[q] = pi;
        phat[d * op.stride + n] = pi * di;
      }
    } else {
#pragma unroll
      for (int d = 0; d < NC; ++d) phat[d * op.stride + n] = T(0);
    }
  }
}

// waves per SIMD the apply is compiled for (operators may raise it)
template <class Op>
struct ApplyWaves {
  static constexpr int value = 1;
};

// y = A xin (xin on the lattice, y and w in node-list order); partials w.y (and
// y.y for MODE 1)

template <typename T, class Op, int MODE>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(ApplyWaves<Op>::value)))
void k_bi_apply(NodeList nl, Op op,
                                                     const T* __restrict__ xin, T* __restrict__ y,
                                                     const T* __restrict__ w,
                                                     double* __restrict__ partials, const KScal* sc) {
  if (sc->done) return;
  constexpr int NC = Op::kNC;
  double s[2] = {0.0, 0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    const bool rw = op.row(n);
    T ay[NC];
    if (rw) op.apply(n, xin, ay);
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      const int64_t q = nl_index(nl, c, d, n, op.stride);
      const T yi = rw ? ay[d] : T(0);
      y[q] = yi;
      s[0] += double(w[q]) * double(yi);
      if (MODE == 1) s[1] += double(yi) * double(yi);
    }
  }
  block_partials<2>(s, partials);
}

// MODE 0: alpha = rho / rhat.v;  MODE 1: omega = t.s / t.t
template <int MODE>
__global__ __launch_bounds__(kBlock) void k_fin_bi_apply(const double* __restrict__ partials, int nb,
                                                         KScal* sc) {
  if (sc->done) return;
  double tot[2];
  sum_partials<2>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  if (MODE == 0) {
    sc->rv = tot[0];
    if (tot[0] == 0.0 || bad(tot[0])) {
      sc->status = bad(tot[0]) ? 2 : 1;
      sc->done = 1;
    } else {
      sc->alpha = sc->rho / tot[0];
    }
  } else {
    sc->ts = tot[0];
    sc->tt = tot[1];
    if (bad(tot[0]) || bad(tot[1])) {
      sc->status = 2;
      sc->done = 1;
    } else {
      sc->omega = tot[1] > 0.0 ? tot[0] / tot[1] : 0.0;
    }
  }
}

// s = r - alpha v, shat = D^-1 s
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_bi_s(NodeList nl, Op op,
                                                 const T* __restrict__ r, const T* __restrict__ v,
                                                 T* __restrict__ s, T* __restrict__ shat,
                                                 const KScal* sc) {
  if (sc->done) return;
  constexpr int NC = Op::kNC;
  const T alpha = T(sc->alpha);
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (op.row(n)) {
      const T di = op.inv_diag(n);
#pragma unroll
      for (int d = 0; d < NC; ++d) {
        const int64_t q = nl_index(nl, c, d, n, op.stride);
        const T si = r[q] - alpha * v[q];
        s[q] = si;
        shat[d * op.stride + n] = si * di;
      }
    } else {
#pragma unroll
      for (int d = 0; d < NC; ++d) {
        s[nl_index(nl, c, d, n, op.stride)] = T(0);
        shat[d * op.stride + n] = T(0);
      }
    }
  }
}

// x += alpha phat + omega shat; r = s - omega t; partials rhat.r, r.r
template <typename T, class Op>
__global__ __launch_bounds__(kBlock) void k_bi_x(NodeList nl, Op op,
                                                 T* __restrict__ x, T* __restrict__ r,
                                                 const T* __restrict__ rhat, const T* __restrict__ phat,
                                                 const T* __restrict__ shat, const T* __restrict__ s,
                                                 const T* __restrict__ t, double* __restrict__ partials,
                                                 const KScal* sc) {
  if (sc->done) return;
  constexpr int NC = Op::kNC;
  const T alpha = T(sc->alpha), omega = T(sc->omega);
  double v[2] = {0.0, 0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (op.row(n)) {
#pragma unroll
      for (int d = 0; d < NC; ++d) {
        const int64_t i = d * op.stride + n;
        const int64_t q = nl_index(nl, c, d, n, op.stride);
        x[i] += alpha * phat[i] + omega * shat[i];
        const T ri = s[q] - omega * t[q];
        r[q] = ri;
        v[0] += double(rhat[q]) * double(ri);
        v[1] += double(ri) * double(ri);
      }
    }
  }
  block_partials<2>(v, partials);
}

__global__ __launch_bounds__(kBlock) void k_fin_bi_x(const double* __restrict__ partials, int nb,
                                                     KScal* sc) {
  if (sc->done) return;
  double tot[2];
  sum_partials<2>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  sc->rho_old = sc->rho;
  sc->rho = tot[0];
  sc->rr = tot[1];
  sc->iters += 1;
  if (bad(tot[0]) || bad(tot[1])) {
    sc->status = 2;
    sc->done = 1;
  } else if (tot[1] <= sc->tol2 * sc->bb || sc->iters >= sc->max_iters) {
    sc->done = 1;
  } else if (sc->omega == 0.0 || tot[0] == 0.0) {
    sc->status = 1;
    sc->done = 1;
  } else if (sc->brk_at > 0 && sc->iters >= sc->brk_at) {
    sc->status = 1;
    sc->done = 1;
    sc->brk_at = 0;
  }
}

// ---------------------------------------------------------------------------
// iterative refinement: FP64 residual r = b - A x on rows, its FP32 copy, and
// partials r.r, b.b
// ---------------------------------------------------------------------------
template <class Op, typename TR = float>
__global__ __launch_bounds__(kBlock) void k_residual(NodeList nl, Op op,
                                                     const double* __restrict__ b,
                                                     const double* __restrict__ x,
                                                     TR* __restrict__ r32,
                                                     double* __restrict__ partials) {
  constexpr int NC = Op::kNC;
  double v[2] = {0.0, 0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    const bool rw = op.row(n);
    double ax[NC];
    if (rw) {
      if constexpr (std::is_same<Op, OpStencil<double, 3>>::value)
        op.apply_staged(n, x, ax);
      else
        op.apply(n, x, ax);
    }
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      const int64_t i = d * op.stride + n;
      const double bi = rw ? b[i] : 0.0;
      const double ri = rw ? bi - ax[d] : 0.0;
      r32[i] = TR(ri);
      v[0] += ri * ri;
      v[1] += bi * bi;
    }
  }
  block_partials<2>(v, partials);
}

// out[0] = r.r, out[1] = b.b of the refinement residual
__global__ __launch_bounds__(kBlock) void k_fin_residual(const double* __restrict__ partials, int nb,
                                                         double* __restrict__ out) {
  double tot[2];
  sum_partials<2>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  out[0] = tot[0];
  out[1] = tot[1];
}

}  // namespace ibfe
