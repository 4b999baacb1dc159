// Geometric multigrid kernels for the pressure increment equation: the first
// Chebyshev step from a zero guess, full-weighting restriction (transpose of
// trilinear prolongation), prolongation with correction, the dense coarsest
// solve, and the vector kernels of multigrid-preconditioned CG.
#pragma once

#include "zblock.hpp"

namespace ibfe {

constexpr uint32_t kMgRow = 16u;  // pressure unknown bit of the level flags

// x = d = c2 D^-1 b on rows (Chebyshev step from x = 0), 0 elsewhere; D is
// c0 times the number of kept cells around the node; NC planes of `stride`.
template <typename T, int NC = 1>
__global__ __launch_bounds__(kBlock) void k_mg_cheb0(NodeList nl,
                                                     const uint8_t* __restrict__ emask,
                                                     const uint8_t* __restrict__ flags, T c0, T c2,
                                                     const T* __restrict__ b, T* __restrict__ d,
                                                     T* __restrict__ x, const KScal* sc,
                                                     uint32_t rowbit = kMgRow, int64_t stride = 0) {
  if (sc && sc->done) return;
  const int n = chunk_node(nl);
  if (n < 0) return;
  const bool rw = flags[n] & rowbit;
  const T dinv = rw ? T(1) / (c0 * T(__builtin_popcount(uint32_t(emask[n])))) : T(0);
#pragma unroll
  for (int q = 0; q < NC; ++q) {
    const T v = rw ? T(c2 * b[q * stride + n] * dinv) : T(0);
    d[q * stride + n] = v;
    x[q * stride + n] = v;
  }
}

__device__ __forceinline__ void node_ijk(int n, int sy, int sz, int& i, int& j, int& k) {
  k = n / sz;
  const int rem = n - k * sz;
  j = rem / sy;
  i = rem - j * sy;
}

// bc[I] = sum_j P_jI rf[j] for coarse unknowns I (0 elsewhere); the fine nodes j
// are the 27 around the node at the same place (2I), weight prod_d (1 - |o_d|/2).
// With xc, also the coarse level's pre-smoothing from zero, xc = c2 D^-1 bc (the
// first Chebyshev step; D = c0 times the kept cells), which saves its own pass.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_restrict(NodeList nl,
                                                        const uint8_t* __restrict__ cflags, int csy,
                                                        int csz, int fsy, int fsz, int fnx, int fny,
                                                        int fnz, const T* __restrict__ rf,
                                                        T* __restrict__ bc, const KScal* sc,
                                                        const uint8_t* __restrict__ cemask = nullptr,
                                                        T c0 = T(0), T c2 = T(0), T* __restrict__ xc = nullptr) {
  if (sc->done) return;
  const int n = chunk_node(nl);
  if (n < 0) return;
  if (!(cflags[n] & kMgRow)) {
    bc[n] = T(0);
    if (xc) xc[n] = T(0);
    return;
  }
  int ic, jc, kc;
  node_ijk(n, csy, csz, ic, jc, kc);
  const int fi = 2 * ic, fj = 2 * jc, fk = 2 * kc;
  const int fc = fi + fsy * fj + fsz * fk;
  // per-axis offsets and weights; an offset that leaves the grid is replaced by
  // the centre with weight 0, so all 27 loads issue at once and the sum (in the
  // fixed order below) equals that over the nodes inside the grid
  int dx[3], dy[3], dz[3];
  T wx[3], wy[3], wz[3];
#pragma unroll
  for (int o = -1; o <= 1; ++o) {
    const T wo = o ? T(0.5) : T(1);
    const bool inx = fi + o >= 0 && fi + o <= fnx;
    const bool iny = fj + o >= 0 && fj + o <= fny;
    const bool inz = fk + o >= 0 && fk + o <= fnz;
    dx[o + 1] = inx ? o : 0;
    dy[o + 1] = iny ? o * fsy : 0;
    dz[o + 1] = inz ? o * fsz : 0;
    wx[o + 1] = inx ? wo : T(0);
    wy[o + 1] = iny ? wo : T(0);
    wz[o + 1] = inz ? wo : T(0);
  }
  T v[27];
#pragma unroll
  for (int q = 0; q < 27; ++q) v[q] = rf[fc + dx[q % 3] + dy[(q / 3) % 3] + dz[q / 9]];
  T acc = T(0);
#pragma unroll
  for (int q = 0; q < 27; ++q) acc += (wx[q % 3] * wy[(q / 3) % 3] * wz[q / 9]) * v[q];
  bc[n] = acc;
  if (xc) xc[n] = T(c2 * acc * (T(1) / (c0 * T(__builtin_popcount(uint32_t(cemask[n]))))));
}

// xf[j] += sum_I P_jI xc[I] on fine unknowns (trilinear interpolation).  All
// eight corner loads are issued at once: along an axis with an even fine index
// the second corner is the first one again with weight 0, so the sum (taken in
// the fixed corner order) equals that over the parents alone.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_prolong(NodeList nl,
                                                       const uint8_t* __restrict__ fflags, int fsy,
                                                       int fsz, int csy, int csz,
                                                       const T* __restrict__ xc, T* __restrict__ xf,
                                                       const KScal* sc) {
  if (sc->done) return;
  const int n = chunk_node(nl);
  if (n < 0 || !(fflags[n] & kMgRow)) return;
  int i, j, k;
  node_ijk(n, fsy, fsz, i, j, k);
  const int ox = i & 1, oy = j & 1, oz = k & 1;
  const T* c0 = xc + (i >> 1) + csy * (j >> 1) + csz * (k >> 1);
  const int dx = ox, dy = oy * csy, dz = oz * csz;
  const T xold = xf[n];
  T v[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) v[c] = c0[(c & 1 ? dx : 0) + (c & 2 ? dy : 0) + (c & 4 ? dz : 0)];
  const T wx[2] = {ox ? T(0.5) : T(1), ox ? T(0.5) : T(0)};
  const T wy[2] = {oy ? T(0.5) : T(1), oy ? T(0.5) : T(0)};
  const T wz[2] = {oz ? T(0.5) : T(1), oz ? T(0.5) : T(0)};
  T acc = T(0);
#pragma unroll
  for (int c = 0; c < 8; ++c) acc += wx[c & 1] * wy[(c >> 1) & 1] * wz[(c >> 2) & 1] * v[c];
  xf[n] = xold + acc;
}

// Coarsest level: x[u_i] = sum_j inv[i][j] b[u_j] (m <= 1024).  The inverse is
// symmetric (formed as L^-T L^-1 with both triangles written from the same sums),
// so row i is the contiguous column i: one wavefront per row reads it coalesced
// along the lanes, sums in FP64 and reduces across the wavefront in a fixed order;
// the m rows spread over m / 4 workgroups.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_dense(int m, const int64_t* __restrict__ ids,
                                                     const T* __restrict__ inv, const T* __restrict__ b,
                                                     T* __restrict__ x, const KScal* sc) {
  if (sc->done) return;
  __shared__ T bs[1024];
  for (int j = threadIdx.x; j < m; j += kBlock) bs[j] = b[ids[j]];
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * kWaves + wave;
  if (i >= m) return;
  const T* row = inv + int64_t(i) * m;
  double acc = 0.0;
  for (int j = lane; j < m; j += 64) acc += double(row[j]) * double(bs[j]);
  acc = wave_sum(acc);
  if (lane == 0) x[ids[i]] = T(acc);
}

// partials of a.b over rows
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mg_dot(NodeList nl,
                                                   const uint8_t* __restrict__ flags,
                                                   const T* __restrict__ a, const T* __restrict__ b,
                                                   double* __restrict__ partials, const KScal* sc) {
  if (sc->done) return;
  double v[1] = {0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (flags[n] & kMgRow) v[0] += double(a[n]) * double(b[n]);
  }
  block_partials<1>(v, partials);
}

// ---- multigrid-preconditioned CG (vectors over the level-0 unknowns) -------

// x = 0, r = b on rows (0 elsewhere); partials r.r, b.b
template <typename T>
// With xpre, also the finest level's pre-smoothing of the V-cycle that follows,
// xpre = c2 D^-1 r from zero (D = c0 times the kept cells around the node).
__global__ __launch_bounds__(kBlock) void k_mgcg_init(NodeList nl,
                                                      const uint8_t* __restrict__ flags,
                                                      const T* __restrict__ b, T* __restrict__ x,
                                                      T* __restrict__ r, double* __restrict__ partials,
                                                      const uint8_t* __restrict__ emask = nullptr,
                                                      T c0 = T(0), T c2 = T(0), T* __restrict__ xpre = nullptr) {
  double v[2] = {0.0, 0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    const bool rw = flags[n] & kMgRow;
    const T bi = rw ? b[n] : T(0);
    x[n] = T(0);
    r[n] = bi;
    if (xpre) xpre[n] = rw ? T(c2 * bi * (T(1) / (c0 * T(__builtin_popcount(uint32_t(emask[n])))))) : T(0);
    v[0] += double(bi) * double(bi);
  }
  v[1] = v[0];
  block_partials<2>(v, partials);
}

// rr, bb -> convergence test; rz is set later by k_fin_mgcg_rz
__global__ __launch_bounds__(kBlock) void k_fin_mgcg_init(const double* __restrict__ partials, int nb,
                                                          KScal* sc, double tol2, int max_iters) {
  double tot[2];
  sum_partials<2>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  sc->tol2 = tol2;
  sc->max_iters = max_iters;
  sc->rr = tot[0];
  sc->bb = tot[1];
  sc->rz = 1.0;
  sc->beta = 0.0;
  sc->iters = 0;
  sc->status = 0;
  sc->done = (tot[0] <= tol2 * tot[1]) ? 1 : 0;
  if (bad(tot[0]) || bad(tot[1])) {
    sc->status = 2;
    sc->done = 1;
  }
}

// rz_new = r.z (from the partials of the last smoothing step): beta = rz_new / rz
// (beta = 0 on the first call, flagged by iters == 0 and rz == 1 set at init)
__global__ __launch_bounds__(kBlock) void k_fin_mgcg_rz(const double* __restrict__ partials, int nb,
                                                        KScal* sc, int first) {
  if (sc->done) return;
  double tot[1];
  sum_partials<1>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  const double rz_new = tot[0];
  if (bad(rz_new) || !(rz_new > 0.0)) {
    sc->status = bad(rz_new) ? 2 : 1;
    sc->done = 1;
    return;
  }
  sc->beta = first ? 0.0 : rz_new / sc->rz;
  sc->rz = rz_new;
}

// x += alpha p, r -= alpha q on rows; partial r.r
template <typename T>
// With xpre, also the finest level's pre-smoothing of the next V-cycle on the
// rows (its off-row entries hold zeros from k_mgcg_init and the smoothing steps).
__global__ __launch_bounds__(kBlock) void k_mgcg_xr(NodeList nl,
                                                    const uint8_t* __restrict__ flags, T* __restrict__ x,
                                                    T* __restrict__ r, const T* __restrict__ p,
                                                    const T* __restrict__ q, double* __restrict__ partials,
                                                    const KScal* sc, const uint8_t* __restrict__ emask = nullptr,
                                                    T c0 = T(0), T c2 = T(0), T* __restrict__ xpre = nullptr) {
  if (sc->done) return;
  const T alpha = T(sc->alpha);
  double v[1] = {0.0};
  const ChunkRange cr = block_chunks(nl.n);
  for (int c = cr.c0 + int(threadIdx.x >> 6); c < cr.c1; c += kWaves) {
    const int n = nl.node(c);
    if (flags[n] & kMgRow) {
      x[n] += alpha * p[n];
      const T ri = r[n] - alpha * q[n];
      r[n] = ri;
      if (xpre) xpre[n] = T(c2 * ri * (T(1) / (c0 * T(__builtin_popcount(uint32_t(emask[n]))))));
      v[0] += double(ri) * double(ri);
    }
  }
  block_partials<1>(v, partials);
}

__global__ __launch_bounds__(kBlock) void k_fin_mgcg_xr(const double* __restrict__ partials, int nb,
                                                        KScal* sc) {
  if (sc->done) return;
  double tot[1];
  sum_partials<1>(partials, nb, tot);
  if (threadIdx.x != 0) return;
  sc->rr = tot[0];
  sc->iters += 1;
  if (bad(tot[0])) {
    sc->status = 2;
    sc->done = 1;
  } else if (tot[0] <= sc->tol2 * sc->bb || sc->iters >= sc->max_iters) {
    sc->done = 1;
  }
}

// p = z + beta p on rows
template <typename T>
__global__ __launch_bounds__(kBlock) void k_mgcg_p(NodeList nl,
                                                   const uint8_t* __restrict__ flags,
                                                   const T* __restrict__ z, T* __restrict__ p,
                                                   const KScal* sc) {
  if (sc->done) return;
  const T beta = T(sc->beta);
  const int n = chunk_node(nl);
  if (n < 0) return;
  p[n] = (flags[n] & kMgRow) ? T(z[n] + beta * p[n]) : T(0);
}

}  // namespace ibfe
