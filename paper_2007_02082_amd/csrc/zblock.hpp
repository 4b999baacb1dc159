// Z-blocked matrix-free apply of the symmetric masked Q1 forms (alpha M + beta K)
// fused with the CG dot product p.q.
//
// A wavefront owns one "column item": 64 consecutive node ids of one z-plane
// (a row segment in the x-fastest numbering, clamped to the plane) and walks it
// up through kZB planes.  A 3-plane sliding window of the 3x3 (y, x) neighbour
// rows stays in registers, so each output node costs 9 coalesced row loads
// instead of 27 gathers, and the y/z row addresses are shared by the x shifts.
// When every lane of the wavefront sits in the interior (all 8 cells kept) the
// constant 27-point stencil is used; otherwise the per-neighbour kept-cell
// counts are evaluated.
#pragma once

#include "kernels.hpp"

namespace ibfe {

constexpr int kZB = 8;

template <typename T>
__device__ __forceinline__ void load_plane(const T* __restrict__ x, int node, int sy, T (&w)[9]) {
#pragma unroll
  for (int y = -1; y <= 1; ++y) {
    const T* row = x + (node + y * sy);
    w[(y + 1) * 3 + 0] = row[-1];
    w[(y + 1) * 3 + 1] = row[0];
    w[(y + 1) * 3 + 2] = row[1];
  }
}

// y = sum_o cw(o) x(o) over the window planes lo (z-1), mid (z), hi (z+1).
template <typename T>
__device__ __forceinline__ T window_apply(const T (&lo)[9], const T (&mid)[9], const T (&hi)[9],
                                          uint32_t e, bool interior, const T (&c)[4]) {
  const T* pl[3] = {lo, mid, hi};
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
  T acc = T(0);
#pragma unroll
  for (int z = 0; z < 3; ++z)
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const int ox = k % 3 - 1, oy = k / 3 - 1, oz = z - 1;
      const int t = (ox != 0) + (oy != 0) + (oz != 0);
      acc += c[t] * T(__builtin_popcount(e & compat(ox, oy, oz))) * pl[z][k];
    }
  return acc;
}

// q = A p on rows (0 elsewhere), partial p.q.  items: plane_block * cpp + chunk.
template <typename T, int NC>
__global__ __launch_bounds__(kBlock) void k_cg_q_zb(const int* __restrict__ items, int nitems, int cpp,
                                                    int nplanes, OpSym<T, NC> op,
                                                    const T* __restrict__ p, T* __restrict__ q,
                                                    double* __restrict__ partials, const KScal* sc) {
  if (sc->done) return;
  const int lane = threadIdx.x & 63;
  const int sy = op.sy, sz = op.sz;
  const T c[4] = {op.c[0], op.c[1], op.c[2], op.c[3]};
  double dot[1] = {0.0};
  const ChunkRange cr = block_chunks(nitems);
  for (int it = cr.c0 + int(threadIdx.x >> 6); it < cr.c1; it += kWaves) {
    const int item = items[it];
    const int pb = item / cpp, ch = item - pb * cpp;
    const int inplane = ch * 64 + lane;
    const bool lane_ok = inplane < sz;
    const int k0 = pb * kZB;
    const int kend = min(kZB, nplanes - k0);
    const int base = k0 * sz + (lane_ok ? inplane : sz - 1);
#pragma unroll
    for (int d = 0; d < NC; ++d) {
      const T* pd = p + d * op.stride;
      T* qd = q + d * op.stride;
      T w0[9], w1[9], w2[9];
      load_plane(pd, base - sz, sy, w0);
      load_plane(pd, base, sy, w1);
      for (int k = 0; k < kend; ++k) {
        const int node = base + k * sz;
        load_plane(pd, node + sz, sy, w2);
        const uint32_t e = op.emask[node];
        const bool rw = lane_ok && (op.flags[node] & op.rowbit);
        const bool interior = __all((!lane_ok) || e == 0xFFu);
        const T y = window_apply<T>(w0, w1, w2, e, interior, c);
        const T qv = rw ? y : T(0);
        if (lane_ok) qd[node] = qv;
        dot[0] += double(w1[4]) * double(qv);
#pragma unroll
        for (int j = 0; j < 9; ++j) {
          w0[j] = w1[j];
          w1[j] = w2[j];
        }
      }
    }
  }
  block_partials<1>(dot, partials);
}

}  // namespace ibfe
