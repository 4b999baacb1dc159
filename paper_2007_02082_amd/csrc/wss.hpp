// Wall shear stress at the Lagrangian points (the paper's clinical output,
// defined in Section 2.6, evaluated at the immersed wall points): the nodal velocity
// gradient by the lumped L2 projection of the Q1 gradient, its symmetric part
// interpolated to each point with the kernel of Eq. 18, and the tangential part
// of the traction 2 mu eps n.
#pragma once

#include "step_kernels.hpp"

namespace ibfe {

// eps at every node of P (0 elsewhere), two fields of 3 planes of `stride`:
// (xx, yy, zz) and (xy, xz, yz).
// g_de = (G_e u_d) / m with the lumped mass m = (h^3 / 8) x kept cells around the node.
__global__ __launch_bounds__(kBlock) void k_nodal_strain(NodeList nl, const uint8_t* __restrict__ emask,
                                                         const uint8_t* __restrict__ flags,
                                                         const double* __restrict__ u, int64_t stride,
                                                         double h, double g0, double g1, double g2, int sy,
                                                         int sz, double* __restrict__ ed,
                                                         double* __restrict__ eo) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  const uint32_t e = emask[n];
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if ((flags[n] & kFlagP) && e != 0u) {
    const double gc[3] = {g0, g1, g2};
    const double inv_m = 8.0 / (h * h * h * double(__builtin_popcount(e)));
    double g[3][3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double* ud = u + d * stride;
      g[d][0] = apply_grad<double, 0>(ud, n, e, gc, sy, sz) * inv_m;
      g[d][1] = apply_grad<double, 1>(ud, n, e, gc, sy, sz) * inv_m;
      g[d][2] = apply_grad<double, 2>(ud, n, e, gc, sy, sz) * inv_m;
    }
    v[0] = g[0][0];
    v[1] = g[1][1];
    v[2] = g[2][2];
    v[3] = 0.5 * (g[0][1] + g[1][0]);
    v[4] = 0.5 * (g[0][2] + g[2][0]);
    v[5] = 0.5 * (g[1][2] + g[2][1]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ed[k * stride + n] = v[k];
    eo[k * stride + n] = v[3 + k];
  }
}

// Refined lattice: eps from the composite weak gradients g_c = (G_0 u_c, G_1 u_c,
// G_2 u_c) (3 planes each, hanging children already gathered) and the row sums m
// of the constrained mass.
__global__ __launch_bounds__(kBlock) void k_strain_from_grad(NodeList nl, const uint8_t* __restrict__ flags,
                                                             const double* __restrict__ g0,
                                                             const double* __restrict__ g1,
                                                             const double* __restrict__ g2,
                                                             const double* __restrict__ m, int64_t stride,
                                                             double* __restrict__ ed, double* __restrict__ eo) {
  const int n = chunk_node(nl);
  if (n < 0) return;
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if ((flags[n] & kFlagP) && m[n] > 0.0) {
    const double inv_m = 1.0 / m[n];
    const double* g[3] = {g0, g1, g2};
    double a[3][3];  // a[d][e] = (G_e u_d) / m
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int e = 0; e < 3; ++e) a[d][e] = g[d][e * stride + n] * inv_m;
    v[0] = a[0][0];
    v[1] = a[1][1];
    v[2] = a[2][2];
    v[3] = 0.5 * (a[0][1] + a[1][0]);
    v[4] = 0.5 * (a[0][2] + a[2][0]);
    v[5] = 0.5 * (a[1][2] + a[2][1]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    ed[k * stride + n] = v[k];
    eo[k * stride + n] = v[3 + k];
  }
}

// tau_i = t - (t.n) n, t = 2 mu eps(X_i) n, eps(X_i) = sum_s w[s][i] eps(idx[s][i]);
// normals and tau are M x 3 row major (the normal is scaled to unit length).
__global__ __launch_bounds__(kBlock) void k_wall_shear(int M, const int32_t* __restrict__ idx,
                                                       const double* __restrict__ w,
                                                       const double* __restrict__ ed,
                                                       const double* __restrict__ eo, int64_t stride,
                                                       const double* __restrict__ normals, double mu,
                                                       double* __restrict__ tau) {
  const int i = blockIdx.x * kBlock + threadIdx.x;
  if (i >= M) return;
  double E[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  for (int s = 0; s < 64; ++s) {
    const int32_t j = idx[int64_t(s) * M + i];
    if (j < 0) continue;
    const double ws = w[int64_t(s) * M + i];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      E[k] += ws * ed[k * stride + j];
      E[3 + k] += ws * eo[k * stride + j];
    }
  }
  double nv[3] = {normals[3 * i], normals[3 * i + 1], normals[3 * i + 2]};
  const double nn = sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
  if (nn > 0.0)
    for (int d = 0; d < 3; ++d) nv[d] /= nn;
  const double t0 = 2.0 * mu * (E[0] * nv[0] + E[3] * nv[1] + E[4] * nv[2]);
  const double t1 = 2.0 * mu * (E[3] * nv[0] + E[1] * nv[1] + E[5] * nv[2]);
  const double t2 = 2.0 * mu * (E[4] * nv[0] + E[5] * nv[1] + E[2] * nv[2]);
  const double tn = t0 * nv[0] + t1 * nv[1] + t2 * nv[2];
  tau[3 * i] = t0 - tn * nv[0];
  tau[3 * i + 1] = t1 - tn * nv[1];
  tau[3 * i + 2] = t2 - tn * nv[2];
}

}  // namespace ibfe
