// Host-side set-up: validation, derived sets, canonical order, IB stencils and
// the IB Gram matrix G = I_F I_F^T (Section 2.3, Eqs. 17-22).
#include "plan.hpp"

#include <algorithm>
#include <cmath>
#include <numeric>

namespace ibfe {

namespace {

bool finite(double v) { return std::isfinite(v); }

}  // namespace

UnionFind::UnionFind(int64_t n) : parent(n) { std::iota(parent.begin(), parent.end(), 0); }
int64_t UnionFind::find(int64_t a) {
  while (parent[a] != a) {
    parent[a] = parent[parent[a]];
    a = parent[a];
  }
  return a;
}
void UnionFind::unite(int64_t a, int64_t b) {
  a = find(a);
  b = find(b);
  if (a != b) parent[std::max(a, b)] = std::min(a, b);
}

// Four-point regularised delta of Eq. 18 (support |r| < 2).
double delta4(double r) {
  r = std::fabs(r);
  if (r <= 1.0) return (3.0 - 2.0 * r + std::sqrt(1.0 + 4.0 * r - 4.0 * r * r)) / 8.0;
  if (r <= 2.0) return (5.0 - 2.0 * r - std::sqrt(-7.0 + 12.0 * r - 4.0 * r * r)) / 8.0;
  return 0.0;
}

// Inverses of the diagonal blocks of G (kIBBlock consecutive points each): a
// principal submatrix of the SPD G is SPD, so a Cholesky factor A = L L^T exists;
// A^-1 = L^-T L^-1, symmetrised and rounded to FP32 (a preconditioner only shapes
// the iteration, the solve itself stays FP64).
static void ib_block_inverses(Plan& P) {
  const int64_t M = P.M;
  const int B = kIBBlock;
  const int64_t nblk = (M + B - 1) / B;
  P.G_binv.assign(size_t(nblk) * B * B, 0.0f);
  std::vector<double> A(B * B), L(B * B), Li(B * B);
  for (int64_t b = 0; b < nblk; ++b) {
    const int64_t i0 = b * B;
    const int n = int(std::min<int64_t>(B, M - i0));
    std::fill(A.begin(), A.end(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int64_t q = P.G_ptr[i0 + i]; q < P.G_ptr[i0 + i + 1]; ++q) {
        const int64_t k = P.G_col[q] - i0;
        if (k >= 0 && k < n) A[i * B + k] = P.G_val[q];
      }
    std::fill(L.begin(), L.end(), 0.0);
    for (int j = 0; j < n; ++j) {
      double d = A[j * B + j];
      for (int k = 0; k < j; ++k) d -= L[j * B + k] * L[j * B + k];
      const double ljj = std::sqrt(std::max(d, 1e-300));
      L[j * B + j] = ljj;
      for (int i = j + 1; i < n; ++i) {
        double v = A[i * B + j];
        for (int k = 0; k < j; ++k) v -= L[i * B + k] * L[j * B + k];
        L[i * B + j] = v / ljj;
      }
    }
    // Li = L^-1 (lower triangular), column by column
    std::fill(Li.begin(), Li.end(), 0.0);
    for (int j = 0; j < n; ++j) {
      Li[j * B + j] = 1.0 / L[j * B + j];
      for (int i = j + 1; i < n; ++i) {
        double v = 0.0;
        for (int k = j; k < i; ++k) v -= L[i * B + k] * Li[k * B + j];
        Li[i * B + j] = v / L[i * B + i];
      }
    }
    float* out = &P.G_binv[size_t(b) * B * B];
    for (int i = 0; i < n; ++i)
      for (int j = 0; j <= i; ++j) {
        double v = 0.0;  // (L^-T L^-1)_ij = sum_k Li_ki Li_kj
        for (int k = i; k < n; ++k) v += Li[k * B + i] * Li[k * B + j];
        out[j * B + i] = float(v);
        out[i * B + j] = float(v);
      }
  }
}

int build_plan(const ibfe_grid* grid, const ibfe_ib* ib, const ibfe_params* params,
               const ibfe_inlet* inlet, Plan& P, std::string& err) {
  if (!grid || !params) {
    err = "grid and params are required";
    return IBFE_EINVAL;
  }
  if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1) {
    err = "nx, ny, nz must be >= 1";
    return IBFE_EINVAL;
  }
  if (!(grid->h > 0.0) || !finite(grid->h) || !finite(grid->origin[0]) ||
      !finite(grid->origin[1]) || !finite(grid->origin[2])) {
    err = "h must be positive and finite, origin finite";
    return IBFE_EINVAL;
  }
  if (!grid->node_mask) {
    err = "node_mask is required";
    return IBFE_EINVAL;
  }
  const ibfe_params& pr = *params;
  if (!(pr.rho > 0.0) || !(pr.mu > 0.0) || !(pr.dt > 0.0) || !finite(pr.rho) ||
      !finite(pr.mu) || !finite(pr.dt)) {
    err = "rho, mu and dt must be positive and finite";
    return IBFE_EINVAL;
  }
  if (pr.precision != 0 && pr.precision != 1) {
    err = "precision must be 0 (FP64) or 1 (FP32 inner / FP64 refinement)";
    return IBFE_EINVAL;
  }
  if (pr.precond < 0 || pr.precond > 2 || pr.advection < 0 || pr.advection > 1) {
    err = "precond must be 0 (Jacobi), 1 (Chebyshev) or 2 (multigrid); advection 0 (semi-implicit) or 1 (explicit)";
    return IBFE_EINVAL;
  }
  P.refined = grid->refine_cell != nullptr;
  if (pr.advdiff < 0 || pr.advdiff > 1) {
    err = "advdiff must be 0 (matrix-free) or 1 (assembled stencil)";
    return IBFE_EINVAL;
  }
  if (pr.mass_precond < 0 || pr.mass_precond > 1) {
    err = "mass_precond must be 0 (Jacobi) or 1 (tensor-product approximate inverse)";
    return IBFE_EINVAL;
  }
  if (pr.viscous < 0 || pr.viscous > 1) {
    err = "viscous must be 0 (mu (grad u, grad v)) or 1 (2 mu (eps(u), eps(v)))";
    return IBFE_EINVAL;
  }
  if (P.refined) {
    // every node array lives on the fine lattice of spacing h/2
    if (grid->nx > (1 << 29) || grid->ny > (1 << 29) || grid->nz > (1 << 29)) {
      err = "grid too large";
      return IBFE_EINVAL;
    }
    P.bnx = grid->nx;
    P.bny = grid->ny;
    P.bnz = grid->nz;
    P.hb = grid->h;
    P.nx = 2 * grid->nx;
    P.ny = 2 * grid->ny;
    P.nz = 2 * grid->nz;
    P.h = 0.5 * grid->h;
  } else {
    P.nx = grid->nx;
    P.ny = grid->ny;
    P.nz = grid->nz;
    P.h = grid->h;
  }
  for (int d = 0; d < 3; ++d) P.origin[d] = grid->origin[d];
  P.sy = int64_t(P.nx) + 1;
  P.sz = P.sy * (int64_t(P.ny) + 1);
  P.N = P.sz * (int64_t(P.nz) + 1);
  // dense padded device vectors are indexed with 32-bit ints
  if (P.N + 4 * (P.sz + P.sy + 1) + 4 * kChunk > (int64_t(1) << 31) - 1) {
    err = "grid too large for 32-bit node indexing";
    return IBFE_EINVAL;
  }
  if (P.refined) {
    const int64_t nc = int64_t(P.bnx) * P.bny * P.bnz;
    P.refine.assign(grid->refine_cell, grid->refine_cell + nc);
    for (uint8_t v : P.refine)
      if (v > 1) {
        err = "refine_cell values must be 0 or 1";
        return IBFE_EINVAL;
      }
  }
  P.params = pr;
  if (P.params.rtol <= 0.0) P.params.rtol = pr.precision == 0 ? 1e-13 : 1e-8;
  if (P.params.max_iters <= 0) P.params.max_iters = 20000;
  if (P.params.ib_rtol <= 0.0) P.params.ib_rtol = pr.precision == 0 ? 1e-13 : 1e-10;

  const int64_t N = P.N;
  const int nx = P.nx, ny = P.ny, nz = P.nz;
  P.mask.assign(grid->node_mask, grid->node_mask + N);
  for (int64_t n = 0; n < N; ++n)
    if (P.mask[n] > 1) {
      err = "node_mask values must be 0 or 1";
      return IBFE_EINVAL;
    }
  // boundary tags: explicit, or the face defaults (wall wins on edges/corners)
  P.tag.assign(N, IBFE_TAG_NONE);
  if (grid->bc_tag) {
    P.tag.assign(grid->bc_tag, grid->bc_tag + N);
    for (int64_t n = 0; n < N; ++n)
      if (P.tag[n] > IBFE_TAG_OUTLET) {
        err = "bc_tag values must be 0..3";
        return IBFE_EINVAL;
      }
  } else {
    for (int k = 0; k <= nz; ++k)
      for (int j = 0; j <= ny; ++j)
        for (int i = 0; i <= nx; ++i) {
          int64_t n = i + P.sy * j + P.sz * k;
          uint8_t t = IBFE_TAG_NONE;
          if (k == 0) t = IBFE_TAG_INLET;
          if (k == nz) t = IBFE_TAG_OUTLET;
          if (i == 0 || i == nx || j == 0 || j == ny) t = IBFE_TAG_WALL;
          P.tag[n] = t;
        }
  }

  // kept cells (elements) -> per-node cell bits, hanging nodes and the set P
  UnionFind uf(N);
  if (P.refined) {
    int rc = build_composite_cells(P, uf, err);
    if (rc) return rc;
  } else {
    P.emask.assign(N, 0);
    P.n_kept = 0;
    for (int k = 0; k < nz; ++k)
      for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
          int64_t c0 = i + P.sy * j + P.sz * k;
          bool kept = false;
          for (int a = 0; a < 8; ++a) {
            int64_t n = c0 + (a & 1) + P.sy * ((a >> 1) & 1) + P.sz * ((a >> 2) & 1);
            if (P.mask[n]) kept = true;
          }
          if (!kept) continue;
          ++P.n_kept;
          for (int a = 0; a < 8; ++a) {
            int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
            int64_t n = c0 + ax + P.sy * ay + P.sz * az;
            // the cell sits on the side s = 1 - a of corner node n
            int s = (1 - ax) + 2 * (1 - ay) + 4 * (1 - az);
            P.emask[n] |= uint8_t(1u << s);
            uf.unite(c0, n);
          }
        }
  }
  P.flags.assign(N, 0);
  for (int32_t n : P.hang_ids) P.flags[n] = IBFE_FLAG_HANG;
  P.P_ids.clear();
  P.n_free = P.n_pfree = 0;
  for (int64_t n = 0; n < N; ++n) {
    if (!P.emask[n] && !(P.refined && P.cmask[n])) continue;
    if (P.flags[n] & IBFE_FLAG_HANG) continue;
    uint8_t f = IBFE_FLAG_P;
    uint8_t t = P.tag[n];
    bool du = P.mask[n] == 0 || t == IBFE_TAG_WALL || t == IBFE_TAG_INLET;
    f |= du ? IBFE_FLAG_DU : IBFE_FLAG_F;
    if (t == IBFE_TAG_OUTLET) f |= IBFE_FLAG_PDIR;
    P.flags[n] = f;
    P.P_ids.push_back(n);
    if (!du) ++P.n_free;
    if (t != IBFE_TAG_OUTLET) ++P.n_pfree;
  }
  if (P.P_ids.empty()) {
    err = "empty domain: no node has mask 1";
    return IBFE_EINVAL;
  }
  // connected parts of the kept region; the ones without an outlet node float
  std::vector<uint8_t> root_has_outlet(N, 0);
  for (int64_t n : P.P_ids)
    if (P.flags[n] & IBFE_FLAG_PDIR) root_has_outlet[uf.find(n)] = 1;
  std::vector<int32_t> root_slot(N, -1);
  P.float_slot.assign(N, -1);
  P.n_floating = 0;
  P.float_count.clear();
  for (int64_t n : P.P_ids) {
    int64_t r = uf.find(n);
    if (root_has_outlet[r]) continue;
    if (root_slot[r] < 0) {
      if (P.n_floating == kMaxFloating) {
        err = "more than 8 connected parts without an outlet";
        return IBFE_EINVAL;
      }
      root_slot[r] = P.n_floating++;
      P.float_count.push_back(0);
    }
    P.float_slot[n] = int8_t(root_slot[r]);
    ++P.float_count[root_slot[r]];
  }
  // chunk list
  P.chunks.clear();
  int64_t nch = (N + kChunk - 1) / kChunk;
  for (int64_t c = 0; c < nch; ++c) {
    int64_t lo = c * kChunk, hi = std::min<int64_t>(N, lo + kChunk);
    for (int64_t n = lo; n < hi; ++n)
      if (P.flags[n] & (IBFE_FLAG_P | IBFE_FLAG_HANG)) {
        P.chunks.push_back(int32_t(c));
        break;
      }
  }
  if (P.refined) composite_diagonals(P);

  // inlet table
  P.K = 0;
  P.omega = 0.0;
  P.inlet_ids.clear();
  P.inlet_shape.clear();
  if (inlet && inlet->n > 0) {
    if (inlet->K < 0 || inlet->K > kMaxHarmonics || !inlet->node_ids || !inlet->shape ||
        !finite(inlet->omega)) {
      err = "inlet: need 0 <= K <= 16, node_ids, shape and a finite omega";
      return IBFE_EINVAL;
    }
    P.K = inlet->K;
    P.omega = inlet->omega;
    const int64_t nin = inlet->n;
    std::vector<uint8_t> seen(N, 0);
    std::vector<int64_t> keep;  // table rows that carry an unknown
    for (int64_t q = 0; q < nin; ++q) {
      const int64_t id = inlet->node_ids[q];
      if (id < 0 || id >= N) {
        err = "inlet node id out of range";
        return IBFE_EINVAL;
      }
      if (seen[id]++) {
        err = "duplicate inlet node";
        return IBFE_EINVAL;
      }
      // on a refined lattice, points that are not nodes of P carry no unknown
      if (P.refined && !(P.flags[id] & IBFE_FLAG_P)) continue;
      if (!(P.flags[id] & IBFE_FLAG_P) || P.tag[id] != IBFE_TAG_INLET || P.mask[id] != 1) {
        err = "inlet table lists a node that is not an in-vessel inlet node of P";
        return IBFE_EINVAL;
      }
      keep.push_back(q);
    }
    const size_t len = size_t(2 * P.K + 1) * size_t(nin) * 3;
    for (size_t q = 0; q < len; ++q)
      if (!finite(inlet->shape[q])) {
        err = "inlet shape must be finite";
        return IBFE_EINVAL;
      }
    const int64_t nk = int64_t(keep.size());
    P.inlet_ids.resize(nk);
    P.inlet_shape.assign(size_t(2 * P.K + 1) * size_t(nk) * 3, 0.0);
    for (int64_t r = 0; r < nk; ++r) {
      const int64_t q = keep[r];
      P.inlet_ids[r] = inlet->node_ids[q];
      for (int b = 0; b < 2 * P.K + 1; ++b)
        for (int d = 0; d < 3; ++d)
          P.inlet_shape[(size_t(b) * nk + r) * 3 + d] = inlet->shape[(size_t(b) * nin + q) * 3 + d];
    }
  } else if (inlet && inlet->n < 0) {
    err = "inlet n must be >= 0";
    return IBFE_EINVAL;
  }

  // immersed boundary: stencils of Eq. 17 (times h^3) with the kernel of Eq. 18
  P.M = ib ? ib->M : 0;
  if (P.M < 0 || (P.M > 0 && !ib->X) || P.M > (int64_t(1) << 30)) {
    err = "ib: need 0 <= M and X when M > 0";
    return IBFE_EINVAL;
  }
  const int64_t M = P.M;
  P.dS = ib ? ib->dS : 0.0;
  if (M > 0 && !(P.dS > 0.0 && finite(P.dS))) {
    err = "ib: dS must be positive";
    return IBFE_EINVAL;
  }
  P.X.assign(3 * M, 0.0);
  P.U_B.assign(3 * M, 0.0);
  if (M > 0) {
    P.X.assign(ib->X, ib->X + 3 * M);
    if (ib->U_B) P.U_B.assign(ib->U_B, ib->U_B + 3 * M);
  }
  for (int64_t q = 0; q < 3 * M; ++q)
    if (!finite(P.X[q]) || !finite(P.U_B[q])) {
      err = "ib: X and U_B must be finite";
      return IBFE_EINVAL;
    }
  P.ib_idx.assign(64 * M, -1);
  P.ib_w.assign(64 * M, 0.0);
  const int dims[3] = {nx, ny, nz};
  int64_t first_singular = -1;
  for (int64_t i = 0; i < M; ++i) {
    int64_t base[3];
    double wd[3][4];
    for (int d = 0; d < 3; ++d) {
      double xi = P.X[3 * i + d];
      base[d] = int64_t(std::floor((xi - P.origin[d]) / P.h)) - 1;
      for (int a = 0; a < 4; ++a) {
        double xn = P.origin[d] + double(base[d] + a) * P.h;
        wd[d][a] = delta4((xn - xi) / P.h);
      }
    }
    double free2 = 0.0;
    for (int c = 0; c < 4; ++c)
      for (int b = 0; b < 4; ++b)
        for (int a = 0; a < 4; ++a) {
          int64_t ii = base[0] + a, jj = base[1] + b, kk = base[2] + c;
          if (ii < 0 || jj < 0 || kk < 0 || ii > dims[0] || jj > dims[1] || kk > dims[2]) continue;
          int s = a + 4 * b + 16 * c;
          int64_t n = ii + P.sy * jj + P.sz * kk;
          double w = wd[0][a] * wd[1][b] * wd[2][c];
          P.ib_idx[s * M + i] = int32_t(n);
          P.ib_w[s * M + i] = w;
          if (P.flags[n] & IBFE_FLAG_F) free2 += w * w;
        }
    if (free2 < 1e-12 && first_singular < 0) first_singular = i;
  }
  if (P.refined && M > 0) {
    int rc = check_ib_support_refined(P, err);
    if (rc) return rc;
  }
  if (first_singular >= 0) {
    err = "Lagrangian point " + std::to_string(first_singular) + " has no free support node";
    return IBFE_ESINGULAR;
  }
  // node -> (point, weight) lists over free nodes (the spreading operator I_F^T)
  P.sp_node.clear();
  P.sp_ptr.assign(1, 0);
  P.sp_pt.clear();
  P.sp_w.clear();
  P.G_ptr.assign(1, 0);
  P.G_col.clear();
  P.G_val.clear();
  P.G_diag.assign(M, 0.0);
  if (M > 0) {
    std::vector<int64_t> cnt(N + 1, 0);
    for (int64_t q = 0; q < 64 * M; ++q) {
      int32_t n = P.ib_idx[q];
      if (n >= 0 && (P.flags[n] & IBFE_FLAG_F)) ++cnt[n + 1];
    }
    std::vector<int64_t> start(N + 1, 0);
    for (int64_t n = 0; n < N; ++n) start[n + 1] = start[n] + cnt[n + 1];
    std::vector<int32_t> lst_pt(start[N]);
    std::vector<double> lst_w(start[N]);
    std::vector<int64_t> fill(start.begin(), start.end() - 1);
    for (int64_t i = 0; i < M; ++i)          // point order inside each node list
      for (int s = 0; s < 64; ++s) {
        int32_t n = P.ib_idx[s * M + i];
        if (n >= 0 && (P.flags[n] & IBFE_FLAG_F)) {
          lst_pt[fill[n]] = int32_t(i);
          lst_w[fill[n]] = P.ib_w[s * M + i];
          ++fill[n];
        }
      }
    for (int64_t n = 0; n < N; ++n) {
      if (start[n + 1] == start[n]) continue;
      P.sp_node.push_back(int32_t(n));
      for (int64_t q = start[n]; q < start[n + 1]; ++q) {
        P.sp_pt.push_back(lst_pt[q]);
        P.sp_w.push_back(lst_w[q]);
      }
      P.sp_ptr.push_back(int64_t(P.sp_pt.size()));
    }
    // G_ik = sum_{j in F} w_ij w_kj, accumulated row by row
    std::vector<double> acc(M, 0.0);
    std::vector<int32_t> marker(M, -1), cols;
    for (int64_t i = 0; i < M; ++i) {
      cols.clear();
      for (int s = 0; s < 64; ++s) {
        int32_t n = P.ib_idx[s * M + i];
        if (n < 0 || !(P.flags[n] & IBFE_FLAG_F)) continue;
        double wi = P.ib_w[s * M + i];
        for (int64_t q = start[n]; q < start[n + 1]; ++q) {
          int32_t k = lst_pt[q];
          if (marker[k] != int32_t(i)) {
            marker[k] = int32_t(i);
            acc[k] = 0.0;
            cols.push_back(k);
          }
          acc[k] += wi * lst_w[q];
        }
      }
      std::sort(cols.begin(), cols.end());
      for (int32_t k : cols) {
        P.G_col.push_back(k);
        P.G_val.push_back(acc[k]);
        if (k == i) P.G_diag[i] = acc[k];
      }
      P.G_ptr.push_back(int64_t(P.G_col.size()));
    }
  }
  ib_block_inverses(P);
  if (P.params.precond >= 1) {
    int rc = build_multigrid(P, err);
    if (rc) return rc;
  }
  return IBFE_OK;
}

}  // namespace ibfe
