// Host construction of the geometric multigrid hierarchy for the pressure
// increment equation (Eq. 12 discretised with Q1, Dirichlet at outlets,
// natural conditions elsewhere).  Coarse cells are unions of 2x2x2 fine cells;
// a coarse cell is kept when one of its children is kept; a coarse node is a
// Dirichlet node when the fine node at the same place is one.  The coarse
// operator is the Q1 stiffness of the coarse kept cells (spacing 2h).  The
// coarsest level (at most kMgCoarsestMax unknowns) is solved with a dense
// inverse; outlet-less connected parts get a rank-one term per part so that
// the inverse acts as the pseudo-inverse on mean-free data.
#include <algorithm>
#include <cmath>
#include <numeric>

#include "plan.hpp"

namespace ibfe {

namespace {

void chunk_list(const std::vector<uint8_t>& emask, std::vector<int32_t>& chunks) {
  chunks.clear();
  const int64_t N = int64_t(emask.size());
  for (int64_t c = 0; c * kChunk < N; ++c) {
    const int64_t hi = std::min<int64_t>(N, (c + 1) * kChunk);
    for (int64_t n = c * kChunk; n < hi; ++n)
      if (emask[n]) {
        chunks.push_back(int32_t(c));
        break;
      }
  }
}

int64_t find_root(std::vector<int64_t>& parent, int64_t a) {
  while (parent[a] != a) {
    parent[a] = parent[parent[a]];
    a = parent[a];
  }
  return a;
}

// Per-cell stiffness entry for a neighbour offset with t nonzero components
// (cube of side h): sum_d k(o_d) prod_{e != d} m(o_e).
double cell_stiffness(int t, double h) {
  const double m0 = h / 3.0, m1 = h / 6.0, k0 = 1.0 / h, k1 = -1.0 / h;
  double kv = 0.0;
  for (int d = 0; d < 3; ++d) {
    double term = (d < t) ? k1 : k0;
    for (int a = 0; a < 3; ++a)
      if (a != d) term *= (a < t) ? m1 : m0;
    kv += term;
  }
  return kv;
}

// Dense symmetric positive definite inverse by Cholesky (in place on a, n x n).
bool spd_inverse(std::vector<double>& a, int n) {
  std::vector<double> L(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    double d = a[size_t(j) * n + j];
    for (int k = 0; k < j; ++k) d -= L[size_t(j) * n + k] * L[size_t(j) * n + k];
    if (!(d > 0.0)) return false;
    const double ljj = std::sqrt(d);
    L[size_t(j) * n + j] = ljj;
    for (int i = j + 1; i < n; ++i) {
      double s = a[size_t(i) * n + j];
      for (int k = 0; k < j; ++k) s -= L[size_t(i) * n + k] * L[size_t(j) * n + k];
      L[size_t(i) * n + j] = s / ljj;
    }
  }
  // inverse of L (lower), then A^-1 = L^-T L^-1
  std::vector<double> Li(size_t(n) * n, 0.0);
  for (int j = 0; j < n; ++j) {
    Li[size_t(j) * n + j] = 1.0 / L[size_t(j) * n + j];
    for (int i = j + 1; i < n; ++i) {
      double s = 0.0;
      for (int k = j; k < i; ++k) s += L[size_t(i) * n + k] * Li[size_t(k) * n + j];
      Li[size_t(i) * n + j] = -s / L[size_t(i) * n + i];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j <= i; ++j) {
      double s = 0.0;
      for (int k = i; k < n; ++k) s += Li[size_t(k) * n + i] * Li[size_t(k) * n + j];
      a[size_t(i) * n + j] = s;
      a[size_t(j) * n + i] = s;
    }
  return true;
}

void coarsest_inverse(MGLevel& L) {
  L.unknowns.clear();
  for (int64_t n = 0; n < L.N; ++n)
    if (L.flags[n] & kMgPp) L.unknowns.push_back(n);
  const int m = int(L.unknowns.size());
  L.inv.clear();
  if (m == 0 || m > kMgCoarsestMax) return;
  std::vector<int32_t> pos(L.N, -1);
  for (int q = 0; q < m; ++q) pos[L.unknowns[q]] = q;
  std::vector<double> A(size_t(m) * m, 0.0);
  double kc[4];
  for (int t = 0; t < 4; ++t) kc[t] = cell_stiffness(t, L.h);
  for (int q = 0; q < m; ++q) {
    const int64_t n = L.unknowns[q];
    const uint32_t e = L.emask[n];
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          uint32_t cm = e;
          const int o[3] = {ox, oy, oz};
          for (int d = 0; d < 3; ++d)
            if (o[d] != 0) {
              uint32_t side = 0;
              for (int s = 0; s < 8; ++s)
                if ((((s >> d) & 1) == 1) == (o[d] > 0)) side |= 1u << s;
              cm &= side;
            }
          const int cnt = __builtin_popcount(cm);
          if (!cnt) continue;
          const int64_t nb = n + ox + L.sy * oy + L.sz * oz;
          if (nb < 0 || nb >= L.N || pos[nb] < 0) continue;
          const int t = (ox != 0) + (oy != 0) + (oz != 0);
          A[size_t(q) * m + pos[nb]] += kc[t] * cnt;
        }
  }
  // outlet-less connected parts: rank-one terms gamma 1_c 1_c^T
  std::vector<int64_t> parent(L.N);
  std::iota(parent.begin(), parent.end(), 0);
  for (int k = 0; k < L.nz; ++k)
    for (int j = 0; j < L.ny; ++j)
      for (int i = 0; i < L.nx; ++i) {
        const int64_t c0 = i + L.sy * j + L.sz * k;
        if (!((L.emask[c0] >> 7) & 1u)) continue;
        for (int a = 1; a < 8; ++a) {
          const int64_t nb = c0 + (a & 1) + L.sy * ((a >> 1) & 1) + L.sz * ((a >> 2) & 1);
          int64_t r0 = find_root(parent, c0), r1 = find_root(parent, nb);
          if (r0 != r1) parent[std::max(r0, r1)] = std::min(r0, r1);
        }
      }
  std::vector<uint8_t> anchored(L.N, 0);
  for (int64_t n = 0; n < L.N; ++n)
    if ((L.flags[n] & kMgP) && !(L.flags[n] & kMgPp)) anchored[find_root(parent, n)] = 1;
  double maxdiag = 0.0;
  for (int q = 0; q < m; ++q) maxdiag = std::max(maxdiag, A[size_t(q) * m + q]);
  std::vector<std::vector<int>> parts;
  std::vector<int64_t> part_of_root(L.N, -1);
  for (int q = 0; q < m; ++q) {
    const int64_t r = find_root(parent, L.unknowns[q]);
    if (anchored[r]) continue;
    if (part_of_root[r] < 0) {
      part_of_root[r] = int64_t(parts.size());
      parts.emplace_back();
    }
    parts[part_of_root[r]].push_back(q);
  }
  for (auto& part : parts) {
    const double gamma = maxdiag / double(part.size());
    for (int a : part)
      for (int b : part) A[size_t(a) * m + b] += gamma;
  }
  if (spd_inverse(A, m)) L.inv.swap(A);
}

}  // namespace

void column_items(const std::vector<uint8_t>& emask, int64_t sz, int nplanes, int zb,
                  std::vector<int32_t>& items, std::vector<int32_t>& lanes) {
  const int npb = (nplanes + zb - 1) / zb;
  items.clear();
  lanes.clear();
  std::vector<uint8_t> used(size_t(sz), 0);
  for (int pb = 0; pb < npb; ++pb) {
    std::fill(used.begin(), used.end(), 0);
    for (int k = pb * zb; k < std::min(nplanes, (pb + 1) * zb); ++k)
      for (int64_t l = 0; l < sz; ++l) used[l] |= emask[k * sz + l] ? 1 : 0;
    int fill = 0;
    for (int64_t l = 0; l < sz; ++l) {
      if (!used[l]) continue;
      if (fill == 0) items.push_back(pb);
      lanes.push_back(int32_t(l));
      fill = (fill + 1) % kChunk;
    }
    if (fill)
      for (; fill < kChunk; ++fill) lanes.push_back(-1);
  }
}

int choose_column_items(const std::vector<uint8_t>& emask, int64_t sz, int nplanes,
                        std::vector<int32_t>& items, std::vector<int32_t>& lanes) {
  int zb = kZBPlanes;
  column_items(emask, sz, nplanes, zb, items, lanes);
  while (zb > 2 && int64_t(items.size()) < kZBMinItems) {
    zb /= 2;
    column_items(emask, sz, nplanes, zb, items, lanes);
  }
  return zb;
}

int build_multigrid(Plan& P, std::string& err) {
  (void)err;
  P.mg.clear();
  MGLevel L0;
  L0.nx = P.nx;
  L0.ny = P.ny;
  L0.nz = P.nz;
  L0.h = P.h;
  L0.N = P.N;
  L0.sy = P.sy;
  L0.sz = P.sz;
  L0.emask = P.emask;
  L0.flags.assign(P.N, 0);
  for (int64_t n = 0; n < P.N; ++n) {
    const uint8_t f = P.flags[n];
    if (f & IBFE_FLAG_P) L0.flags[n] = kMgP | ((f & IBFE_FLAG_PDIR) ? 0 : kMgPp);
  }
  L0.chunks = P.chunks;
  if (!P.refined) L0.zb = choose_column_items(L0.emask, L0.sz, L0.nz + 1, L0.zitems, L0.zlanes);
  P.mg.push_back(std::move(L0));
  // Chebyshev preconditioner: the grid level alone, smoothed without a coarse correction
  if (P.params.precond == 1) return IBFE_OK;
  if (P.refined) {
    // level 1 = the base grid: a base cell is kept when it is a kept unrefined
    // cell or one of its 2x2x2 children is kept; Dirichlet colocated as below
    const MGLevel& F = P.mg.back();
    MGLevel C;
    C.nx = P.bnx;
    C.ny = P.bny;
    C.nz = P.bnz;
    C.h = P.hb;
    C.sy = C.nx + 1;
    C.sz = C.sy * (C.ny + 1);
    C.N = C.sz * (C.nz + 1);
    C.emask.assign(C.N, 0);
    for (int k = 0; k < C.nz; ++k)
      for (int j = 0; j < C.ny; ++j)
        for (int i = 0; i < C.nx; ++i) {
          const int64_t f0 = 2 * i + F.sy * 2 * j + F.sz * 2 * k;
          bool kept;
          if (P.refine[i + int64_t(C.nx) * (j + int64_t(C.ny) * k)]) {
            kept = false;
            for (int a = 0; a < 8 && !kept; ++a)
              kept = (P.emask[f0 + (a & 1) + F.sy * ((a >> 1) & 1) + F.sz * ((a >> 2) & 1)] >> 7) & 1u;
          } else {
            kept = (P.cmask[f0] >> 7) & 1u;
          }
          if (!kept) continue;
          for (int a = 0; a < 8; ++a) {
            const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
            const int64_t cn = (i + ax) + C.sy * (j + ay) + C.sz * (k + az);
            C.emask[cn] |= uint8_t(1u << ((1 - ax) + 2 * (1 - ay) + 4 * (1 - az)));
          }
        }
    C.flags.assign(C.N, 0);
    for (int k = 0; k <= C.nz; ++k)
      for (int j = 0; j <= C.ny; ++j)
        for (int i = 0; i <= C.nx; ++i) {
          const int64_t cn = i + C.sy * j + C.sz * k;
          if (!C.emask[cn]) continue;
          const int64_t fn = 2 * i + F.sy * 2 * j + F.sz * 2 * k;
          const bool dir = (F.flags[fn] & kMgP) && !(F.flags[fn] & kMgPp);
          C.flags[cn] = kMgP | (dir ? 0 : kMgPp);
        }
    chunk_list(C.emask, C.chunks);
    C.zb = choose_column_items(C.emask, C.sz, C.nz + 1, C.zitems, C.zlanes);
    P.mg.push_back(std::move(C));
  }
  auto unknowns = [](const MGLevel& L) {
    int64_t c = 0;
    for (uint8_t f : L.flags) c += (f & kMgPp) ? 1 : 0;
    return c;
  };
  while (true) {
    const MGLevel& F = P.mg.back();
    if (unknowns(F) <= kMgCoarsestMax) break;
    if ((F.nx & 1) || (F.ny & 1) || (F.nz & 1) || F.nx < 2 || F.ny < 2 || F.nz < 2) break;
    MGLevel C;
    C.nx = F.nx / 2;
    C.ny = F.ny / 2;
    C.nz = F.nz / 2;
    C.h = 2.0 * F.h;
    C.sy = C.nx + 1;
    C.sz = C.sy * (C.ny + 1);
    C.N = C.sz * (C.nz + 1);
    C.emask.assign(C.N, 0);
    for (int k = 0; k < C.nz; ++k)
      for (int j = 0; j < C.ny; ++j)
        for (int i = 0; i < C.nx; ++i) {
          bool kept = false;
          for (int a = 0; a < 8 && !kept; ++a) {
            const int64_t fn = (2 * i + (a & 1)) + F.sy * (2 * j + ((a >> 1) & 1)) + F.sz * (2 * k + ((a >> 2) & 1));
            kept = (F.emask[fn] >> 7) & 1u;  // fine cell with lower corner fn
          }
          if (!kept) continue;
          for (int a = 0; a < 8; ++a) {
            const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
            const int64_t cn = (i + ax) + C.sy * (j + ay) + C.sz * (k + az);
            C.emask[cn] |= uint8_t(1u << ((1 - ax) + 2 * (1 - ay) + 4 * (1 - az)));
          }
        }
    C.flags.assign(C.N, 0);
    for (int k = 0; k <= C.nz; ++k)
      for (int j = 0; j <= C.ny; ++j)
        for (int i = 0; i <= C.nx; ++i) {
          const int64_t cn = i + C.sy * j + C.sz * k;
          if (!C.emask[cn]) continue;
          const int64_t fn = 2 * i + F.sy * 2 * j + F.sz * 2 * k;
          const bool dir = (F.flags[fn] & kMgP) && !(F.flags[fn] & kMgPp);
          C.flags[cn] = kMgP | (dir ? 0 : kMgPp);
        }
    chunk_list(C.emask, C.chunks);
    C.zb = choose_column_items(C.emask, C.sz, C.nz + 1, C.zitems, C.zlanes);
    P.mg.push_back(std::move(C));
  }
  coarsest_inverse(P.mg.back());
  return IBFE_OK;
}

}  // namespace ibfe
