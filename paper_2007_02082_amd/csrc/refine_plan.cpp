// Host set-up of a 2:1 locally refined grid (the paper refines its mesh near
// and inside the immersed boundary, Section 4).  Everything lives on the fine
// lattice (spacing h/2): the 2x2x2 children of flagged base cells are fine
// elements, unflagged base cells are coarse elements (corners at even lattice
// positions), each kept when a corner has mask 1.  A corner of a kept fine
// element strictly inside an edge (one odd coordinate) or a face (two odd
// coordinates) of a kept coarse element is hanging: its value is the mean of
// the 2 edge end points or the 4 face corners.
#include <algorithm>
#include <cmath>

#include "plan.hpp"

namespace ibfe {

namespace {

inline uint8_t side_bit(int ax, int ay, int az) {
  // the element lies on side (1 - a) of its corner a
  return uint8_t(1u << ((1 - ax) + 2 * (1 - ay) + 4 * (1 - az)));
}

}  // namespace

int build_composite_cells(Plan& P, UnionFind& uf, std::string& err) {
  const int bnx = P.bnx, bny = P.bny, bnz = P.bnz;
  const int64_t N = P.N, sy = P.sy, sz = P.sz;
  auto id = [&](int64_t i, int64_t j, int64_t k) { return i + sy * j + sz * k; };
  P.emask.assign(N, 0);
  P.cmask.assign(N, 0);
  P.n_kept = 0;
  std::vector<uint8_t> ckept(size_t(bnx) * bny * bnz, 0);
  for (int bk = 0; bk < bnz; ++bk)
    for (int bj = 0; bj < bny; ++bj)
      for (int bi = 0; bi < bnx; ++bi) {
        const int64_t cell = bi + int64_t(bnx) * (bj + int64_t(bny) * bk);
        if (P.refine[cell]) {
          for (int c = 0; c < 8; ++c) {
            const int64_t c0 = id(2 * bi + (c & 1), 2 * bj + ((c >> 1) & 1), 2 * bk + ((c >> 2) & 1));
            bool kept = false;
            for (int a = 0; a < 8 && !kept; ++a)
              kept = P.mask[c0 + (a & 1) + sy * ((a >> 1) & 1) + sz * ((a >> 2) & 1)] == 1;
            if (!kept) continue;
            ++P.n_kept;
            for (int a = 0; a < 8; ++a) {
              const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
              const int64_t n = c0 + ax + sy * ay + sz * az;
              P.emask[n] |= side_bit(ax, ay, az);
              uf.unite(c0, n);
            }
          }
        } else {
          const int64_t c0 = id(2 * bi, 2 * bj, 2 * bk);
          bool kept = false;
          for (int a = 0; a < 8 && !kept; ++a)
            kept = P.mask[c0 + 2 * ((a & 1) + sy * ((a >> 1) & 1) + sz * ((a >> 2) & 1))] == 1;
          if (!kept) continue;
          ckept[cell] = 1;
          ++P.n_kept;
          for (int a = 0; a < 8; ++a) {
            const int ax = a & 1, ay = (a >> 1) & 1, az = (a >> 2) & 1;
            const int64_t n = c0 + 2 * (ax + sy * ay + sz * az);
            P.cmask[n] |= side_bit(ax, ay, az);
            uf.unite(c0, n);
          }
        }
      }

  // hanging nodes and their parents, in ascending node order
  std::vector<int32_t> hidx(N, -1);
  std::vector<std::pair<int64_t, std::vector<int64_t>>> found;
  for (int bk = 0; bk < bnz; ++bk)
    for (int bj = 0; bj < bny; ++bj)
      for (int bi = 0; bi < bnx; ++bi) {
        if (!ckept[bi + int64_t(bnx) * (bj + int64_t(bny) * bk)]) continue;
        const int x0 = 2 * bi, y0 = 2 * bj, z0 = 2 * bk;
        for (int dz = 0; dz < 3; ++dz)
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx) {
              const int odd = (dx == 1) + (dy == 1) + (dz == 1);
              if (odd == 0 || odd == 3) continue;
              const int64_t n = id(x0 + dx, y0 + dy, z0 + dz);
              if (!P.emask[n] || hidx[n] >= 0) continue;
              std::vector<int64_t> par;
              for (int az = (dz == 1 ? 0 : dz); az <= (dz == 1 ? 2 : dz); az += 2)
                for (int ay = (dy == 1 ? 0 : dy); ay <= (dy == 1 ? 2 : dy); ay += 2)
                  for (int ax = (dx == 1 ? 0 : dx); ax <= (dx == 1 ? 2 : dx); ax += 2)
                    par.push_back(id(x0 + ax, y0 + ay, z0 + az));
              hidx[n] = 0;  // claimed; the real index is assigned after sorting
              found.emplace_back(n, std::move(par));
            }
      }
  std::sort(found.begin(), found.end(),
            [](const auto& a, const auto& b) { return a.first < b.first; });
  const int64_t nh = int64_t(found.size());
  if (nh > (int64_t(1) << 30)) {
    err = "too many hanging nodes";
    return IBFE_EINVAL;
  }
  P.hang_ids.assign(nh, 0);
  P.hang_par.assign(4 * nh, -1);
  std::vector<std::pair<int64_t, int32_t>> edges;  // (parent, hanging index)
  for (int64_t k = 0; k < nh; ++k) {
    const int64_t n = found[k].first;
    std::vector<int64_t>& par = found[k].second;
    std::sort(par.begin(), par.end());
    P.hang_ids[k] = int32_t(n);
    hidx[n] = int32_t(k);
    for (size_t q = 0; q < par.size(); ++q) {
      P.hang_par[q * nh + k] = int32_t(par[q]);
      edges.emplace_back(par[q], int32_t(k));
      uf.unite(n, par[q]);
    }
  }
  std::sort(edges.begin(), edges.end());
  P.par_ids.clear();
  P.par_ptr.assign(1, 0);
  P.par_child.clear();
  P.par_w.clear();
  P.par_slot.assign(N, -1);
  for (size_t e = 0; e < edges.size(); ++e) {
    const int64_t q = edges[e].first;
    if (P.par_ids.empty() || P.par_ids.back() != q) {
      if (!P.par_ids.empty()) P.par_ptr.push_back(int32_t(P.par_child.size()));
      P.par_slot[q] = int32_t(P.par_ids.size());
      P.par_ids.push_back(int32_t(q));
    }
    const int32_t k = edges[e].second;
    P.par_child.push_back(k);
    const int np = P.hang_par[3 * nh + k] >= 0 ? 4 : 2;
    P.par_w.push_back(1.0 / np);
  }
  if (!P.par_ids.empty()) P.par_ptr.push_back(int32_t(P.par_child.size()));
  return IBFE_OK;
}

void composite_diagonals(Plan& P) {
  // per-cell diagonal entries: mass (h/3)^3, stiffness 3 (1/h)(h/3)^2 = h/3
  const double hf = P.h, hc = P.hb;
  const double mf = hf * hf * hf / 27.0, mc = hc * hc * hc / 27.0;
  const double kf = hf / 3.0, kc = hc / 3.0;
  const int64_t N = P.N, nh = int64_t(P.hang_ids.size());
  P.dmass.assign(N, 0.0);
  P.dstiff.assign(N, 0.0);
  for (int64_t n = 0; n < N; ++n) {
    if (!(P.flags[n] & IBFE_FLAG_P)) continue;
    const int ef = __builtin_popcount(P.emask[n]), ec = __builtin_popcount(P.cmask[n]);
    P.dmass[n] = mf * ef + mc * ec;
    P.dstiff[n] = kf * ef + kc * ec;
  }
  // row sums: each kept cell gives an eighth of its volume to each of its corners
  P.lmass.assign(N, 0.0);
  for (int64_t n = 0; n < N; ++n) {
    if (!(P.flags[n] & IBFE_FLAG_P)) continue;
    P.lmass[n] = (hf * hf * hf / 8.0) * __builtin_popcount(P.emask[n]) +
                 (hc * hc * hc / 8.0) * __builtin_popcount(P.cmask[n]);
  }
  for (size_t s = 0; s < P.par_ids.size(); ++s)
    for (int32_t q = P.par_ptr[s]; q < P.par_ptr[s + 1]; ++q)
      P.lmass[P.par_ids[s]] += P.par_w[q] * (hf * hf * hf / 8.0) * __builtin_popcount(P.emask[P.hang_ids[P.par_child[q]]]);
  std::vector<double> base_mass(P.dmass);
  for (size_t s = 0; s < P.par_ids.size(); ++s) {
    const int64_t n = P.par_ids[s];
    for (int32_t q = P.par_ptr[s]; q < P.par_ptr[s + 1]; ++q) {
      const int64_t h = P.hang_ids[P.par_child[q]];
      const int eh = __builtin_popcount(P.emask[h]);
      P.dmass[n] += P.par_w[q] * mf * eh;
      P.dstiff[n] += P.par_w[q] * kf * eh;
    }
  }
  (void)nh;
  // Chebyshev lower bound for the constrained mass on F with D' = dmass:
  // eig >= (1/8) min_F d(n) / d'(n)
  double ratio = 1.0;
  for (int64_t n = 0; n < N; ++n)
    if (P.flags[n] & IBFE_FLAG_F) ratio = std::min(ratio, base_mass[n] / P.dmass[n]);
  P.mass_lmin = 0.125 * ratio;
}

void ib_band_mask(const Plan& P, std::vector<uint8_t>& ok) {
  ok.assign(P.N, 0);
  for (int bk = 0; bk < P.bnz; ++bk)
    for (int bj = 0; bj < P.bny; ++bj)
      for (int bi = 0; bi < P.bnx; ++bi) {
        if (!P.refine[bi + int64_t(P.bnx) * (bj + int64_t(P.bny) * bk)]) continue;
        for (int dz = 0; dz < 3; ++dz)
          for (int dy = 0; dy < 3; ++dy)
            for (int dx = 0; dx < 3; ++dx)
              ok[(2 * bi + dx) + P.sy * (2 * bj + dy) + P.sz * (2 * bk + dz)] = 1;
      }
  for (int32_t n : P.hang_ids) ok[n] = 0;
}

int check_ib_support_refined(const Plan& P, std::string& err) {
  std::vector<uint8_t> ok;
  ib_band_mask(P, ok);
  for (int64_t q = 0; q < int64_t(P.ib_idx.size()); ++q) {
    const int32_t n = P.ib_idx[q];
    if (n >= 0 && !ok[n]) {
      err = "Lagrangian point " + std::to_string(q % std::max<int64_t>(1, P.M)) +
            ": kernel support leaves the refined band";
      return IBFE_EINVAL;
    }
  }
  return IBFE_OK;
}

}  // namespace ibfe
