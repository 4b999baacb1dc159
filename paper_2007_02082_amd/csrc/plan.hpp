// Host-side set-up of one flow problem: validation, derived node sets on the
// masked Q1 grid, canonical ordering, IB stencils and the IB Gram matrix.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "ibfe.h"

namespace ibfe {

constexpr int kChunk = 64;      // nodes per chunk (one wavefront)
constexpr double kLaneFill = 0.75;  // per-lane node lists below this fill of the chunks
constexpr int kIBBlock = 128;       // points per diagonal block of the force-solve preconditioner
constexpr int kMaxHarmonics = 16;
constexpr int kMaxFloating = 8; // outlet-less connected parts supported

constexpr uint8_t kMgP = 1u, kMgPp = 16u;
constexpr int kZBPlanes = 8;     // most planes per z-blocked column item
constexpr int kZBMinItems = 4096;
constexpr int kMgCoarsestMax = 1024;

// One level of the geometric multigrid hierarchy of the pressure Poisson
// operator (level 0 = the grid itself).  Node flags use bit 0 = in P, bit 4 =
// pressure unknown (P minus Dirichlet).
struct MGLevel {
  int nx = 0, ny = 0, nz = 0;
  double h = 0.0;
  int64_t N = 0, sy = 0, sz = 0;
  std::vector<uint8_t> emask, flags;
  std::vector<int32_t> chunks;    // 64-node chunks holding a node of P
  std::vector<int32_t> zitems;    // z-blocked column items: plane block of each item
  std::vector<int32_t> zlanes;    // 64 in-plane positions per item (-1 = none)
  int zb = kZBPlanes;             // planes per column item
  std::vector<int64_t> unknowns;  // ids of pressure unknowns (coarsest level only)
  std::vector<double> inv;        // dense inverse on `unknowns` (coarsest level only)
};


struct UnionFind {
  std::vector<int64_t> parent;
  explicit UnionFind(int64_t n);
  int64_t find(int64_t a);
  void unite(int64_t a, int64_t b);
};

struct Plan {
  // grid: the node lattice (with refinement: the fine lattice of spacing h/2)
  int nx = 0, ny = 0, nz = 0;
  double h = 0.0, origin[3] = {0, 0, 0};
  // 2:1 refinement: base cells, base spacing, per-node bits of the kept
  // unrefined cells around an all-even lattice node (bit s as in emask, for the
  // base cell (I-1+sx, J-1+sy, K-1+sz) around base node (I, J, K))
  bool refined = false;
  int bnx = 0, bny = 0, bnz = 0;
  double hb = 0.0;
  std::vector<uint8_t> refine;   // base cells (refined only)
  std::vector<uint8_t> cmask;    // per lattice node (refined only)
  // hanging nodes (ascending ids) with their 2 or 4 parents ([4][nh], -1 unused)
  std::vector<int32_t> hang_ids;
  std::vector<int32_t> hang_par;
  // parents: ascending ids, CSR of (hanging index, weight); slot per lattice node
  std::vector<int32_t> par_ids, par_ptr, par_child;
  std::vector<double> par_w;
  std::vector<int32_t> par_slot;
  // lumped diagonals of the constrained mass and stiffness forms (refined only):
  // d'(n) = a_nn + sum over hanging children h of w_h a_hh
  std::vector<double> dmass, dstiff;
  // row sums of the constrained mass C^T M C (the lumped mass of the wall-shear
  // gradient recovery; refined only)
  std::vector<double> lmass;
  double mass_lmin = 0.125;      // lower bound of eig(D'^-1 M) on F
  int64_t N = 0;                 // grid nodes
  int64_t sy = 0, sz = 0;        // id strides in y and z
  // physics
  ibfe_params params{};
  // per node
  std::vector<uint8_t> mask, tag;
  std::vector<uint8_t> emask;    // bit s = sx + 2 sy + 4 sz: cell (i-1+sx, j-1+sy, k-1+sz) kept
  std::vector<uint8_t> flags;    // IBFE_FLAG_* bits
  std::vector<int8_t> float_slot;// -1, or slot of the outlet-less part the node belongs to
  int n_floating = 0;
  std::vector<int64_t> float_count; // P' nodes per floating slot
  // sets
  std::vector<int64_t> P_ids;    // canonical order
  int64_t n_free = 0, n_pfree = 0, n_kept = 0;
  std::vector<int32_t> chunks;   // 64-node chunks holding at least one node of P
  // inlet table
  int K = 0;
  double omega = 0.0;
  std::vector<int64_t> inlet_ids;
  std::vector<double> inlet_shape;   // (2K+1) x n x 3
  // immersed boundary
  int64_t M = 0;
  double dS = 0.0;
  std::vector<double> X, U_B;        // M x 3
  std::vector<int32_t> ib_idx;       // [64][M]: support node id or -1
  std::vector<double> ib_w;          // [64][M]: weights (0 where idx = -1)
  std::vector<int64_t> G_ptr;        // CSR of G = I_F I_F^T (M x M)
  std::vector<int32_t> G_col;
  std::vector<double> G_val, G_diag;
  // block-Jacobi preconditioner of the force solve: inverses of the diagonal
  // blocks of G over kIBBlock consecutive points, [block][column j][row i]
  std::vector<float> G_binv;
  std::vector<int32_t> sp_node;      // nodes of F inside some support
  std::vector<int64_t> sp_ptr;       // CSR rows over sp_node: (point, weight)
  std::vector<int32_t> sp_pt;
  std::vector<double> sp_w;
  // multigrid hierarchy of the pressure operator (empty unless precond == 2)
  std::vector<MGLevel> mg;
};

// Build the multigrid hierarchy from level 0 (already holding emask/flags).
int build_multigrid(Plan& plan, std::string& err);
// z-blocked column items of a level: item q covers planes zb items[q] .. zb
// items[q] + zb - 1 at the in-plane positions lanes[64 q .. 64 q + 63]: the
// positions where some plane of the block has a kept cell, ascending, 64 per
// item, the last item of a block padded with -1.
void column_items(const std::vector<uint8_t>& emask, int64_t sz, int nplanes, int zb,
                  std::vector<int32_t>& items, std::vector<int32_t>& lanes);
// Column items with the most planes per item (8, 4 or 2) that still gives at
// least kZBMinItems items (enough wavefronts to fill the chip); returns zb.
int choose_column_items(const std::vector<uint8_t>& emask, int64_t sz, int nplanes,
                        std::vector<int32_t>& items, std::vector<int32_t>& lanes);

// Kept elements, hanging nodes and parents of a refined lattice: fills emask
// (children of refined cells), cmask, the hanging and parent tables and joins
// the corners of every kept element (and hanging nodes with their parents).
int build_composite_cells(Plan& plan, UnionFind& uf, std::string& err);
// Lumped diagonals and the Chebyshev lower bound of a refined plan (after flags).
void composite_diagonals(Plan& plan);
// Every IB support node inside the closure of a refined cell and not hanging.
int check_ib_support_refined(const Plan& plan, std::string& err);
// Lattice nodes an IB kernel support may touch on a refined lattice: nodes in the
// closure of a flagged cell that are not hanging (1), all others 0.
void ib_band_mask(const Plan& plan, std::vector<uint8_t>& ok);

// Returns IBFE_OK or an error code with `err` set.
int build_plan(const ibfe_grid* grid, const ibfe_ib* ib, const ibfe_params* params,
               const ibfe_inlet* inlet, Plan& plan, std::string& err);

double delta4(double r);

}  // namespace ibfe
