// Step driver and C ABI of the IPCS + BCE-IB time step (Section 2.4 order):
// tentative velocity (BiCGStab), IB force solve (CG on G = I_F I_F^T) and
// spreading, pressure increment (PCG), L2 velocity correction (PCG).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cxxabi.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <chrono>
#include <condition_variable>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "ibfe.h"
#include "plan.hpp"
#include "step_kernels.hpp"
#include "zblock.hpp"
#include "mg.hpp"
#include "composite.hpp"
#include "conv.hpp"
#include "ib_pcg.hpp"
#include "strain.hpp"
#include "wss.hpp"
#include "steady.hpp"
#include "ib_move.hpp"
#include "sort_scan.hpp"


using namespace ibfe;

namespace ibfe {
// Thread-local message of the last failure (shared by every translation unit).
std::string& last_error_message() {
  thread_local std::string msg;
  return msg;
}
}  // namespace ibfe

namespace {

int fail(int code, const std::string& msg) {
  ibfe::last_error_message() = msg;
  return code;
}

#define HIP_TRY(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return fail(IBFE_EHIP, std::string(#expr " failed: ") + hipGetErrorString(e_));   \
  } while (0)

#define CHECK_LAUNCH() HIP_TRY(hipGetLastError())

constexpr uint32_t kFlagPp = 16u;  // pressure unknown: node of P that is not an outlet node
constexpr int kMaxRows = 8;        // partial rows per reduction (K <= 8)
constexpr int kRedBlocks = 2048;   // workgroups of a reducing kernel (8 per CU)
constexpr int kMaxSweeps = 12;     // refinement sweeps of a mixed-precision solve
// tightest relative target of an inner FP32 solve: each refinement sweep asks for
// max(kInnerRtol, 0.5 rtol / residual); tighter floors cost more inner iterations
// than the FP64 sweeps they save
constexpr double kInnerRtol = 1e-3;
// the floor of the tensor-preconditioned mass correction: with 1e-4 its first sweep
// usually meets the target, one FP64 residual sweep fewer per step for about the
// same number of inner steps (1e-3 .. 1e-6 measured within 1 % of each other)
constexpr double kTmInnerRtol = 1e-4;

enum ScalSlot { kScS1 = 0, kScIB, kScS3, kScS4, kScS1i, kScS3i, kScS4i, kScMisc, kNumScal };

int blocks_for(int nchunks) { return (nchunks + kWaves - 1) / kWaves; }
int red_blocks(int nchunks) { return std::max(1, std::min(kRedBlocks, blocks_for(nchunks))); }
int blocks_lin(int64_t n) { return int((n + kBlock - 1) / kBlock); }

}  // namespace

struct ibfe_plan {
  Plan p;
};

// Device copy of one multigrid level (node-0 pointers into padded planes).
template <typename T>
struct MGDev {
  int nx = 0, ny = 0, nz = 0, nchunks = 0, nzitems = 0, zb = kZBPlanes;
  int64_t N = 0, sy = 0, sz = 0, halo = 0, stride = 0;
  uint8_t* emask = nullptr;
  uint8_t* flags = nullptr;
  NodeList nl;
  int* zitems = nullptr;
  int* zlanes = nullptr;
  T *b = nullptr, *x = nullptr, *xt = nullptr, *d = nullptr, *r = nullptr;
  double kc[4] = {0, 0, 0, 0};  // per-cell stiffness entries at this spacing
  bool composite = false;       // level 0 of a refined lattice (composite operator)
  int m = 0;                    // coarsest: unknowns with a dense inverse
  int64_t* ids = nullptr;
  T* inv = nullptr;
};

// Per-dispatch kernel timer (ibfe_set_kernel_timing): while it is on, every
// dispatch of the context carries a start/end event pair recorded by the
// dispatch packet itself (hipExtLaunchKernelGGL, no extra packets), tagged with
// the kernel's name.  The Krylov drivers mark where each iteration's dispatches
// begin; dispatches of iterations past convergence (which return at once) are
// dropped.  collect() resolves the pairs and sums them per kernel name.
struct KTimer {
  std::vector<hipEvent_t> ev;     // 2 per recorded dispatch (a pool, reused)
  std::vector<const char*> tag;   // kernel name of each recorded dispatch
  std::vector<uint8_t> skip;      // 1: dispatch past convergence, not counted
  size_t used = 0;
  std::vector<size_t> marks;      // first dispatch of each iteration of the current solve
  struct Acc {
    double ms = 0.0;
    int64_t launches = 0;
  };
  std::map<std::string, Acc> acc;
  std::string only;               // non-empty: time this kernel's dispatches only

  ~KTimer() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  // event pair for the next dispatch (false: no event could be created)
  bool next(const char* name, hipEvent_t& e0, hipEvent_t& e1) {
    while (ev.size() < 2 * used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return false;
      ev.push_back(e);
    }
    if (tag.size() < used + 1) {
      tag.resize(used + 1);
      skip.resize(used + 1);
    }
    e0 = ev[2 * used];
    e1 = ev[2 * used + 1];
    tag[used] = name;
    skip[used] = 0;
    ++used;
    return true;
  }
  void begin_solve() { marks.clear(); }
  void mark() { marks.push_back(used); }
  // iterations iters.. of the current solve returned at once: drop their dispatches
  void drop_from(int iters) {
    if (iters >= 0 && size_t(iters) < marks.size())
      for (size_t i = marks[size_t(iters)]; i < used; ++i) skip[i] = 1;
    marks.clear();
  }
};

struct ibfe_ctx {
  Plan plan;
  hipStream_t stream = nullptr;
  ibfe_alloc alloc{};
  bool user_alloc = false;
  std::vector<void*> blocks;

  int64_t halo = 0, stride = 0;   // padded plane length
  int nchunks = 0;
  int ib_nchunks = 0;
  int64_t mstride = 0;            // padded plane length of IB vectors
  int nP = 0;

  // geometry (node-0 pointers)
  uint8_t* emask = nullptr;
  uint8_t* flags = nullptr;
  int8_t* slot = nullptr;
  NodeList nl;                    // active nodes (P and hanging)
  NodeList ib_nl;                 // Lagrangian points
  int* zitems = nullptr;          // z-blocked column items (plane block of each item)
  int* zlanes = nullptr;          // their 64 in-plane positions (-1 = none)
  int nzitems = 0, zb = kZBPlanes;
  // the walked positions' cell bits and flags in walk order, and mixed mode's
  // walk-order vectors of the mass correction (its residual and Chebyshev d)
  uint8_t* em_im = nullptr;
  uint8_t* fl_im = nullptr;
  int64_t imstride = 0;
  float* rim = nullptr;
  float* dim = nullptr;
  int64_t* pids = nullptr;
  double* float_count = nullptr;
  double* float_means = nullptr;

  // state and fields (node-0 pointers; velocities have 3 planes)
  double *u = nullptr, *p = nullptr, *u_next = nullptr, *p_next = nullptr;
  double *g = nullptr, *ustar = nullptr, *uib = nullptr, *phi = nullptr;
  double* coef64 = nullptr;     // assembled advection-diffusion stencil (advdiff 1)
  float* coef32 = nullptr;
  double* dinvS64 = nullptr;     // matrix-free form: inverse Jacobi diagonal of the rows
  float* dinvS32 = nullptr;
  double* w64 = nullptr;         // u^n copied per step: the matrix-free operators' advecting velocity
  float* w32 = nullptr;          // (FP64, and FP32 in mixed mode)
  double* w[10] = {};   // FP64 Krylov work vectors, 3 planes each
  float* v32[10] = {};  // FP32 Krylov work vectors (mixed mode), 3 planes each
  double* compact = nullptr;

  // immersed boundary
  int32_t* ib_idx = nullptr;
  double* ib_w = nullptr;
  double* UB = nullptr;
  int64_t* G_ptr = nullptr;
  int32_t* G_col = nullptr;
  double* G_val = nullptr;
  double* G_diag = nullptr;
  float* G_binv = nullptr;
  int32_t* sp_node = nullptr;
  int64_t* sp_ptr = nullptr;
  int32_t* sp_pt = nullptr;
  double* sp_wt = nullptr;
  uint8_t* ib_band = nullptr;  // refined lattice: nodes a kernel support may touch
  double* ibv[7] = {};  // b, lam, r, p, q, z, p' (3 planes of mstride)
  int n_sp = 0;         // nodes of the spreading lists
  // moving Lagrangian points: device rebuild buffers, allocated on the first
  // ibfe_set_points (the spreading lists and G are then reallocated at their
  // largest sizes)
  struct Moving {
    bool ready = false;
    double* X = nullptr;  // M x 3
    uint32_t *keys = nullptr, *vals = nullptr, *skeys = nullptr, *svals = nullptr;
    int *flag = nullptr, *pos = nullptr, *counters = nullptr;
    int64_t* cnt = nullptr;
    uint32_t* hist = nullptr;  // radix digit counts, 256 per tile of the pairs
    void* sums = nullptr;      // tile sums of the scans (8 bytes per tile)
    int64_t g_cap = 0;         // entries of G the device arrays hold
  } mv;
  int device = 0;          // HIP device the context was created on
  ibfe_batcher* batcher = nullptr;            // joins the mass-correction sequences of contexts
  hipEvent_t ev_ready = nullptr, ev_done = nullptr;
  bool ib_valid = true;  // false after a failed ibfe_set_points
  // ibv[1] holds the force of the last step: the initial guess of the next force
  // solve (the right-hand side U_B - I u* changes little from step to step)
  bool lam_warm = false;
  // Phi and the mass correction delta of the last step start the next step's
  // mixed-precision solves (both change little from step to step)
  double* delta = nullptr;
  bool phi_warm = false, delta_warm = false;

  // inlet
  int64_t* inlet_ids = nullptr;
  int32_t* lift_rows = nullptr;   // free rows next to an inlet-table node
  int nlift = 0;
  int lift_lo[3] = {1, 1, 1}, lift_hi[3] = {0, 0, 0};  // refined: lattice box of the rows that see g
  double* inlet_shape = nullptr;

  // reductions
  double* partials = nullptr;
  double* res2 = nullptr;      // refinement residual: r.r, b.b
  double* nrmse = nullptr;     // step-to-step NRMSE of the three components
  double* host_res2 = nullptr; // pinned
  double* host_nrmse = nullptr; // pinned, 3 values
  KScal* scal = nullptr;
  KScal* host_scal = nullptr;  // pinned

  std::vector<MGDev<double>> mg64;
  std::vector<MGDev<float>> mg32;

  // 2:1 refined lattice (empty on uniform grids)
  uint8_t* cmask = nullptr;
  int32_t* pslot = nullptr;
  int nh = 0;
  int32_t* hang_ids = nullptr;
  int32_t* hang_par = nullptr;
  int32_t* par_ptr = nullptr;
  int32_t* par_child = nullptr;
  double* pw64 = nullptr;
  float* pw32 = nullptr;
  double *dinvM64 = nullptr, *dinvK64 = nullptr, *dinvA64 = nullptr;
  float *dinvM32 = nullptr, *dinvK32 = nullptr, *dinvA32 = nullptr;  // A: (rho/dt) M + mu K
  double* yh64 = nullptr;
  float* yh32 = nullptr;
  FormCoefs fcc{};   // forms of the coarse elements (spacing 2h)
  int32_t* xnodes = nullptr;  // nodes of P with kFlagExtra (coarse cells or hanging children)
  int nxn = 0;
  double* extra64 = nullptr;  // their extra row terms, 3 planes
  double* lmass64 = nullptr;  // row sums of the constrained mass
  float* extra32 = nullptr;
  // mass correction with the tensor-product preconditioner: D^-1/2 times the
  // residual on the lattice (3 planes; 0 off the walked rows) and, on a refined
  // lattice, its kFlagExtra rows (3 planes; 0 elsewhere)
  double *tmw64 = nullptr, *tmwx64 = nullptr;
  float *tmw32 = nullptr, *tmwx32 = nullptr;
  // BiCGStab's r, rhat, p, v, s, t in node-list order (6 vectors of 3 x 64 nchunks)
  double* bc64 = nullptr;
  float* bc32 = nullptr;

  FormCoefs fc{};
  // lower end of the Chebyshev interval of the mass correction on a refined
  // lattice (the proven bound, or the Lanczos estimate when it is larger)
  double mass_lmin = 0.125;
  double t = 0.0;
  int64_t steps = 0;
  ibfe_stats stats{};
  bool timing = false;
  KTimer kt;
  // executable graphs of fixed kernel sequences (iteration batches, Chebyshev
  // sequences), captured on first use; only on a non-null stream
  bool graphs = true;
  std::map<uint64_t, hipGraphExec_t> graph_cache;
  int est[kNumScal] = {};

  ~ibfe_ctx() {
    if (ev_ready) (void)hipEventDestroy(ev_ready);
    if (ev_done) (void)hipEventDestroy(ev_done);
    for (auto& kv : graph_cache) (void)hipGraphExecDestroy(kv.second);
    for (void* b : blocks) {
      if (user_alloc)
        alloc.free(b, alloc.user);
      else
        (void)hipFree(b);
    }
    if (host_scal) (void)hipHostFree(host_scal);
    if (host_res2) (void)hipHostFree(host_res2);
    if (host_nrmse) (void)hipHostFree(host_nrmse);
  }

  int dalloc(void** out, size_t bytes) {
    bytes = (bytes + 255) & ~size_t(255);
    void* ptr = nullptr;
    if (user_alloc) {
      ptr = alloc.alloc(bytes, (void*)stream, alloc.user);
      if (!ptr) return fail(IBFE_ENOMEM, "device allocator returned NULL");
    } else {
      hipError_t e = hipMalloc(&ptr, bytes);
      if (e != hipSuccess) return fail(IBFE_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    }
    blocks.push_back(ptr);
    HIP_TRY(hipMemsetAsync(ptr, 0, bytes, stream));
    *out = ptr;
    return IBFE_OK;
  }
  template <typename T>
  int field(T** out, int planes) {  // zeroed, padded, returns node-0 pointer
    void* base = nullptr;
    int rc = dalloc(&base, sizeof(T) * size_t(stride) * planes);
    if (rc) return rc;
    *out = reinterpret_cast<T*>(base) + halo;
    return IBFE_OK;
  }
  template <typename T>
  int upload(T** out, const T* src, size_t count, size_t min_count = 1) {
    void* base = nullptr;
    int rc = dalloc(&base, sizeof(T) * std::max(count, min_count));
    if (rc) return rc;
    if (count) {
      // src may be a temporary: wait until the copy has consumed it
      HIP_TRY(hipMemcpyAsync(base, src, sizeof(T) * count, hipMemcpyHostToDevice, stream));
      HIP_TRY(hipStreamSynchronize(stream));
    }
    *out = reinterpret_cast<T*>(base);
    return IBFE_OK;
  }
};

namespace {

// Readable name of a kernel instantiation from its symbol ("k_zb_cheb<float,
// false, 3>"): demangled, without the return type, the parameter list and the
// namespace.
std::string kernel_label(const char* mangled) {
  if (!mangled) return "kernel";
  int status = 0;
  char* dem = abi::__cxa_demangle(mangled, nullptr, nullptr, &status);
  std::string n = (status == 0 && dem) ? std::string(dem) : std::string(mangled);
  std::free(dem);
  if (n.rfind("void ", 0) == 0) n.erase(0, 5);
  int depth = 0;
  for (size_t i = 0; i < n.size(); ++i) {
    if (n[i] == '<') ++depth;
    else if (n[i] == '>') --depth;
    else if (n[i] == '(' && depth == 0 && n.compare(i, 11, "(anonymous ") != 0) {
      n.resize(i);
      break;
    }
  }
  for (size_t q; (q = n.find("(anonymous namespace)::")) != std::string::npos;) n.erase(q, 23);
  for (size_t q; (q = n.find("ibfe::")) != std::string::npos;) n.erase(q, 6);
  return n;
}

template <auto K>
const char* kname(hipStream_t stream) {
  static const std::string name = kernel_label(hipKernelNameRefByPtr((const void*)K, stream));
  return name.c_str();
}

// Every kernel of the library is dispatched through here: with the kernel timer
// on, the dispatch records its own start and end events.
template <auto K, typename... Args>
inline void klaunch(ibfe_ctx& c, dim3 grid, dim3 block, uint32_t shmem, hipStream_t stream, Args... args) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c.timing && (c.kt.only.empty() || c.kt.only == kname<K>(stream)) && c.kt.next(kname<K>(stream), e0, e1))
    hipExtLaunchKernelGGL(K, grid, block, shmem, stream, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(K, grid, block, shmem, stream, args...);
}

// Resolve the recorded event pairs (synchronises the stream) and add them to the
// per-kernel sums; the mass Chebyshev step and the pressure stiffness apply also
// feed the two summary fields of ibfe_stats.
int collect_kernel_times(ibfe_ctx& c) {
  KTimer& kt = c.kt;
  if (kt.used == 0) return IBFE_OK;
  HIP_TRY(hipEventSynchronize(kt.ev[2 * kt.used - 1]));
  for (size_t i = 0; i < kt.used; ++i) {
    if (kt.skip[i]) continue;
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, kt.ev[2 * i], kt.ev[2 * i + 1]));
    const std::string name(kt.tag[i]);
    KTimer::Acc& a = kt.acc[name];
    a.ms += ms;
    a.launches += 1;
    // the mass Chebyshev step (three components, lattice or walk-order vectors):
    // the Jacobi step, or the update pass of the tensor-preconditioned one
    auto ends = [&](const std::string& tail) {
      return name.size() > tail.size() && name.compare(name.size() - tail.size(), tail.size(), tail) == 0;
    };
    const bool mass = (name.rfind("k_zb_cheb<", 0) == 0 &&
                       (ends(", false, 3>") || ends(", false, 3, true>") || ends(", false, 3, false>"))) ||
                      name.rfind("k_tm_cheb<", 0) == 0;
    const bool pressure = name == "k_cg_q_zb<float, 1>" || name == "k_cg_q_zb<double, 1>";
    if (mass) {
      c.stats.mass_apply_ms += ms;
      c.stats.mass_applies += 1;
    } else if (pressure) {
      c.stats.poisson_apply_ms += ms;
      c.stats.poisson_applies += 1;
    }
  }
  kt.used = 0;
  kt.marks.clear();
  return IBFE_OK;
}

// -------------------------------------------------------------------------
// set-up
// -------------------------------------------------------------------------

// Multigrid levels on the device.  Level 0 shares the grid's node bits, chunk
// and column lists; its work vectors are taken from the Krylov work space.
template <typename T>
int setup_mg(ibfe_ctx& c, std::vector<MGDev<T>>& out, T* xt0, T* d0, T* r0) {
  const Plan& P = c.plan;
  out.clear();
  int rc;
  for (size_t l = 0; l < P.mg.size(); ++l) {
    const MGLevel& L = P.mg[l];
    MGDev<T> D;
    D.nx = L.nx;
    D.ny = L.ny;
    D.nz = L.nz;
    D.N = L.N;
    D.sy = L.sy;
    D.sz = L.sz;
    D.zb = L.zb;
    const FormCoefs f = form_coefs(L.h);
    for (int t = 0; t < 4; ++t) D.kc[t] = f.k[t];
    if (l == 0) {
      D.halo = c.halo;
      D.stride = c.stride;
      D.emask = c.emask;
      D.flags = c.flags;
      D.nl = c.nl;
      D.nchunks = c.nchunks;
      D.zitems = c.zitems;
      D.zlanes = c.zlanes;
      D.nzitems = c.nzitems;
      D.zb = c.zb;
      D.xt = xt0;
      D.d = d0;
      D.r = r0;
      D.composite = P.refined;
    } else {
      const int64_t nch = (L.N + kChunk - 1) / kChunk;
      D.halo = ((L.sz + L.sy + 1 + kChunk - 1) / kChunk) * kChunk;
      D.stride = 2 * D.halo + nch * kChunk;
      auto plane = [&](size_t bytes_per, void** base) { return c.dalloc(base, bytes_per * size_t(D.stride)); };
      void* base = nullptr;
      if ((rc = plane(1, &base))) return rc;
      D.emask = reinterpret_cast<uint8_t*>(base) + D.halo;
      HIP_TRY(hipMemcpyAsync(D.emask, L.emask.data(), L.N, hipMemcpyHostToDevice, c.stream));
      if ((rc = plane(1, &base))) return rc;
      D.flags = reinterpret_cast<uint8_t*>(base) + D.halo;
      HIP_TRY(hipMemcpyAsync(D.flags, L.flags.data(), L.N, hipMemcpyHostToDevice, c.stream));
      int* lc = nullptr;
      if ((rc = c.upload(&lc, L.chunks.data(), L.chunks.size()))) return rc;
      D.nchunks = int(L.chunks.size());
      D.nl = NodeList{lc, D.nchunks, 0};
      if ((rc = c.upload(&D.zitems, L.zitems.data(), L.zitems.size()))) return rc;
      if ((rc = c.upload(&D.zlanes, L.zlanes.data(), L.zlanes.size()))) return rc;
      D.nzitems = int(L.zitems.size());
      T** vecs[5] = {&D.b, &D.x, &D.xt, &D.d, &D.r};
      for (T** v : vecs) {
        if ((rc = plane(sizeof(T), &base))) return rc;
        *v = reinterpret_cast<T*>(base) + D.halo;
      }
    }
    if (l + 1 == P.mg.size() && !L.inv.empty()) {
      D.m = int(L.unknowns.size());
      if ((rc = c.upload(&D.ids, L.unknowns.data(), L.unknowns.size()))) return rc;
      std::vector<T> inv(L.inv.begin(), L.inv.end());
      if ((rc = c.upload(&D.inv, inv.data(), inv.size()))) return rc;
    }
    out.push_back(D);
  }
  return IBFE_OK;
}

// Device tables of a refined lattice: coarse cell bits, parent slots, the
// hanging and parent lists, inverse lumped diagonals and the hanging-row buffers.
int setup_refined(ibfe_ctx& c) {
  const Plan& P = c.plan;
  int rc;
  c.fcc = form_coefs(P.hb);
  if ((rc = c.field(&c.cmask, 1))) return rc;
  HIP_TRY(hipMemcpyAsync(c.cmask, P.cmask.data(), P.N, hipMemcpyHostToDevice, c.stream));
  if ((rc = c.field(&c.pslot, 1))) return rc;
  HIP_TRY(hipMemcpyAsync(c.pslot, P.par_slot.data(), sizeof(int32_t) * P.N, hipMemcpyHostToDevice, c.stream));
  c.nh = int(P.hang_ids.size());
  {
    std::vector<int32_t> xn;
    for (int64_t n = 0; n < P.N; ++n)
      if ((P.flags[n] & IBFE_FLAG_P) && (P.cmask[n] != 0 || P.par_slot[n] >= 0)) xn.push_back(int32_t(n));
    c.nxn = int(xn.size());
    if ((rc = c.upload(&c.xnodes, xn.data(), xn.size()))) return rc;
    if ((rc = c.field(&c.extra64, 3))) return rc;
    if ((rc = c.field(&c.lmass64, 1))) return rc;
    HIP_TRY(hipMemcpyAsync(c.lmass64, P.lmass.data(), sizeof(double) * P.N, hipMemcpyHostToDevice, c.stream));
    if (P.params.precision == 1 && (rc = c.field(&c.extra32, 3))) return rc;
  }
  if ((rc = c.upload(&c.hang_ids, P.hang_ids.data(), P.hang_ids.size()))) return rc;
  if ((rc = c.upload(&c.hang_par, P.hang_par.data(), P.hang_par.size()))) return rc;
  if ((rc = c.upload(&c.par_ptr, P.par_ptr.data(), P.par_ptr.size()))) return rc;
  if ((rc = c.upload(&c.par_child, P.par_child.data(), P.par_child.size()))) return rc;
  if ((rc = c.upload(&c.pw64, P.par_w.data(), P.par_w.size()))) return rc;
  {
    std::vector<float> w32(P.par_w.begin(), P.par_w.end());
    if ((rc = c.upload(&c.pw32, w32.data(), w32.size()))) return rc;
  }
  std::vector<double> im(P.N, 0.0), ik(P.N, 0.0);
  for (int64_t n = 0; n < P.N; ++n) {
    if (P.dmass[n] > 0.0) im[n] = 1.0 / P.dmass[n];
    if (P.dstiff[n] > 0.0) ik[n] = 1.0 / P.dstiff[n];
  }
  if (P.params.advection == 1) {
    // Jacobi scaling of the symmetric tentative-velocity operator (rho/dt) M + mu K
    const double rdt = P.params.rho / P.params.dt, mu = P.params.mu;
    std::vector<double> ia(P.N, 0.0);
    for (int64_t n = 0; n < P.N; ++n) {
      const double dA = rdt * P.dmass[n] + mu * P.dstiff[n];
      if (dA > 0.0) ia[n] = 1.0 / dA;
    }
    std::vector<float> ia32(ia.begin(), ia.end());
    if ((rc = c.field(&c.dinvA64, 1))) return rc;
    if ((rc = c.field(&c.dinvA32, 1))) return rc;
    HIP_TRY(hipMemcpyAsync(c.dinvA64, ia.data(), sizeof(double) * P.N, hipMemcpyHostToDevice, c.stream));
    HIP_TRY(hipMemcpyAsync(c.dinvA32, ia32.data(), sizeof(float) * P.N, hipMemcpyHostToDevice, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
  }
  if ((rc = c.field(&c.dinvM64, 1))) return rc;
  if ((rc = c.field(&c.dinvK64, 1))) return rc;
  if ((rc = c.field(&c.dinvM32, 1))) return rc;
  if ((rc = c.field(&c.dinvK32, 1))) return rc;
  HIP_TRY(hipMemcpyAsync(c.dinvM64, im.data(), sizeof(double) * P.N, hipMemcpyHostToDevice, c.stream));
  HIP_TRY(hipMemcpyAsync(c.dinvK64, ik.data(), sizeof(double) * P.N, hipMemcpyHostToDevice, c.stream));
  {
    std::vector<float> m32(im.begin(), im.end()), k32(ik.begin(), ik.end());
    HIP_TRY(hipMemcpyAsync(c.dinvM32, m32.data(), sizeof(float) * P.N, hipMemcpyHostToDevice, c.stream));
    HIP_TRY(hipMemcpyAsync(c.dinvK32, k32.data(), sizeof(float) * P.N, hipMemcpyHostToDevice, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));  // the host staging vectors go out of scope
  }
  void* base = nullptr;
  if ((rc = c.dalloc(&base, sizeof(double) * 3 * std::max(1, c.nh)))) return rc;
  c.yh64 = reinterpret_cast<double*>(base);
  if ((rc = c.dalloc(&base, sizeof(float) * 3 * std::max(1, c.nh)))) return rc;
  c.yh32 = reinterpret_cast<float*>(base);
  return IBFE_OK;
}

// The active nodes (P and hanging) as 64-node chunks, or one node per lane when
// they fill their chunks sparsely: a thin vessel in a large box leaves most
// lanes of its chunks idle, and the per-lane list runs the same kernels on
// 2-3x fewer wavefronts.  The padding node of a per-lane list is a lattice node
// outside every set, so kernels see it as a non-row.
int setup_node_list(ibfe_ctx& c) {
  const Plan& P = c.plan;
  int64_t active = 0;
  for (int64_t n = 0; n < P.N; ++n) active += (P.flags[n] & (IBFE_FLAG_P | IBFE_FLAG_HANG)) ? 1 : 0;
  const double fill = double(active) / (double(kChunk) * double(std::max<size_t>(1, P.chunks.size())));
  int64_t pad = -1;
  if (fill < kLaneFill)
    for (int64_t n = 0; n < P.N && pad < 0; ++n)
      if (P.flags[n] == 0 && P.emask[n] == 0 && (!P.refined || P.cmask[n] == 0) && P.float_slot[n] < 0) pad = n;
  int rc;
  int* ids = nullptr;
  if (pad < 0) {
    if ((rc = c.upload(&ids, P.chunks.data(), P.chunks.size()))) return rc;
    c.nl = NodeList{ids, int(P.chunks.size()), 0};
  } else {
    std::vector<int32_t> lanes;
    lanes.reserve(size_t(active + kChunk));
    for (int64_t n = 0; n < P.N; ++n)
      if (P.flags[n] & (IBFE_FLAG_P | IBFE_FLAG_HANG)) lanes.push_back(int32_t(n));
    while (lanes.size() % kChunk) lanes.push_back(int32_t(pad));
    if ((rc = c.upload(&ids, lanes.data(), lanes.size()))) return rc;
    c.nl = NodeList{ids, int(lanes.size() / kChunk), 1};
  }
  c.nchunks = c.nl.n;
  return IBFE_OK;
}

int setup_device(ibfe_ctx& c) {
  Plan& P = c.plan;
  const int64_t nch_total = (P.N + kChunk - 1) / kChunk;
  // the coarse elements of a refined lattice reach neighbours at offset 2
  const int64_t reach = (P.refined ? 2 : 1) * (P.sz + P.sy + 1);
  c.halo = ((reach + kChunk - 1) / kChunk) * kChunk;
  c.stride = 2 * c.halo + nch_total * kChunk;
  c.nP = int(P.P_ids.size());
  c.fc = form_coefs(P.h);
  int rc;
  // per-node geometry, padded like the fields
  std::vector<uint8_t> fl(P.N);
  for (int64_t n = 0; n < P.N; ++n) {
    uint8_t f = P.flags[n];
    if ((f & IBFE_FLAG_P) && !(f & IBFE_FLAG_PDIR)) f |= kFlagPp;
    if (P.refined && P.par_slot[n] >= 0) f |= kFlagPar;
    if (P.refined && (f & IBFE_FLAG_P) && (P.cmask[n] != 0 || P.par_slot[n] >= 0)) f |= kFlagExtra;
    fl[n] = f;
  }
  if ((rc = c.field(&c.emask, 1))) return rc;
  if ((rc = c.field(&c.flags, 1))) return rc;
  if ((rc = c.field(&c.slot, 1))) return rc;
  HIP_TRY(hipMemcpyAsync(c.emask, P.emask.data(), P.N, hipMemcpyHostToDevice, c.stream));
  HIP_TRY(hipMemcpyAsync(c.flags, fl.data(), P.N, hipMemcpyHostToDevice, c.stream));
  HIP_TRY(hipMemcpyAsync(c.slot, P.float_slot.data(), P.N, hipMemcpyHostToDevice, c.stream));
  // nodes past N in the last chunk carry slot 0 after the memset: mark them -1
  {
    int64_t tail = nch_total * kChunk - P.N;
    if (tail > 0) HIP_TRY(hipMemsetAsync(c.slot + P.N, 0xFF, tail, c.stream));
  }
  if ((rc = setup_node_list(c))) return rc;
  {
    // column items of the z-blocked applies: zb planes x 64 in-plane positions
    // (on a refined lattice also the all-even nodes with unrefined cells only)
    std::vector<int> items, lanes;
    if (P.refined) {
      std::vector<uint8_t> act(P.N);
      for (int64_t n = 0; n < P.N; ++n) act[n] = P.emask[n] | P.cmask[n];
      c.zb = choose_column_items(act, P.sz, P.nz + 1, items, lanes);
    } else {
      c.zb = choose_column_items(P.emask, P.sz, P.nz + 1, items, lanes);
    }
    c.nzitems = int(items.size());
    if ((rc = c.upload(&c.zitems, items.data(), items.size()))) return rc;
    if ((rc = c.upload(&c.zlanes, lanes.data(), lanes.size()))) return rc;
    // walk order: (item, plane, lane) -> cell bits and flags of that lattice position
    c.imstride = int64_t(c.nzitems) * c.zb * 64;
    std::vector<uint8_t> emi(size_t(std::max<int64_t>(1, c.imstride)), 0), fli(emi.size(), 0);
    for (int it = 0; it < c.nzitems; ++it) {
      const int k0 = items[it] * c.zb;
      const int kend = std::min<int>(c.zb, int(P.nz + 1) - k0);
      for (int lane = 0; lane < 64; ++lane) {
        const int inplane = lanes[size_t(it) * 64 + lane];
        if (inplane < 0) continue;
        for (int k = 0; k < kend; ++k) {
          const int64_t node = int64_t(k0 + k) * P.sz + inplane;
          const size_t im = (size_t(it) * c.zb + k) * 64 + lane;
          emi[im] = P.emask[node];
          fli[im] = fl[node];
        }
      }
    }
    if ((rc = c.upload(&c.em_im, emi.data(), emi.size()))) return rc;
    if ((rc = c.upload(&c.fl_im, fli.data(), fli.size()))) return rc;
  }
  if ((rc = c.upload(&c.pids, P.P_ids.data(), P.P_ids.size()))) return rc;
  {
    std::vector<double> cnt(kMaxFloating, 1.0);
    for (int s = 0; s < P.n_floating; ++s) cnt[s] = double(P.float_count[s]);
    if ((rc = c.upload(&c.float_count, cnt.data(), cnt.size()))) return rc;
    std::vector<double> zero(kMaxFloating, 0.0);
    if ((rc = c.upload(&c.float_means, zero.data(), zero.size()))) return rc;
  }
  // fields
  if ((rc = c.field(&c.u, 3))) return rc;
  if ((rc = c.field(&c.u_next, 3))) return rc;
  if ((rc = c.field(&c.p, 1))) return rc;
  if ((rc = c.field(&c.p_next, 1))) return rc;
  if ((rc = c.field(&c.g, 3))) return rc;
  if ((rc = c.field(&c.ustar, 3))) return rc;
  if ((rc = c.field(&c.uib, 3))) return rc;
  if ((rc = c.field(&c.phi, 1))) return rc;
  if ((rc = c.field(&c.delta, 3))) return rc;
  const int ncoef = P.refined ? 54 : 27;
  const bool stencil = P.params.advdiff == 1 || P.params.advection == 1;
  if (stencil && (rc = c.field(&c.coef64, ncoef))) return rc;
  if (!stencil && ((rc = c.field(&c.dinvS64, 1)) || (rc = c.field(&c.w64, 3)))) return rc;
  for (int i = 0; i < 10; ++i)
    if ((rc = c.field(&c.w[i], 3))) return rc;
  if (P.params.mass_precond == 1) {
    // the tensor-preconditioned mass correction: FP32 with the mixed scheme
    if (P.params.precision == 1) {
      if ((rc = c.field(&c.tmw32, 3))) return rc;
      if (P.refined && (rc = c.field(&c.tmwx32, 3))) return rc;
    } else {
      if ((rc = c.field(&c.tmw64, 3))) return rc;
      if (P.refined && (rc = c.field(&c.tmwx64, 3))) return rc;
    }
  }
  if (P.params.advection == 0 && c.nl.per_lane) {
    // the tentative-velocity BiCGStab (FP32 inner solves with the mixed scheme)
    const size_t nbc = size_t(6) * 3 * size_t(c.nchunks) * 64;
    void* base = nullptr;
    if (P.params.precision == 1) {
      if ((rc = c.dalloc(&base, sizeof(float) * nbc))) return rc;
      c.bc32 = reinterpret_cast<float*>(base);
    } else {
      if ((rc = c.dalloc(&base, sizeof(double) * nbc))) return rc;
      c.bc64 = reinterpret_cast<double*>(base);
    }
  }
  if (P.refined && (rc = setup_refined(c))) return rc;
  if (P.params.precision == 1) {
    if (stencil && (rc = c.field(&c.coef32, ncoef))) return rc;
    if (!stencil && ((rc = c.field(&c.dinvS32, 1)) || (rc = c.field(&c.w32, 3)))) return rc;
    for (int i = 0; i < 10; ++i)
      if ((rc = c.field(&c.v32[i], 3))) return rc;
    void* base = nullptr;
    if ((rc = c.dalloc(&base, sizeof(float) * 3 * std::max<int64_t>(1, c.imstride)))) return rc;
    c.rim = reinterpret_cast<float*>(base);
    if ((rc = c.dalloc(&base, sizeof(float) * 3 * std::max<int64_t>(1, c.imstride)))) return rc;
    c.dim = reinterpret_cast<float*>(base);
  }
  {
    void* base = nullptr;
    if ((rc = c.dalloc(&base, sizeof(double) * 3 * std::max<int64_t>(1, P.P_ids.size() + P.M))))
      return rc;
    c.compact = reinterpret_cast<double*>(base);
  }
  // immersed boundary
  const int64_t M = P.M;
  c.ib_nchunks = int((M + kChunk - 1) / kChunk);
  c.mstride = std::max<int64_t>(kChunk, int64_t(c.ib_nchunks) * kChunk);
  if (M > 0) {
    std::vector<int> ibc(c.ib_nchunks);
    for (int i = 0; i < c.ib_nchunks; ++i) ibc[i] = i;
    int* ic = nullptr;
    if ((rc = c.upload(&ic, ibc.data(), ibc.size()))) return rc;
    c.ib_nl = NodeList{ic, c.ib_nchunks, 0};
    if ((rc = c.upload(&c.ib_idx, P.ib_idx.data(), P.ib_idx.size()))) return rc;
    if ((rc = c.upload(&c.ib_w, P.ib_w.data(), P.ib_w.size()))) return rc;
    if ((rc = c.upload(&c.UB, P.U_B.data(), P.U_B.size()))) return rc;
    // the points may move (ibfe_set_points): the spreading lists and G are held at
    // their largest sizes from the start (every support pair free; four times the
    // entries of G at the initial positions, at least 128 per row), so that a
    // rebuild writes them in place
    const int64_t np = 64 * M;
    c.mv.g_cap = std::max<int64_t>(4 * int64_t(P.G_col.size()), 128 * M);
    if (P.refined) {
      std::vector<uint8_t> band;
      ib_band_mask(P, band);
      if ((rc = c.upload(&c.ib_band, band.data(), band.size()))) return rc;
    }
    const size_t gc = size_t(c.mv.g_cap);
    if ((rc = c.upload(&c.G_ptr, P.G_ptr.data(), P.G_ptr.size()))) return rc;
    if ((rc = c.upload(&c.G_col, P.G_col.data(), P.G_col.size(), gc))) return rc;
    if ((rc = c.upload(&c.G_val, P.G_val.data(), P.G_val.size(), gc))) return rc;
    if ((rc = c.upload(&c.G_diag, P.G_diag.data(), P.G_diag.size()))) return rc;
    if ((rc = c.upload(&c.G_binv, P.G_binv.data(), P.G_binv.size()))) return rc;
    if ((rc = c.upload(&c.sp_node, P.sp_node.data(), P.sp_node.size(), size_t(np)))) return rc;
    if ((rc = c.upload(&c.sp_ptr, P.sp_ptr.data(), P.sp_ptr.size(), size_t(np + 1)))) return rc;
    if ((rc = c.upload(&c.sp_pt, P.sp_pt.data(), P.sp_pt.size(), size_t(np)))) return rc;
    if ((rc = c.upload(&c.sp_wt, P.sp_w.data(), P.sp_w.size(), size_t(np)))) return rc;
    c.n_sp = int(P.sp_node.size());
    for (int i = 0; i < 7; ++i) {
      void* base = nullptr;
      if ((rc = c.dalloc(&base, sizeof(double) * 3 * c.mstride))) return rc;
      c.ibv[i] = reinterpret_cast<double*>(base);
    }
  }
  if (!P.inlet_ids.empty()) {
    if ((rc = c.upload(&c.inlet_ids, P.inlet_ids.data(), P.inlet_ids.size()))) return rc;
    if (P.refined) {
      // the inlet-table nodes' bounding box widened by 4 lattice steps
      const int64_t ext[3] = {P.sy - 1, P.sz / P.sy - 1, P.N / P.sz - 1};
      int64_t lo[3] = {ext[0], ext[1], ext[2]}, hi[3] = {0, 0, 0};
      for (int64_t id : P.inlet_ids) {
        const int64_t q[3] = {id % P.sy, (id % P.sz) / P.sy, id / P.sz};
        for (int a = 0; a < 3; ++a) {
          lo[a] = std::min(lo[a], q[a]);
          hi[a] = std::max(hi[a], q[a]);
        }
      }
      for (int a = 0; a < 3; ++a) {
        c.lift_lo[a] = int(std::max<int64_t>(0, lo[a] - 4));
        c.lift_hi[a] = int(std::min<int64_t>(ext[a], hi[a] + 4));
      }
    }
    if (!P.refined) {
      // the rows that see g: free nodes with an inlet-table node among their 27 neighbours
      std::vector<int32_t> rows;
      for (int64_t id : P.inlet_ids) {
        const int64_t k = id / P.sz, j = (id % P.sz) / P.sy, i = id % P.sy;
        for (int oz = -1; oz <= 1; ++oz)
          for (int oy = -1; oy <= 1; ++oy)
            for (int ox = -1; ox <= 1; ++ox) {
              const int64_t ii = i + ox, jj = j + oy, kk = k + oz;
              if (ii < 0 || jj < 0 || kk < 0 || ii > P.nx || jj > P.ny || kk > P.nz) continue;
              const int64_t m = ii + P.sy * jj + P.sz * kk;
              if (P.flags[m] & IBFE_FLAG_F) rows.push_back(int32_t(m));
            }
      }
      std::sort(rows.begin(), rows.end());
      rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
      c.nlift = int(rows.size());
      if ((rc = c.upload(&c.lift_rows, rows.data(), rows.size()))) return rc;
    }
    if ((rc = c.upload(&c.inlet_shape, P.inlet_shape.data(), P.inlet_shape.size()))) return rc;
  }
  if (P.params.precond >= 1) {
    if (P.params.precision == 1)
      rc = setup_mg<float>(c, c.mg32, c.v32[4], c.v32[5], c.v32[6]);
    else
      rc = setup_mg<double>(c, c.mg64, c.w[4], c.w[5], c.w[6]);
    if (rc) return rc;
  }
  // reductions
  {
    void* base = nullptr;
    if ((rc = c.dalloc(&base, sizeof(double) * kMaxRows * size_t(kRedBlocks)))) return rc;
    c.partials = reinterpret_cast<double*>(base);
    if ((rc = c.dalloc(&base, 256))) return rc;
    c.res2 = reinterpret_cast<double*>(base);
    if ((rc = c.dalloc(&base, 256))) return rc;
    c.nrmse = reinterpret_cast<double*>(base);
    if ((rc = c.dalloc(&base, sizeof(KScal) * kNumScal))) return rc;
    c.scal = reinterpret_cast<KScal*>(base);
  }
  HIP_TRY(hipHostMalloc((void**)&c.host_scal, sizeof(KScal) * kNumScal, hipHostMallocDefault));
  std::memset(c.host_scal, 0, sizeof(KScal) * kNumScal);
  HIP_TRY(hipHostMalloc((void**)&c.host_res2, 2 * sizeof(double), hipHostMallocDefault));
  HIP_TRY(hipHostMalloc((void**)&c.host_nrmse, 3 * sizeof(double), hipHostMallocDefault));
  HIP_TRY(hipStreamSynchronize(c.stream));
  return IBFE_OK;
}

// -------------------------------------------------------------------------
// Krylov drivers.  The kernels keep every scalar on the device; the host only
// polls the `done` flag between batches of iterations.
// -------------------------------------------------------------------------

int poll(ibfe_ctx& c, int slot, KScal& out) {
  HIP_TRY(hipMemcpyAsync(&c.host_scal[slot], &c.scal[slot], sizeof(KScal), hipMemcpyDeviceToHost,
                         c.stream));
  HIP_TRY(hipStreamSynchronize(c.stream));
  out = c.host_scal[slot];
  return IBFE_OK;
}

int finish_status(const KScal& s, const char* what) {
  if (s.status == 2) return fail(IBFE_ENONFINITE, std::string(what) + ": non-finite residual");
  if (s.status == 1) return fail(IBFE_ESINGULAR, std::string(what) + ": Krylov breakdown");
  if (!s.done || (s.iters >= s.max_iters && s.rr > s.tol2 * s.bb))
    return fail(IBFE_ENOCONV, std::string(what) + ": iteration cap reached");
  return IBFE_OK;
}

struct SolveOut {
  int iters = 0;
  double res = 0.0;
  int outer = 1;     // refinement sweeps (mixed precision)
  int restarts = 0;  // BiCGStab restarts after a breakdown
};

// Iterations per replayed batch between convergence polls: a little under the
// last solve's count first, then 2 at a time (iterations launched past
// convergence return at once but still cost a dispatch each; batches of 8 after
// the first cost about 1 % of the step against batches of 2)
// The first batch is capped: a solve that ran into its iteration cap leaves an
// estimate of up to max_iters, and one graph of that many iterations (hundreds
// of thousands of kernel nodes) is more than capture and instantiation handle.
constexpr int kMaxGraphIters = 256;
int next_batch(int est, int done_so_far) {
  if (done_so_far == 0) return std::min(kMaxGraphIters, std::max(4, est - 2));
  return 2;
}

// The walk-order cell bits and flags serve every walk over the context's own
// column items with the context's own bits and flags.
template <typename T>
ZOp<T> with_im(const ibfe_ctx& c, ZOp<T> z) {
  if (z.lanes == c.zlanes && z.emask == c.emask && z.flags == c.flags) {
    z.em_im = c.em_im;
    z.fl_im = c.fl_im;
  }
  return z;
}

// q = A p with partial p.q; returns the number of partials written.
template <typename T, class Op>
int launch_q(ibfe_ctx& c, const Op& op, NodeList nl, const T* p, T* q, const KScal* sc) {
  const int nr = red_blocks(nl.n);
  klaunch<(k_cg_q<T, Op>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, p, q, c.partials, sc);
  return nr;
}
template <typename T, int NC>
int launch_q(ibfe_ctx& c, const OpSym<T, NC>& op, NodeList, const T* p, T* q, const KScal* sc) {
  const int nr = red_blocks(c.nzitems);
  ZOp<T> z{op.emask, op.flags, op.rowbit, op.sy, op.sz, c.plan.nz + 1,
           {op.c[0], op.c[1], op.c[2], op.c[3]}, c.zb, c.zlanes};
  z = with_im(c, z);
  klaunch<(k_cg_q_zb<T, NC>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems, c.nzitems, z,
                              op.stride, p, q, c.partials, sc);
  return nr;
}

// Operators of a refined lattice need C x at the hanging nodes and the
// element rows there before every apply (see composite.hpp); uniform
// operators need nothing.
template <typename T, class Op>
int pre_apply(ibfe_ctx&, const Op&, T*, const KScal*) {
  return IBFE_OK;
}

template <typename T, class Op>
int hang_prepare(ibfe_ctx& c, const Op& op, T* x, const KScal* sc) {
  if (c.nh == 0) return IBFE_OK;
  const int nb = blocks_lin(c.nh);
  klaunch<k_hang_fill<T>>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nh, (const int32_t*)c.hang_ids,
                     (const int32_t*)c.hang_par, x, int(Op::kNC), c.stride, sc);
  OpElem<T, Op> f{op, x};
  klaunch<(k_hang_elem<T, OpElem<T, Op>>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nh,
                     (const int32_t*)c.hang_ids, f, const_cast<T*>(op.yh), sc);
  CHECK_LAUNCH();
  return IBFE_OK;
}
template <typename T, class B>
int pre_apply(ibfe_ctx& c, const OpCStencilStrain<T, B>& op, T* x, const KScal* sc) {
  return hang_prepare<T>(c, op, x, sc);
}
template <typename T>
int pre_apply(ibfe_ctx& c, const OpCConv<T>& op, T* x, const KScal* sc) {
  int rc = hang_prepare<T>(c, op, x, sc);
  if (rc || !op.extra || c.nxn == 0) return rc;
  klaunch<k_conv_extra<T>>(c, dim3(blocks_lin(c.nxn)), dim3(kBlock), 0, c.stream, c.nxn,
                           (const int32_t*)c.xnodes, op, (const T*)x, const_cast<T*>(op.extra), sc);
  CHECK_LAUNCH();
  return IBFE_OK;
}
template <typename T>
int pre_apply(ibfe_ctx& c, const OpCSymStrain<T>& op, T* x, const KScal* sc) {
  return hang_prepare<T>(c, op, x, sc);
}
template <typename T, int NC>
int pre_apply(ibfe_ctx& c, const OpCSym<T, NC>& op, T* x, const KScal* sc) {
  return hang_prepare<T>(c, op, x, sc);
}
template <typename T, int NC>
int pre_apply(ibfe_ctx& c, const OpCStencil<T, NC>& op, T* x, const KScal* sc) {
  return hang_prepare<T>(c, op, x, sc);
}

// Graph keys: call site, Krylov slot, scalar size, sequence length.
enum GraphSite : uint64_t { kGsCg = 1, kGsBicg, kGsPcgMg, kGsChebMass, kGsChebGen, kGsIbPcg, kGsChebTm };
uint64_t graph_key(GraphSite site, int slot, int tbytes, int len) {
  return (uint64_t(site) << 56) | (uint64_t(slot & 0xff) << 48) | (uint64_t(tbytes & 0xff) << 40) |
         uint64_t(uint32_t(len));
}

// Issue the kernels of body() on the context's stream, through an executable
// graph captured on the first call with this key (the sequence and every kernel
// argument are fixed per key: buffers and scalar slots belong to the context,
// convergence is read by the kernels from the device scalar block).  Eager when
// graphs are off, kernel timing is on or the stream is the null stream.
template <class Body>
int graph_run(ibfe_ctx& c, uint64_t key, Body&& body) {
  if (!c.graphs || c.timing || c.stream == nullptr) return body();
  auto it = c.graph_cache.find(key);
  if (it == c.graph_cache.end()) {
    HIP_TRY(hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal));
    const int rc = body();
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c.stream, &g);
    if (rc || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return rc ? rc : fail(IBFE_EHIP, std::string("stream capture failed: ") + hipGetErrorString(e));
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(IBFE_EHIP, std::string("graph instantiation: ") + hipGetErrorString(ei));
    it = c.graph_cache.emplace(key, ex).first;
  }
  HIP_TRY(hipGraphLaunch(it->second, c.stream));
  return IBFE_OK;
}

// composite pressure operator: z-blocked walk (defined with the refined-lattice helpers)
template <typename T>
int launch_q(ibfe_ctx& c, const OpCSym<T, 1>& op, NodeList, const T* p, T* q, const KScal* sc);

template <typename T, class Op>
int run_cg(ibfe_ctx& c, const Op& op, NodeList nl, const T* b, T* x, T* r, T* p,
           T* q, int slot, double rtol, int max_iters, bool zero_guess, SolveOut& out) {
  const int nb = blocks_for(nl.n), nr = red_blocks(nl.n);
  KScal* sc = &c.scal[slot];
  int prc;
  if (!zero_guess && (prc = pre_apply(c, op, x, (const KScal*)nullptr))) return prc;
  klaunch<(k_cg_init<T, Op>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, b, x,
                     r, p, c.partials, zero_guess ? 1 : 0);
  klaunch<k_fin_cg_init>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr, sc,
                     rtol * rtol, max_iters);
  CHECK_LAUNCH();
  int launched = 0;
  KScal s{};
  c.kt.begin_solve();
  while (true) {
    const int batch = std::min(next_batch(c.est[slot], launched), max_iters + 1 - launched);
    auto body = [&]() -> int {
      for (int k = 0; k < batch; ++k) {
        if (c.timing) c.kt.mark();
        int rc2;
        if ((rc2 = pre_apply(c, op, p, (const KScal*)sc))) return rc2;
        const int nq = launch_q<T>(c, op, nl, p, q, (const KScal*)sc);
        klaunch<k_fin_cg_q>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nq, sc);
        klaunch<(k_cg_xr<T, Op>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, x, r,
                           p, q, c.partials, (const KScal*)sc);
        klaunch<k_fin_cg_xr>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr,
                           sc);
        klaunch<(k_cg_p<T, Op>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, nl, op, r, p,
                           (const KScal*)sc);
        CHECK_LAUNCH();
      }
      return IBFE_OK;
    };
    if ((prc = graph_run(c, graph_key(kGsCg, slot, sizeof(T), batch), body))) return prc;
    launched += batch;
    int rc = poll(c, slot, s);
    if (rc) return rc;
    if (s.done || launched > max_iters) break;
  }
  // dispatches past convergence returned at once
  if (c.timing) c.kt.drop_from(s.iters);
  c.est[slot] = std::max(1, s.iters);
  out.iters = s.iters;
  out.res = s.bb > 0.0 ? std::sqrt(s.rr / s.bb) : 0.0;
  return finish_status(s, "CG");
}

// y = A xin with the BiCGStab products of step MODE; returns the number of partials.
template <typename T, int MODE, class Op>
int launch_bi_apply(ibfe_ctx& c, const Op& op, NodeList nl, const T* xin, T* y, const T* w, const KScal* sc) {
  const int nr = red_blocks(nl.n);
  klaunch<(k_bi_apply<T, Op, MODE>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, xin, y, w, c.partials, sc);
  return nr;
}

template <typename T>
T* bicg_bufs(const ibfe_ctx& c);
template <>
double* bicg_bufs<double>(const ibfe_ctx& c) { return c.bc64; }
template <>
float* bicg_bufs<float>(const ibfe_ctx& c) { return c.bc32; }

// wv: 8 lattice vectors (r, rhat, p, v, phat, s, shat, t); with a per-lane node
// list only phat and shat are used, the others come from the node-list buffers
template <typename T, class Op>
int run_bicgstab(ibfe_ctx& c, const Op& op, const T* b, T* x, T* const* wv, int slot, double rtol,
                 int max_iters, SolveOut& out, bool zero_guess = false) {
  const int nb = blocks_for(c.nchunks), nr = red_blocks(c.nchunks);
  const NodeList nl = c.nl;
  const double* pa = c.partials;
  // with a per-lane node list, r, rhat, p, v, s, t in node-list order
  T* bc = bicg_bufs<T>(c);
  if (nl.per_lane && bc == nullptr) return fail(IBFE_EINVAL, "internal: BiCGStab buffers not allocated");
  const int64_t cv = int64_t(3) * c.nchunks * 64;
  T *r = wv[0], *rhat = wv[1], *p = wv[2], *v = wv[3], *phat = wv[4], *s = wv[5], *shat = wv[6],
    *t = wv[7];
  if (nl.per_lane) {
    r = bc;
    rhat = bc + cv;
    p = bc + 2 * cv;
    v = bc + 3 * cv;
    s = bc + 4 * cv;
    t = bc + 5 * cv;
  }
  KScal* sc = &c.scal[slot];
  const KScal* csc = sc;
  int prc;
  // a breakdown (rhat.v = 0 or t.t = 0 before convergence) restarts the method from
  // the current iterate with a fresh shadow residual, at most three times
  int total = 0, restarts = 0;
  KScal st{};
  for (int restart = 0;; ++restart) {
    restarts = restart;
    // x = 0 at the first start of an inner correction solve: r = b, no apply
    const int zg = (zero_guess && restart == 0) ? 1 : 0;
    if (!zg && (prc = pre_apply(c, op, x, (const KScal*)nullptr))) return prc;
    klaunch<(k_bi_init<T, Op>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, b, x, r, rhat, p,
                       v, c.partials, zg);
    klaunch<k_fin_bi_init>(c, dim3(1), dim3(kBlock), 0, c.stream, pa, nr, sc, rtol * rtol,
                       max_iters - total);
    CHECK_LAUNCH();
    int launched = 0;
    c.kt.begin_solve();
    while (true) {
      const int batch = std::min(next_batch(c.est[slot], launched), max_iters - total + 1 - launched);
      auto body = [&]() -> int {
        for (int k = 0; k < batch; ++k) {
          if (c.timing) c.kt.mark();
          int rc2;
          klaunch<(k_bi_p<T, Op>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, nl, op, r, p, v, phat,
                             csc);
          if ((rc2 = pre_apply(c, op, phat, csc))) return rc2;
          const int na = launch_bi_apply<T, 0>(c, op, nl, (const T*)phat, v, (const T*)rhat, csc);
          klaunch<k_fin_bi_apply<0>>(c, dim3(1), dim3(kBlock), 0, c.stream, pa, na, sc);
          klaunch<(k_bi_s<T, Op>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, nl, op, r, v, s, shat,
                             csc);
          if ((rc2 = pre_apply(c, op, shat, csc))) return rc2;
          const int nt = launch_bi_apply<T, 1>(c, op, nl, (const T*)shat, t, (const T*)s, csc);
          klaunch<k_fin_bi_apply<1>>(c, dim3(1), dim3(kBlock), 0, c.stream, pa, nt, sc);
          klaunch<(k_bi_x<T, Op>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, x, r, rhat,
                             phat, shat, s, t, c.partials, csc);
          klaunch<k_fin_bi_x>(c, dim3(1), dim3(kBlock), 0, c.stream, pa, nr, sc);
          CHECK_LAUNCH();
        }
        return IBFE_OK;
      };
      if ((prc = graph_run(c, graph_key(kGsBicg, slot, sizeof(T), batch), body))) return prc;
      launched += batch;
      int rc = poll(c, slot, st);
      if (rc) return rc;
      if (st.done || launched > max_iters - total) break;
    }
    if (c.timing) c.kt.drop_from(st.iters);
    total += st.iters;
    if (st.status == 1 && restart < 3 && total < max_iters) continue;
    break;
  }
  st.iters = total;
  c.est[slot] = std::max(1, total);
  out.iters = total;
  out.restarts = restarts;
  out.res = st.bb > 0.0 ? std::sqrt(st.rr / st.bb) : 0.0;
  return finish_status(st, "BiCGStab");
}

template <typename T, int NC>
void launch_extra(ibfe_ctx& c, const OpCSym<T, NC>& o, const T* x, const KScal* sc);
template <typename T, int NC>
ZOp<T> zcomp_op(const ibfe_ctx& c, const OpCSym<T, NC>& o);

// FP64 residual of the refinement loop: returns |r|^2 and |b|^2 on the host and
// leaves r in FP32 in r32.
template <class Op64, typename TR>
int ir_residual(ibfe_ctx& c, const Op64& op, const double* b, double* x, TR* r32, double& rr,
                double& bb, bool r_im = false) {
  int nr = red_blocks(c.nchunks);
  int prc;
  if ((prc = pre_apply(c, op, x, (const KScal*)nullptr))) return prc;
  if constexpr (std::is_same<Op64, OpSym<double, 1>>::value || std::is_same<Op64, OpSym<double, 3>>::value) {
    // constant-coefficient symmetric forms of the uniform grid: the z-blocked walk
    ZOp<double> z{};
    z.emask = op.emask;
    z.flags = op.flags;
    z.rowbit = op.rowbit;
    z.sy = op.sy;
    z.sz = op.sz;
    z.nplanes = c.plan.nz + 1;
    z.lanes = c.zlanes;
    z.zb = c.zb;
    for (int t = 0; t < 4; ++t) z.c[t] = op.c[t];
    z = with_im(c, z);
    nr = red_blocks(c.nzitems);
    if (r_im)
      klaunch<(k_zb_residual<TR, Op64::kNC, true>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                         c.nzitems, z, b, (const double*)x, r32, op.stride, c.partials, c.imstride);
    else
      klaunch<(k_zb_residual<TR, Op64::kNC>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                         c.nzitems, z, b, (const double*)x, r32, op.stride, c.partials, int64_t(0));
  } else if constexpr (std::is_same<Op64, OpCSym<double, 1>>::value ||
                       std::is_same<Op64, OpCSym<double, 3>>::value) {
    // composite symmetric forms: the fine-cell walk plus the precomputed extra rows
    launch_extra<double, Op64::kNC>(c, op, (const double*)x, (const KScal*)nullptr);
    const ZOp<double> z = zcomp_op(c, op);
    nr = red_blocks(c.nzitems);
    if (r_im)
      klaunch<(k_zb_residual<TR, Op64::kNC, true>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                                                    c.nzitems, z, b, (const double*)x, r32, op.stride, c.partials,
                                                    c.imstride);
    else
      klaunch<(k_zb_residual<TR, Op64::kNC>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                                              c.nzitems, z, b, (const double*)x, r32, op.stride, c.partials,
                                              int64_t(0));
  } else {
    if (r_im) return fail(IBFE_EINVAL, "internal: walk-order residual of a per-node operator");
    klaunch<(k_residual<Op64, TR>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, c.nl, op, b,
                       x, r32, c.partials);
  }
  klaunch<k_fin_residual>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr,
                     c.res2);
  CHECK_LAUNCH();
  HIP_TRY(hipMemcpyAsync(c.host_res2, c.res2, 2 * sizeof(double), hipMemcpyDeviceToHost, c.stream));
  HIP_TRY(hipStreamSynchronize(c.stream));
  rr = c.host_res2[0];
  bb = c.host_res2[1];
  if (!std::isfinite(rr) || !std::isfinite(bb)) return fail(IBFE_ENONFINITE, "refinement residual");
  return IBFE_OK;
}

// Mixed-precision solve A x = b: FP64 residuals and updates, FP32 inner Krylov
// corrections computed by inner(r32, d32, inner_rtol, SolveOut&) with inner_rtol =
// max(floor, 0.5 rtol / residual).  x holds the initial guess (zero off rows).
template <class Op64, class Inner>
int run_refined(ibfe_ctx& c, const Op64& op64, uint32_t rowbit, int nc, const double* b, double* x,
                float* r32, float* d32, double rtol, SolveOut& out, Inner&& inner, bool r_im = false,
                double floor = kInnerRtol) {
  const int nb = blocks_for(c.nchunks);
  int total = 0;
  double rr = 0, bb = 0, res = 0;
  int sweeps = 0;
  for (; sweeps <= kMaxSweeps; ++sweeps) {
    int rc = ir_residual(c, op64, b, x, r32, rr, bb, r_im);
    if (rc) return rc;
    res = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
    if (res <= rtol || sweeps == kMaxSweeps) break;
    const double tol_in = std::min(0.5, std::max(floor, 0.5 * rtol / res));
    SolveOut so;
    rc = inner((const float*)r32, d32, tol_in, so);
    total += so.iters;
    out.restarts += so.restarts;
    if (rc && rc != IBFE_ENOCONV) return rc;
    klaunch<k_add_correction<float>>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl,
                       c.flags, rowbit, (const float*)d32, x, nc, c.stride);
    CHECK_LAUNCH();
  }
  out.iters = total;
  out.res = res;
  out.outer = sweeps;
  if (res > rtol) return fail(IBFE_ENOCONV, "iterative refinement did not reach the tolerance");
  return IBFE_OK;
}

// -------------------------------------------------------------------------
// operators
// -------------------------------------------------------------------------

template <typename T, int NC>
OpSym<T, NC> sym_op(const ibfe_ctx& c, const double (&coef)[4], uint32_t rowbit) {
  OpSym<T, NC> op{};
  op.emask = c.emask;
  op.flags = c.flags;
  op.rowbit = rowbit;
  op.sy = int(c.plan.sy);
  op.sz = int(c.plan.sz);
  op.stride = c.stride;
  for (int t = 0; t < 4; ++t) op.c[t] = T(coef[t]);
  return op;
}

template <typename T>
OpStencil<T, 3> stencil_op(const ibfe_ctx& c, const T* coef, uint32_t rowbit) {
  OpStencil<T, 3> op{};
  op.coef = coef;
  op.flags = c.flags;
  op.rowbit = rowbit;
  op.sy = int(c.plan.sy);
  op.sz = int(c.plan.sz);
  op.stride = c.stride;
  return op;
}

// The tentative-velocity operator with the strain-rate cross blocks.
template <typename T>
OpStencilStrain<T> strain_op(const ibfe_ctx& c, const T* coef, uint32_t rowbit) {
  OpStencilStrain<T> op{};
  op.base = stencil_op<T>(c, coef, rowbit);
  op.emask = c.emask;
  op.mu = T(c.plan.params.mu);
  op.h = T(c.plan.h);
  op.stride = c.stride;
  return op;
}

OpCSR<3> gram_op(const ibfe_ctx& c) {
  OpCSR<3> op{};
  op.ptr = c.G_ptr;
  op.col = c.G_col;
  op.val = c.G_val;
  op.diag = c.G_diag;
  op.nrows = int(c.plan.M);
  op.stride = c.mstride;
  return op;
}


// -------------------------------------------------------------------------
// 2:1 refined lattice: composite operators (fine + coarse elements with the
// hanging-node constraint) behind the same Krylov drivers
// -------------------------------------------------------------------------

Children children_of(const ibfe_ctx& c) { return Children{c.pslot, c.par_ptr, c.par_child, c.nh}; }

template <typename T>
struct RefBufs;
template <>
struct RefBufs<double> {
  static const double* pw(const ibfe_ctx& c) { return c.pw64; }
  static double* yh(const ibfe_ctx& c) { return c.yh64; }
  static const double* dinvM(const ibfe_ctx& c) { return c.dinvM64; }
  static const double* dinvK(const ibfe_ctx& c) { return c.dinvK64; }
  static double* extra(const ibfe_ctx& c) { return c.extra64; }
};
template <>
struct RefBufs<float> {
  static const float* pw(const ibfe_ctx& c) { return c.pw32; }
  static float* yh(const ibfe_ctx& c) { return c.yh32; }
  static const float* dinvM(const ibfe_ctx& c) { return c.dinvM32; }
  static const float* dinvK(const ibfe_ctx& c) { return c.dinvK32; }
  static float* extra(const ibfe_ctx& c) { return c.extra32; }
};

// alpha M + beta K of the composite mesh: coef(h) = alpha m(h) + beta k(h)
template <typename T, int NC>
OpCSym<T, NC> csym_op(const ibfe_ctx& c, double alpha, double beta, uint32_t rowbit, const T* dinv) {
  OpCSym<T, NC> op{};
  op.emask = c.emask;
  op.cmask = c.cmask;
  op.flags = c.flags;
  op.rowbit = rowbit;
  op.sy = int(c.plan.sy);
  op.sz = int(c.plan.sz);
  op.stride = c.stride;
  for (int t = 0; t < 4; ++t) {
    op.cf[t] = T(alpha * c.fc.m[t] + beta * c.fc.k[t]);
    op.cc[t] = T(alpha * c.fcc.m[t] + beta * c.fcc.k[t]);
  }
  op.dinv = dinv;
  op.ch = children_of(c);
  op.pw = RefBufs<T>::pw(c);
  op.yh = RefBufs<T>::yh(c);
  return op;
}

// The z-blocked form of a composite symmetric operator: the fine-cell stencil
// walked over the column items, the Jacobi diagonal D' and the extra terms of
// the rows with coarse cells or hanging children (k_comp_extra, launched first).
template <typename T, int NC>
ZOp<T> zcomp_op(const ibfe_ctx& c, const OpCSym<T, NC>& o) {
  ZOp<T> z{};
  z.emask = o.emask;
  z.flags = o.flags;
  z.rowbit = o.rowbit;
  z.sy = o.sy;
  z.sz = o.sz;
  z.nplanes = c.plan.nz + 1;
  for (int t = 0; t < 4; ++t) z.c[t] = o.cf[t];
  z.zb = c.zb;
  z.lanes = c.zlanes;
  z.dinv = o.dinv;
  z.extra = RefBufs<T>::extra(c);
  z = with_im(c, z);
  return z;
}

template <typename T, int NC>
void launch_extra(ibfe_ctx& c, const OpCSym<T, NC>& o, const T* x, const KScal* sc) {
  if (c.nxn == 0) return;
  klaunch<(k_comp_extra<T, NC>)>(c, dim3(blocks_lin(c.nxn)), dim3(kBlock), 0, c.stream, c.nxn,
                     (const int32_t*)c.xnodes, o, x, RefBufs<T>::extra(c), sc);
}

// q = A p for the composite pressure operator (hanging rows already prepared).
template <typename T>
int launch_q(ibfe_ctx& c, const OpCSym<T, 1>& op, NodeList, const T* p, T* q, const KScal* sc) {
  launch_extra<T, 1>(c, op, p, sc);
  const int nr = red_blocks(c.nzitems);
  const ZOp<T> z = zcomp_op(c, op);
  klaunch<(k_cg_q_zb<T, 1>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems, c.nzitems, z,
                             op.stride, p, q, c.partials, sc);
  return nr;
}

template <typename T>
OpCStencil<T, 3> cstencil_op(const ibfe_ctx& c, const T* coef, uint32_t rowbit) {
  OpCStencil<T, 3> op{};
  op.coef = coef;
  op.cmask = c.cmask;
  op.flags = c.flags;
  op.rowbit = rowbit;
  op.sy = int(c.plan.sy);
  op.sz = int(c.plan.sz);
  op.stride = c.stride;
  op.ch = children_of(c);
  op.pw = RefBufs<T>::pw(c);
  op.yh = RefBufs<T>::yh(c);
  return op;
}

// The composite tentative-velocity operator with the strain-rate cross blocks.
template <typename T>
OpCStencilStrain<T> cstrain_op(const ibfe_ctx& c, const T* coef, uint32_t rowbit) {
  OpCStencilStrain<T> op{};
  op.base = cstencil_op<T>(c, coef, rowbit);
  op.emask = c.emask;
  op.mu = T(c.plan.params.mu);
  op.hf = T(c.plan.h);
  op.hc = T(c.plan.hb);
  op.stride = c.stride;
  op.yh = op.base.yh;
  return op;
}

// The matrix-free tentative-velocity operator: rows from the cell bits and u^n
// (FP64 u, or its FP32 copy w32 for the inner solves).
template <typename T>
OpConv<T> conv_op(const ibfe_ctx& c, uint32_t rowbit) {
  const Plan& P = c.plan;
  const double rdt = P.params.rho / P.params.dt, mu = P.params.mu;
  OpConv<T> op{};
  op.emask = c.emask;
  op.flags = c.flags;
  op.rowbit = rowbit;
  op.sy = int(P.sy);
  op.sz = int(P.sz);
  op.stride = c.stride;
  for (int t = 0; t < 4; ++t) op.c[t] = T(rdt * c.fc.m[t] + mu * c.fc.k[t]);
  op.rh2 = T(P.params.rho * P.h * P.h);
  if constexpr (std::is_same<T, double>::value) {
    op.w = c.w64;
    op.dinv = c.dinvS64;
  } else {
    op.w = c.w32;
    op.dinv = c.dinvS32;
  }
  return op;
}

template <typename T>
OpConvStrain<T> conv_strain_op(const ibfe_ctx& c, uint32_t rowbit) {
  OpConvStrain<T> op{};
  op.base = conv_op<T>(c, rowbit);
  op.mu = T(c.plan.params.mu);
  op.h = T(c.plan.h);
  op.stride = c.stride;
  return op;
}

template <typename T>
OpCConv<T> cconv_op(const ibfe_ctx& c, uint32_t rowbit) {
  const Plan& P = c.plan;
  const double rdt = P.params.rho / P.params.dt, mu = P.params.mu;
  OpCConv<T> op{};
  op.emask = c.emask;
  op.cmask = c.cmask;
  op.flags = c.flags;
  op.rowbit = rowbit;
  op.sy = int(P.sy);
  op.sz = int(P.sz);
  op.stride = c.stride;
  for (int t = 0; t < 4; ++t) {
    op.cf[t] = T(rdt * c.fc.m[t] + mu * c.fc.k[t]);
    op.cc[t] = T(rdt * c.fcc.m[t] + mu * c.fcc.k[t]);
  }
  op.rh2f = T(P.params.rho * P.h * P.h);
  op.rh2c = T(P.params.rho * P.hb * P.hb);
  if constexpr (std::is_same<T, double>::value) {
    op.w = c.w64;
    op.dinv = c.dinvS64;
  } else {
    op.w = c.w32;
    op.dinv = c.dinvS32;
  }
  op.ch = children_of(c);
  op.pw = RefBufs<T>::pw(c);
  op.yh = RefBufs<T>::yh(c);
  return op;
}

// The same for the Krylov solves and refinement residuals, whose pre_apply
// precomputes the coarse-cell and hanging-children terms of the flagged rows.
template <typename T>
OpCConv<T> cconv_solver_op(const ibfe_ctx& c, uint32_t rowbit) {
  OpCConv<T> op = cconv_op<T>(c, rowbit);
  op.extra = RefBufs<T>::extra(c);
  return op;
}

template <typename T>
OpCStencilStrain<T, OpCConv<T>> cconv_strain_op(const ibfe_ctx& c, uint32_t rowbit) {
  OpCStencilStrain<T, OpCConv<T>> op{};
  op.base = cconv_op<T>(c, rowbit);
  op.emask = c.emask;
  op.mu = T(c.plan.params.mu);
  op.hf = T(c.plan.h);
  op.hc = T(c.plan.hb);
  op.stride = c.stride;
  op.yh = op.base.yh;
  return op;
}

// Per step, matrix-free form: the inverse Jacobi diagonal of the rows of P (FP64,
// and with fp32 its FP32 rounding) and the FP32 copy of u^n (with fp32); u^n
// holds its hanging values.
int prep_s1_mf(ibfe_ctx& c, bool fp32) {
  const int nb = blocks_for(c.nchunks);
  float* d32 = fp32 ? c.dinvS32 : nullptr;
  float* w32 = fp32 ? c.w32 : nullptr;
  // the diagonal reads u^n itself (the copies are being written by the same kernel)
  if (c.plan.refined) {
    CConvDiag<double> f{cconv_op<double>(c, kFlagP), c.stride};
    f.op.w = c.u;
    klaunch<(k_conv_prep<CConvDiag<double>>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, f,
                                              (const double*)c.u, c.w64, w32, c.dinvS64, d32);
  } else {
    ConvDiag<double> f{conv_op<double>(c, kFlagP), c.stride};
    f.op.w = c.u;
    klaunch<(k_conv_prep<ConvDiag<double>>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, f,
                                             (const double*)c.u, c.w64, w32, c.dinvS64, d32);
  }
  CHECK_LAUNCH();
  return IBFE_OK;
}

GradElem grad_elem(const ibfe_ctx& c, const double* x) {
  GradElem g{};
  g.emask = c.emask;
  g.cmask = c.cmask;
  g.x = x;
  g.sy = int(c.plan.sy);
  g.sz = int(c.plan.sz);
  for (int k = 0; k < 3; ++k) {
    g.gf[k] = c.fc.g2[k];
    g.gc[k] = c.fcc.g2[k];
  }
  return g;
}

// x[h] = mean of the parents of every hanging node (nc planes)
template <typename T>
int fill_hanging(ibfe_ctx& c, T* x, int nc) {
  if (c.nh == 0) return IBFE_OK;
  klaunch<k_hang_fill<T>>(c, dim3(blocks_lin(c.nh)), dim3(kBlock), 0, c.stream, c.nh,
                     (const int32_t*)c.hang_ids, (const int32_t*)c.hang_par, x, nc, c.stride,
                     (const KScal*)nullptr);
  CHECK_LAUNCH();
  return IBFE_OK;
}

// out = scale * C^T (element rows of f) on rows; f's inputs must be filled.
template <typename T, class F>
int comp_rows(ibfe_ctx& c, const F& f, uint32_t rowbit, uint32_t exclude, T scale, T* out) {
  T* yh = RefBufs<T>::yh(c);
  if (c.nh)
    klaunch<(k_hang_elem<T, F>)>(c, dim3(blocks_lin(c.nh)), dim3(kBlock), 0, c.stream, c.nh,
                       (const int32_t*)c.hang_ids, f, yh, (const KScal*)nullptr);
  klaunch<(k_comp_rows<T, F>)>(c, dim3(blocks_for(c.nchunks)), dim3(kBlock), 0, c.stream,
                     c.nl, f, (const uint8_t*)c.flags, rowbit, exclude, scale,
                     children_of(c), RefBufs<T>::pw(c), (const T*)yh, out, c.stride);
  CHECK_LAUNCH();
  return IBFE_OK;
}

int cheb_steps(double tol, double lmin, double lmax) {
  const double kappa = lmax / lmin;
  const double q = (std::sqrt(kappa) - 1.0) / (std::sqrt(kappa) + 1.0);
  return int(std::ceil((std::log(2.0 / tol) + 0.5 * std::log(kappa)) / std::log(1.0 / q)));
}

// x = Cheb_iters(b) from x = 0 for any operator on [lmin, lmax] of D^-1 A.
// With IMV, b and d are in walk order (the mass correction's residual and
// Chebyshev direction), x and xalt on the lattice.
template <typename T, class Op, bool IMV = false>
int run_cheb_gen(ibfe_ctx& c, const Op& op, const T* b, T* x, T* xalt, T* d, int iters, double lmin,
                 double lmax) {
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  T* cur = ((iters - 1) % 2 == 0) ? x : xalt;
  T* alt = cur == x ? xalt : x;
  const int nr = red_blocks(c.nzitems);
  const ZOp<T> zop = zcomp_op(c, op);
  if (IMV)
    klaunch<(k_cheb0_im<T, Op::kNC>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems, c.nzitems,
                                      zop, b, d, cur, T(1.0 / theta), c.stride, c.imstride);
  else
    klaunch<(k_cheb0_gen<T, Op>)>(c, dim3(blocks_for(c.nchunks)), dim3(kBlock), 0, c.stream,
                       c.nl, op, b, d, cur, T(1.0 / theta), (const KScal*)nullptr);
  int rc;
  T* const cur0 = cur;
  T* const alt0 = alt;
  auto body = [&]() -> int {
    double rho = 1.0 / sigma;
    int rc2;
    for (int k = 1; k < iters; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      const T c1 = T(rn * rho), c2 = T(2.0 * rn / delta);
      rho = rn;
      if ((rc2 = pre_apply(c, op, cur, (const KScal*)nullptr))) return rc2;
      constexpr int NC = Op::kNC;
      launch_extra<T, NC>(c, op, cur, (const KScal*)nullptr);
      // the first step writes the zeros off the rows into the second buffer (the
      // zero-start step did so for the first one and for d, over every active node)
      klaunch<(k_zb_cheb<T, false, NC, IMV>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                                              c.nzitems, zop, (const T*)cur, b, d, alt, c1, c2, c.partials,
                                              (const KScal*)nullptr, op.stride, k == 1 ? 1 : 0,
                                              IMV ? c.imstride : int64_t(0));
      std::swap(cur, alt);
    }
    CHECK_LAUNCH();
    return IBFE_OK;
  };
  if ((rc = graph_run(c, graph_key(kGsChebGen, IMV ? 1 : 0, sizeof(T), iters), body))) return rc;
  // the sequence swaps the buffers iters - 1 times (a graph replay does not run body)
  cur = ((iters - 1) % 2 == 0) ? cur0 : alt0;
  if (cur != x) return fail(IBFE_EINVAL, "internal: Chebyshev result buffer");
  return IBFE_OK;
}

// -------------------------------------------------------------------------
// multigrid-preconditioned CG for the pressure increment
// -------------------------------------------------------------------------

// Chebyshev-Jacobi smoother on [lambda_max / 4, lambda_max] with the bound
// lambda_max = 2 of D^-1 K (Gershgorin: every off-diagonal of the Q1
// stiffness is <= 0 and its rows sum to zero).
struct Cheb {
  double c1[32], c2[32];
};
Cheb cheb_coefs(int m) {
  const double lmax = 2.0, lmin = 0.5;
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  Cheb ch{};
  double rho = 1.0 / sigma;
  ch.c1[0] = 0.0;
  ch.c2[0] = 1.0 / theta;
  for (int k = 1; k < m && k < 32; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    ch.c1[k] = rn * rho;
    ch.c2[k] = 2.0 * rn / delta;
    rho = rn;
  }
  return ch;
}

constexpr int kSmooth = 1;        // Chebyshev degree of pre- and post-smoothing
constexpr int kCoarseSmooth = 16; // coarsest-level smoothing when no dense inverse; with a
                                  // single level this is the Chebyshev preconditioner

template <typename T>
ZOp<T> level_op(const MGDev<T>& L) {
  ZOp<T> z{};
  z.emask = L.emask;
  z.flags = L.flags;
  z.rowbit = kMgRow;
  z.sy = int(L.sy);
  z.sz = int(L.sz);
  z.nplanes = L.nz + 1;
  z.lanes = L.zlanes;
  z.zb = L.zb;
  for (int t = 0; t < 4; ++t) z.c[t] = T(L.kc[t]);
  return z;
}

// m Chebyshev steps on level L for b, continuing from *x (zero_start: from x = 0);
// ping-pongs between *x and *alt.  With dot, the last step writes partials of b.x.
// The same smoother on the composite level of a refined lattice: Jacobi with
// the lumped constrained diagonal D', whose D'^-1 K spectrum is also bounded by
// 2 (every element stiffness has non-positive off-diagonal entries and zero row
// sums, and the constraint only adds the children's diagonals to the parents).
template <typename T>
int smooth_comp(ibfe_ctx& c, const MGDev<T>& L, const T* b, T*& x, T*& alt, int m, bool zero_start,
                bool dot, const KScal* sc, int& nparts) {
  const Cheb ch = cheb_coefs(m);
  const auto op = csym_op<T, 1>(c, 0.0, 1.0, kMgRow, RefBufs<T>::dinvK(c));
  const ZOp<T> zop = zcomp_op(c, op);
  using Op = OpCSym<T, 1>;
  const int nr = red_blocks(c.nzitems), nb = blocks_for(c.nchunks);
  int rc;
  for (int k = 0; k < m; ++k) {
    const bool last = k == m - 1;
    if (k == 0 && zero_start && !(last && dot)) {
      klaunch<(k_cheb0_gen<T, Op>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, op, b, L.d, x, T(ch.c2[0]), sc);
      continue;
    }
    if (k == 0 && zero_start)
      klaunch<(k_cheb0_gen<T, Op>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, op, b, L.d, x, T(0), sc);
    if ((rc = pre_apply(c, op, x, sc))) return rc;
    launch_extra<T, 1>(c, op, x, sc);
    if (last && dot)
      klaunch<(k_zb_cheb<T, true>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                         c.nzitems, zop, (const T*)x, b, L.d, alt, T(ch.c1[k]), T(ch.c2[k]), c.partials, sc, int64_t(0), 1, int64_t(0));
    else
      klaunch<(k_zb_cheb<T, false>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                         c.nzitems, zop, (const T*)x, b, L.d, alt, T(ch.c1[k]), T(ch.c2[k]), c.partials, sc, int64_t(0), 1, int64_t(0));
    std::swap(x, alt);
  }
  nparts = nr;
  CHECK_LAUNCH();
  return IBFE_OK;
}

template <typename T>
int smooth(ibfe_ctx& c, const MGDev<T>& L, const T* b, T*& x, T*& alt, int m, bool zero_start,
           bool dot, const KScal* sc, int& nparts) {
  if (L.composite) return smooth_comp<T>(c, L, b, x, alt, m, zero_start, dot, sc, nparts);
  const Cheb ch = cheb_coefs(m);
  const ZOp<T> op = level_op(L);
  const int nr = red_blocks(L.nzitems);
  for (int k = 0; k < m; ++k) {
    const bool last = k == m - 1;
    if (k == 0 && zero_start && !(last && dot)) {
      klaunch<k_mg_cheb0<T>>(c, dim3(blocks_for(L.nchunks)), dim3(kBlock), 0, c.stream,
                         L.nl, (const uint8_t*)L.emask, (const uint8_t*)L.flags,
                         T(L.kc[0]), T(ch.c2[0]), b, L.d, x, sc, kMgRow, int64_t(0));
      continue;  // x already holds the result: no swap
    }
    const T* xin = x;
    if (k == 0 && zero_start) {
      // degree-1 smoothing from zero with a dot: x is zero on entry
      klaunch<k_mg_cheb0<T>>(c, dim3(blocks_for(L.nchunks)), dim3(kBlock), 0, c.stream,
                         L.nl, (const uint8_t*)L.emask, (const uint8_t*)L.flags,
                         T(L.kc[0]), T(0), b, L.d, x, sc, kMgRow, int64_t(0));
      xin = x;
    }
    if (last && dot)
      klaunch<(k_zb_cheb<T, true>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)L.zitems,
                         L.nzitems, op, xin, b, L.d, alt, T(ch.c1[k]), T(ch.c2[k]), c.partials, sc, int64_t(0), 1, int64_t(0));
    else
      klaunch<(k_zb_cheb<T, false>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)L.zitems,
                         L.nzitems, op, xin, b, L.d, alt, T(ch.c1[k]), T(ch.c2[k]), c.partials, sc, int64_t(0), 1, int64_t(0));
    std::swap(x, alt);
  }
  nparts = nr;
  CHECK_LAUNCH();
  return IBFE_OK;
}

// z = V(r): one symmetric V(kSmooth, kSmooth) cycle.  Writes the partials of r.z
// and returns their count in nparts.
// pre0: the caller has already written the finest level's pre-smoothing into
// lv[0].xt (fused into the CG update that produced r0).
template <typename T>
int vcycle(ibfe_ctx& c, std::vector<MGDev<T>>& lv, const T* r0, T* z0, const KScal* sc, int& nparts,
           bool pre0 = false) {
  const int L = int(lv.size());
  std::vector<T*> cur(L), alt(L);
  // level 0 result must end in z0: pre (m-1 swaps) + post (m swaps) is odd
  cur[0] = lv[0].xt;
  alt[0] = z0;
  for (int l = 1; l < L; ++l) {
    cur[l] = lv[l].x;
    alt[l] = lv[l].xt;
  }
  int np = 0, rc;
  // with degree-1 pre-smoothing, the restriction onto a level that is not the
  // coarsest also writes that level's pre-smoothed iterate (c2 D^-1 b from zero)
  static_assert(kSmooth == 1, "the restriction forms the degree-1 pre-smoothing");
  const T c2pre = T(cheb_coefs(kSmooth).c2[0]);
  for (int l = 0; l + 1 < L; ++l) {
    const MGDev<T>& A = lv[l];
    const T* b = l == 0 ? r0 : A.b;
    if (l == 0 && !pre0 && (rc = smooth<T>(c, A, b, cur[l], alt[l], kSmooth, true, false, sc, np))) return rc;
    if (A.composite) {
      const auto op = csym_op<T, 1>(c, 0.0, 1.0, kMgRow, RefBufs<T>::dinvK(c));
      if ((rc = pre_apply(c, op, cur[l], sc))) return rc;
      launch_extra<T, 1>(c, op, cur[l], sc);
      klaunch<k_zb_resid<T>>(c, dim3(red_blocks(c.nzitems)), dim3(kBlock), 0, c.stream,
                         (const int*)c.zitems, c.nzitems, zcomp_op(c, op), (const T*)cur[l], b, A.r, sc);
    } else {
      klaunch<k_zb_resid<T>>(c, dim3(red_blocks(A.nzitems)), dim3(kBlock), 0, c.stream,
                         (const int*)A.zitems, A.nzitems, level_op(A), (const T*)cur[l], b, A.r, sc);
    }
    const MGDev<T>& C = lv[l + 1];
    const bool fuse = l + 2 < L;  // level l + 1 is smoothed, not solved
    klaunch<k_mg_restrict<T>>(c, dim3(blocks_for(C.nchunks)), dim3(kBlock), 0, c.stream,
                       C.nl, (const uint8_t*)C.flags, int(C.sy), int(C.sz),
                       int(A.sy), int(A.sz), A.nx, A.ny, A.nz, (const T*)A.r, C.b, sc,
                       fuse ? (const uint8_t*)C.emask : (const uint8_t*)nullptr, T(C.kc[0]), c2pre,
                       fuse ? cur[l + 1] : (T*)nullptr);
    CHECK_LAUNCH();
  }
  {
    const MGDev<T>& C = lv[L - 1];
    const T* b = L == 1 ? r0 : C.b;
    if (C.m > 0) {
      if (L == 1) cur[0] = z0;  // single level: the dense solve is the whole cycle
      klaunch<k_mg_dense<T>>(c, dim3((C.m + kWaves - 1) / kWaves), dim3(kBlock), 0, c.stream, C.m,
                         (const int64_t*)C.ids, (const T*)C.inv, b, cur[L - 1], sc);
      if (L == 1) {
        np = red_blocks(C.nchunks);
        klaunch<k_mg_dot<T>>(c, dim3(np), dim3(kBlock), 0, c.stream, C.nl,
                           (const uint8_t*)C.flags, b, (const T*)z0, c.partials, sc);
      }
      CHECK_LAUNCH();
    } else if ((rc = smooth<T>(c, C, b, cur[L - 1], alt[L - 1], kCoarseSmooth, true, L == 1, sc, np))) {
      return rc;
    }
  }
  for (int l = L - 2; l >= 0; --l) {
    const MGDev<T>& A = lv[l];
    const MGDev<T>& C = lv[l + 1];
    klaunch<k_mg_prolong<T>>(c, dim3(blocks_for(A.nchunks)), dim3(kBlock), 0, c.stream,
                       A.nl, (const uint8_t*)A.flags, int(A.sy), int(A.sz),
                       int(C.sy), int(C.sz), (const T*)cur[l + 1], cur[l], sc);
    CHECK_LAUNCH();
    const T* b = l == 0 ? r0 : A.b;
    if ((rc = smooth<T>(c, A, b, cur[l], alt[l], kSmooth, false, l == 0, sc, np))) return rc;
  }
  if (cur[0] != z0) return fail(IBFE_EINVAL, "internal: V-cycle result buffer");
  nparts = np;
  return IBFE_OK;
}

// CG on K_{P'P'} x = b preconditioned by one V-cycle per iteration; x starts at 0.
template <typename T, class Op>
int run_pcg_mg(ibfe_ctx& c, const Op& op, std::vector<MGDev<T>>& lv, const T* b, T* x, T* r, T* p, T* q,
               T* z, int slot, double rtol, int max_iters, SolveOut& out) {
  const int nr = red_blocks(c.nchunks);
  KScal* sc = &c.scal[slot];
  const KScal* csc = sc;
  int rc, np = 0;
  // the finest level's degree-1 pre-smoothing is formed by the CG kernels that
  // produce the V-cycle's input (a uniform finest level with more levels below)
  const bool pre0 = !lv[0].composite && lv.size() > 1;
  const uint8_t* pe = pre0 ? (const uint8_t*)lv[0].emask : nullptr;
  T* const px = pre0 ? lv[0].xt : nullptr;
  const T pc0 = T(lv[0].kc[0]), pc2 = T(cheb_coefs(kSmooth).c2[0]);
  klaunch<k_mgcg_init<T>>(c, dim3(nr), dim3(kBlock), 0, c.stream, c.nl,
                     (const uint8_t*)c.flags, b, x, r, c.partials, pe, pc0, pc2, px);
  klaunch<k_fin_mgcg_init>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr, sc,
                     rtol * rtol, max_iters);
  CHECK_LAUNCH();
  if ((rc = vcycle<T>(c, lv, r, z, csc, np, pre0))) return rc;
  klaunch<k_fin_mgcg_rz>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, np, sc, 1);
  klaunch<k_mgcg_p<T>>(c, dim3(blocks_for(c.nchunks)), dim3(kBlock), 0, c.stream, c.nl, (const uint8_t*)c.flags, (const T*)z, p, csc);
  CHECK_LAUNCH();
  int launched = 0;
  KScal s{};
  c.kt.begin_solve();
  while (true) {
    const int batch = std::min(launched == 0 ? std::min(kMaxGraphIters, std::max(2, c.est[slot] - 1)) : 2, max_iters + 1 - launched);
    auto body = [&]() -> int {
      for (int k = 0; k < batch; ++k) {
        if (c.timing) c.kt.mark();
        int rc2;
        if ((rc2 = pre_apply(c, op, p, csc))) return rc2;
        const int nq = launch_q<T>(c, op, c.nl, (const T*)p, q, csc);
        klaunch<k_fin_cg_q>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nq, sc);
        klaunch<k_mgcg_xr<T>>(c, dim3(nr), dim3(kBlock), 0, c.stream, c.nl,
                           (const uint8_t*)c.flags, x, r, (const T*)p, (const T*)q, c.partials, csc, pe, pc0,
                           pc2, px);
        klaunch<k_fin_mgcg_xr>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr,
                           sc);
        CHECK_LAUNCH();
        if ((rc2 = vcycle<T>(c, lv, r, z, csc, np, pre0))) return rc2;
        klaunch<k_fin_mgcg_rz>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, np,
                           sc, 0);
        klaunch<k_mgcg_p<T>>(c, dim3(blocks_for(c.nchunks)), dim3(kBlock), 0, c.stream,
                           c.nl, (const uint8_t*)c.flags, (const T*)z, p, csc);
        CHECK_LAUNCH();
      }
      return IBFE_OK;
    };
    if ((rc = graph_run(c, graph_key(kGsPcgMg, slot, sizeof(T), batch), body))) return rc;
    launched += batch;
    if ((rc = poll(c, slot, s))) return rc;
    if (s.done || launched > max_iters) break;
  }
  if (c.timing) c.kt.drop_from(s.iters);
  c.est[slot] = std::max(1, s.iters);
  out.iters = s.iters;
  out.res = s.bb > 0.0 ? std::sqrt(s.rr / s.bb) : 0.0;
  return finish_status(s, "multigrid CG");
}


// Force system G Lambda = b of the IB correction (FP64): CG with the block-Jacobi
// preconditioner of ib_pcg.hpp, from x (the last step's force) unless zero_guess;
// four kernels per iteration, the search direction alternating between p and p2.
int run_ib_pcg(ibfe_ctx& c, const double* b, double* x, double* r, double* p, double* p2, double* q,
               double* z, int slot, double rtol, int max_iters, bool zero_guess, SolveOut& out) {
  const OpCSR<3> op = gram_op(c);
  const NodeList nl = c.ib_nl;
  const int M = int(c.plan.M);
  const int nr = red_blocks(nl.n), nb = blocks_for(nl.n);
  const int nblk = (M + kIBBlock - 1) / kIBBlock;
  const int nj = std::max(1, std::min(kRedBlocks, nblk));
  const int ng = std::max(1, std::min(kRedBlocks, (M + kBlock / kIBLanes - 1) / (kBlock / kIBLanes)));
  const int64_t S = c.mstride;
  KScal* sc = &c.scal[slot];
  const KScal* csc = sc;
  klaunch<k_ibcg_init>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, b, x, r, c.partials,
                     zero_guess ? 1 : 0);
  klaunch<k_fin_mgcg_init>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr, sc,
                     rtol * rtol, max_iters);
  klaunch<k_ib_bjac>(c, dim3(nj), dim3(kBlock), 0, c.stream, M, nblk, (const float*)c.G_binv,
                     (const double*)r, z, S, c.partials, csc);
  klaunch<k_fin_mgcg_rz>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nj, sc, 1);
  // the first direction is z + 0 p: p must hold finite values
  klaunch<k_zero<double>>(c, dim3(nb), dim3(kBlock), 0, c.stream, nl, p, 3, S);
  CHECK_LAUNCH();
  double* pb[2] = {p, p2};
  int par = 0;  // pb[par] holds the current direction
  int launched = 0, rc;
  KScal s{};
  c.kt.begin_solve();
  while (true) {
    const int batch = std::min(next_batch(c.est[slot], launched), max_iters + 1 - launched);
    auto body = [&]() -> int {
      for (int k = 0; k < batch; ++k) {
        if (c.timing) c.kt.mark();
        const double* pold = pb[(par + k) % 2];
        double* pnew = pb[(par + k + 1) % 2];
        klaunch<k_ibcg_qp>(c, dim3(ng), dim3(kBlock), 0, c.stream, M, (const int64_t*)c.G_ptr,
                           (const int32_t*)c.G_col, (const double*)c.G_val, S, (const double*)z, pold, pnew, q,
                           c.partials, csc);
        klaunch<k_fin_cg_q>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, ng, sc);
        klaunch<k_ib_xr_bjac>(c, dim3(nj), dim3(kBlock), 0, c.stream, M, nblk, (const float*)c.G_binv,
                           x, r, (const double*)pnew, (const double*)q, z, S, c.partials, csc);
        klaunch<k_fin_ibcg>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nj, sc);
        CHECK_LAUNCH();
      }
      return IBFE_OK;
    };
    if ((rc = graph_run(c, graph_key(kGsIbPcg, slot, sizeof(double), batch | (par << 20)), body))) return rc;
    launched += batch;
    par = (par + batch) % 2;
    if ((rc = poll(c, slot, s))) return rc;
    if (s.done || launched > max_iters) break;
  }
  if (c.timing) c.kt.drop_from(s.iters);
  c.est[slot] = std::max(1, s.iters);
  out.iters = s.iters;
  out.res = s.bb > 0.0 ? std::sqrt(s.rr / s.bb) : 0.0;
  return finish_status(s, "IB force CG");
}

// -------------------------------------------------------------------------
// Chebyshev iteration for the consistent-mass correction M_FF x = b.  For Q1
// cubes the generalized eigenvalues of (M, diag M) lie in [1/8, 27/8]: the
// Rayleigh quotient is a ratio of sums of element quadratic forms and each
// element gives diag(M_e)^-1 M_e = (1/2..3/2)^3; a principal submatrix (free
// rows) stays inside.  No inner products are needed.
// -------------------------------------------------------------------------

constexpr double kMassLmin = 1.0 / 8.0, kMassLmax = 27.0 / 8.0;

int mass_cheb_steps(double tol) {
  const double kappa = kMassLmax / kMassLmin;
  const double q = (std::sqrt(kappa) - 1.0) / (std::sqrt(kappa) + 1.0);
  return int(std::ceil((std::log(2.0 / tol) + 0.5 * std::log(kappa)) / std::log(1.0 / q)));
}

// x = Cheb_iters(b) from x = 0 (x, xalt, d: 3-plane vectors).
template <typename T, bool IMV = false>
int run_cheb_mass(ibfe_ctx& c, const T* b, T* x, T* xalt, T* d, int iters) {
  const Plan& P = c.plan;
  const double theta = 0.5 * (kMassLmax + kMassLmin), delta = 0.5 * (kMassLmax - kMassLmin);
  const double sigma = theta / delta;
  ZOp<T> op{};
  op.emask = c.emask;
  op.flags = c.flags;
  op.rowbit = kFlagF;
  op.sy = int(P.sy);
  op.sz = int(P.sz);
  op.nplanes = P.nz + 1;
  op.lanes = c.zlanes;
  op.zb = c.zb;
  for (int t = 0; t < 4; ++t) op.c[t] = T(c.fc.m[t]);
  op = with_im(c, op);
  T* cur = ((iters - 1) % 2 == 0) ? x : xalt;
  T* alt = cur == x ? xalt : x;
  const int nr = red_blocks(c.nzitems);
  if (IMV)
    klaunch<(k_cheb0_im<T, 3>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems, c.nzitems, op, b,
                                d, cur, T(1.0 / theta), c.stride, c.imstride);
  else
    klaunch<(k_mg_cheb0<T, 3>)>(c, dim3(blocks_for(c.nchunks)), dim3(kBlock), 0, c.stream,
                       c.nl, (const uint8_t*)c.emask, (const uint8_t*)c.flags,
                       T(c.fc.m[0]), T(1.0 / theta), b, d, cur, (const KScal*)nullptr, kFlagF, c.stride);
  T* const cur0 = cur;
  T* const alt0 = alt;
  auto body = [&]() -> int {
    double rho = 1.0 / sigma;
    for (int k = 1; k < iters; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      const T c1 = T(rn * rho), c2 = T(2.0 * rn / delta);
      rho = rn;
      // the first step writes the zeros off the free rows into the second buffer
      // (the zero-start step did so for the first one and for d)
      const int zero_off = k == 1 ? 1 : 0;
      klaunch<(k_zb_cheb<T, false, 3, IMV>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                                             c.nzitems, op, (const T*)cur, b, d, alt, c1, c2, c.partials,
                                             (const KScal*)nullptr, c.stride, zero_off,
                                             IMV ? c.imstride : int64_t(0));
      std::swap(cur, alt);
    }
    CHECK_LAUNCH();
    return IBFE_OK;
  };
  if (int rcb = graph_run(c, graph_key(kGsChebMass, IMV ? 1 : 0, sizeof(T), iters), body)) return rcb;
  // the sequence swaps the buffers iters - 1 times (a graph replay does not run body)
  cur = ((iters - 1) % 2 == 0) ? cur0 : alt0;
  if (cur != x) return fail(IBFE_EINVAL, "internal: Chebyshev result buffer");
  return IBFE_OK;
}

// Chebyshev interval of P M for the tensor-product preconditioner of the mass
// correction (zblock.hpp).  The interior spectrum is [27/64, 1]; the rows at the
// wall widen it (measured: 0.41 .. 1.06 on the cylinder, 0.41 .. 1.23 on the
// three-branch arch, up to 1.57 on irregular blob masks).  The iteration reduces
// every error component whose eigenvalue lies in (0, lmin + lmax), those inside
// the interval at the designed rate.
constexpr double kTmLmin = 0.40, kTmLmax = 1.60;

template <typename T>
struct TmBufs;
template <>
struct TmBufs<double> {
  static double* w(const ibfe_ctx& c) { return c.tmw64; }
  static double* wx(const ibfe_ctx& c) { return c.tmwx64; }
};
template <>
struct TmBufs<float> {
  static float* w(const ibfe_ctx& c) { return c.tmw32; }
  static float* wx(const ibfe_ctx& c) { return c.tmwx32; }
};

// The mass walk of the uniform grid (cell diagonal op.c[0]; walk-order cell
// bits and flags).
template <typename T>
ZOp<T> mass_zop(const ibfe_ctx& c) {
  const Plan& P = c.plan;
  ZOp<T> op{};
  op.emask = c.emask;
  op.flags = c.flags;
  op.rowbit = kFlagF;
  op.sy = int(P.sy);
  op.sz = int(P.sz);
  op.nplanes = P.nz + 1;
  op.lanes = c.zlanes;
  op.zb = c.zb;
  for (int t = 0; t < 4; ++t) op.c[t] = T(c.fc.m[t]);
  return with_im(c, op);
}

// x = Cheb_iters(b) from x = 0 for M_FF x = b preconditioned by P = D^-1/2 T D^-1/2
// on [kTmLmin, kTmLmax].  zop: the mass walk (on a refined lattice with the
// lumped constrained diagonal and the extra terms); pre(x) runs before each
// residual pass (the hanging values and extra terms of x).  With IMV, b and d
// are in walk order; x on the lattice, updated in place.
template <typename T, int NC, bool IMV, class Pre>
int run_cheb_tm(ibfe_ctx& c, const ZOp<T>& zop, const T* b, T* x, T* d, int iters, Pre&& pre) {
  const double theta = 0.5 * (kTmLmax + kTmLmin), delta = 0.5 * (kTmLmax - kTmLmin);
  const double sigma = theta / delta;
  T* w = TmBufs<T>::w(c);
  if (w == nullptr) return fail(IBFE_EINVAL, "internal: tensor mass buffers not allocated");
  T* wx = c.plan.refined ? TmBufs<T>::wx(c) : nullptr;
  T* zx = c.plan.refined ? RefBufs<T>::extra(c) : nullptr;
  const int nr = red_blocks(c.nzitems);
  const int64_t ims = IMV ? c.imstride : int64_t(0);
  const T tw = T(kTensorT);
  auto tsum = [&]() {
    if (wx != nullptr && c.nxn > 0)
      klaunch<(k_tm_extra<T, NC>)>(c, dim3(blocks_lin(c.nxn)), dim3(kBlock), 0, c.stream, c.nxn,
                                   (const int32_t*)c.xnodes, (const uint8_t*)c.flags, zop.rowbit, (const T*)wx, zx,
                                   tw, zop.sy, zop.sz, zop.nplanes, c.stride);
  };
  auto body = [&]() -> int {
    klaunch<(k_tm_scale<T, NC, IMV>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems, c.nzitems,
                                      zop, b, w, wx, c.stride, ims);
    tsum();
    klaunch<(k_tm_cheb<T, NC, IMV, true>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                                           c.nzitems, zop, (const T*)w, (const T*)zx, d, x, T(0),
                                           T(1.0 / theta), tw, c.stride, ims);
    double rho = 1.0 / sigma;
    for (int k = 1; k < iters; ++k) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      const T c1 = T(rn * rho), c2 = T(2.0 * rn / delta);
      rho = rn;
      int rc2;
      if ((rc2 = pre(x))) return rc2;
      klaunch<(k_tm_resid<T, NC, IMV>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                                        c.nzitems, zop, (const T*)x, b, w, wx, c.stride, ims);
      tsum();
      klaunch<(k_tm_cheb<T, NC, IMV, false>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, (const int*)c.zitems,
                                              c.nzitems, zop, (const T*)w, (const T*)zx, d, x, c1, c2, tw,
                                              c.stride, ims);
    }
    CHECK_LAUNCH();
    return IBFE_OK;
  };
  return graph_run(c, graph_key(kGsChebTm, IMV ? 1 : 0, sizeof(T), iters), body);
}

}  // namespace
extern "C" {
struct ibfe_batcher {
  int device = 0;
  hipStream_t stream = nullptr;
  double window_us = 0.0;
  std::mutex mu;
  std::condition_variable cv;
  struct Pending {
    ibfe::ChebJob<float> job{};
    ibfe_ctx* ctx = nullptr;
    bool launched = false;
    int rc = 0;
  };
  std::vector<Pending*> queue;
  int members = 0;       // attached contexts
  bool leading = false;  // a member thread is forming and launching a batch
  int64_t batches = 0, jobs = 0;
  int32_t widest = 0;
};
}  // extern "C"
namespace {

// Launch one batch on the batcher's stream: after every member's ready event,
// the Chebyshev steps 1 .. max iters - 1 over all members' items, then each
// member's done event.
int launch_cheb_batch(ibfe_batcher& B, const std::vector<ibfe_batcher::Pending*>& take) {
  const double theta = 0.5 * (kMassLmax + kMassLmin), delta = 0.5 * (kMassLmax - kMassLmin);
  const double sigma = theta / delta;
  ChebBatch<float> cb{};
  cb.njobs = int(take.size());
  cb.off[0] = 0;
  int maxit = 1;
  for (int i = 0; i < cb.njobs; ++i) {
    HIP_TRY(hipStreamWaitEvent(B.stream, take[i]->ctx->ev_ready, 0));
    cb.job[i] = take[i]->job;
    cb.off[i + 1] = cb.off[i] + cb.job[i].nblocks;
    maxit = std::max(maxit, cb.job[i].iters);
  }
  double rho = 1.0 / sigma;
  for (int k = 1; k < maxit; ++k) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    const float c1 = float(rn * rho), c2 = float(2.0 * rn / delta);
    rho = rn;
    hipLaunchKernelGGL((k_zb_cheb_batch<float, 3>), dim3(cb.off[cb.njobs]), dim3(kBlock), 0, B.stream, cb, k, c1,
                       c2);
  }
  HIP_TRY(hipGetLastError());
  for (auto* p : take) HIP_TRY(hipEventRecord(p->ctx->ev_done, B.stream));
  return IBFE_OK;
}

// run_cheb_mass<float> through the context's batcher: the zero-start step on
// the context's stream, then steps 1 .. iters - 1 in a batch with the other
// members that reach this stage within the window.
int batched_cheb_mass(ibfe_ctx& c, const float* b, float* x, float* xalt, float* d, int iters) {
  const Plan& P = c.plan;
  const double theta = 0.5 * (kMassLmax + kMassLmin);
  float* cur0 = ((iters - 1) % 2 == 0) ? x : xalt;
  float* alt0 = cur0 == x ? xalt : x;
  ibfe_batcher::Pending me;
  ChebJob<float>& J = me.job;
  J.items = c.zitems;
  J.nitems = c.nzitems;
  J.nblocks = red_blocks(c.nzitems);
  J.iters = iters;
  J.op.emask = c.emask;
  J.op.flags = c.flags;
  J.op.rowbit = kFlagF;
  J.op.sy = int(P.sy);
  J.op.sz = int(P.sz);
  J.op.nplanes = P.nz + 1;
  J.op.lanes = c.zlanes;
  J.op.zb = c.zb;
  for (int t = 0; t < 4; ++t) J.op.c[t] = float(c.fc.m[t]);
  J.op = with_im(c, J.op);
  J.b = b;
  J.d = d;
  J.buf0 = cur0;
  J.buf1 = alt0;
  J.stride = c.stride;
  J.imstride = c.imstride;
  klaunch<(k_cheb0_im<float, 3>)>(c, dim3(J.nblocks), dim3(kBlock), 0, c.stream, (const int*)c.zitems, c.nzitems,
                                  J.op, b, d, cur0, float(1.0 / theta), c.stride, c.imstride);
  CHECK_LAUNCH();
  if (iters <= 1) return IBFE_OK;
  ibfe_batcher& B = *c.batcher;
  me.ctx = &c;
  HIP_TRY(hipEventRecord(c.ev_ready, c.stream));
  std::unique_lock<std::mutex> lk(B.mu);
  B.queue.push_back(&me);
  B.cv.notify_all();
  while (!me.launched) {
    if (B.leading) {
      B.cv.wait(lk, [&] { return me.launched || !B.leading; });
      continue;
    }
    B.leading = true;
    const int want = std::min(B.members, kMaxBatch);
    B.cv.wait_for(lk, std::chrono::duration<double, std::micro>(B.window_us),
                  [&] { return int(B.queue.size()) >= want; });
    const size_t n = std::min<size_t>(B.queue.size(), kMaxBatch);
    std::vector<ibfe_batcher::Pending*> take(B.queue.begin(), B.queue.begin() + n);
    B.queue.erase(B.queue.begin(), B.queue.begin() + n);
    lk.unlock();
    const int rc = launch_cheb_batch(B, take);
    lk.lock();
    for (auto* p : take) {
      p->rc = rc;
      p->launched = true;
    }
    B.batches += 1;
    B.jobs += int64_t(n);
    B.widest = std::max(B.widest, int32_t(n));
    B.leading = false;
    B.cv.notify_all();
  }
  lk.unlock();
  if (me.rc) return me.rc;
  HIP_TRY(hipStreamWaitEvent(c.stream, c.ev_done, 0));
  return IBFE_OK;
}

// -------------------------------------------------------------------------
// one time step
// -------------------------------------------------------------------------

int build_s1(ibfe_ctx& c) {
  const Plan& P = c.plan;
  const double rdt = P.params.rho / P.params.dt, mu = P.params.mu;
  double cm[4];
  for (int t = 0; t < 4; ++t) cm[t] = rdt * c.fc.m[t] + mu * c.fc.k[t];
  klaunch<k_s1_build>(c, dim3(blocks_for(c.nchunks)), dim3(kBlock), 0, c.stream, c.nl, c.emask, c.flags, c.u, c.stride, int(P.sy), int(P.sz), P.h, cm[0], cm[1],
                     cm[2], cm[3], P.params.rho, c.coef64, c.coef32, 1, kFlagP);
  CHECK_LAUNCH();
  return IBFE_OK;
}

// Tentative velocity with explicit advection (uniform grid): the stencil of
// rho C(u^n) alone, the right-hand side (rho/dt) M u^n - rho C(u^n) u^n - G p^n
// - A' g, and CG on the symmetric A' = (rho/dt) M + mu K over the free rows.
// Leaves the free part of u* in w[9].
int s1_explicit(ibfe_ctx& c) {
  const Plan& P = c.plan;
  const double rho = P.params.rho, dt = P.params.dt, mu = P.params.mu, rdt = rho / dt;
  const int nb = blocks_for(c.nchunks);
  const int64_t S = c.stride;
  double* b1 = c.w[8];
  double* x1 = c.w[9];
  klaunch<k_s1_build>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.emask, c.flags,
                     c.u, S, int(P.sy), int(P.sz), P.h, 0.0, 0.0, 0.0, 0.0, rho, c.coef64, (float*)nullptr, 1,
                     kFlagP);
  double cm[4], ca[4];
  for (int t = 0; t < 4; ++t) {
    cm[t] = rdt * c.fc.m[t];
    ca[t] = rdt * c.fc.m[t] + mu * c.fc.k[t];
  }
  klaunch<k_s1_rhs_explicit>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.emask,
                     c.flags, c.coef64, c.u, c.p, c.g, b1, S, int(P.sy), int(P.sz), cm[0], cm[1], cm[2], cm[3],
                     ca[0], ca[1], ca[2], ca[3], c.fc.g2[0], c.fc.g2[1], c.fc.g2[2]);
  if (P.params.viscous == 1 && c.nlift > 0)
    klaunch<k_strain_lift>(c, dim3(blocks_lin(c.nlift)), dim3(kBlock), 0, c.stream, c.nlift,
                       (const int32_t*)c.lift_rows, (const uint8_t*)c.emask, (const double*)c.g, b1, S, mu, P.h,
                       int(P.sy), int(P.sz));
  klaunch<(k_masked_copy<double, double>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl,
                     c.flags, kFlagF, c.u, x1, 3, S);
  CHECK_LAUNCH();
  SolveOut so;
  const int maxit = P.params.max_iters;
  auto solve = [&](const auto& op, const auto& op32) -> int {
    if (P.params.precision == 1) {
      float* const* v = c.v32;
      return run_refined(c, op, kFlagF, 3, b1, x1, v[8], v[9], P.params.rtol, so,
                         [&](const float* r32, float* d32, double tol, SolveOut& o) {
                           return run_cg<float>(c, op32, c.nl, r32, d32, v[0], v[1], v[2], kScS1, tol,
                                                maxit, true, o);
                         });
    }
    return run_cg<double>(c, op, c.nl, b1, x1, c.w[0], c.w[1], c.w[2], kScS1, P.params.rtol, maxit, false,
                          so);
  };
  int rc;
  if (P.params.viscous == 1) {
    auto strain = [&](auto base) {
      using T = std::remove_reference_t<decltype(base.c[0])>;
      OpSymStrain<T> o{};
      o.base = base;
      o.emask = c.emask;
      o.mu = T(mu);
      o.h = T(P.h);
      o.stride = c.stride;
      return o;
    };
    rc = solve(strain(sym_op<double, 3>(c, ca, kFlagF)), strain(sym_op<float, 3>(c, ca, kFlagF)));
  } else {
    rc = solve(sym_op<double, 3>(c, ca, kFlagF), sym_op<float, 3>(c, ca, kFlagF));
  }
  if (rc) return rc;
  c.stats.s1_iters = so.iters;
  c.stats.s1_res = so.res;
  c.stats.s1_outer = so.outer;
  c.stats.s1_restarts = so.restarts;
  return IBFE_OK;
}

int remove_slot_means(ibfe_ctx& c, double* x) {
  const Plan& P = c.plan;
  const int nr = red_blocks(c.nchunks);
  klaunch<k_slot_sum>(c, dim3(nr), dim3(kBlock), 0, c.stream, c.nl, c.slot,
                     (const double*)x, c.partials);
  klaunch<k_fin_slot>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr,
                     P.n_floating, (const double*)c.float_count, c.float_means);
  klaunch<k_slot_sub>(c, dim3(blocks_for(c.nchunks)), dim3(kBlock), 0, c.stream, c.nl,
                     c.slot, x, (const double*)c.float_means);
  CHECK_LAUNCH();
  return IBFE_OK;
}

int step_once(ibfe_ctx& c) {
  const Plan& P = c.plan;
  const double rho = P.params.rho, dt = P.params.dt;
  const double t1 = c.t + dt;
  const int nb = blocks_for(c.nchunks);
  const int sy = int(P.sy), sz = int(P.sz);
  const int64_t S = c.stride;
  const bool mixed = P.params.precision == 1;
  const double rtol = P.params.rtol;
  const int maxit = P.params.max_iters;
  int rc;

  // Dirichlet data g(t^{n+1}) at the inlet table nodes (zero elsewhere)
  if (!P.inlet_ids.empty()) {
    Harmonics hm{};
    hm.K = P.K;
    for (int k = 1; k <= P.K; ++k) {
      hm.c[k - 1] = std::cos(k * P.omega * t1);
      hm.s[k - 1] = std::sin(k * P.omega * t1);
    }
    klaunch<k_inlet>(c, dim3(blocks_lin(int64_t(P.inlet_ids.size()))), dim3(kBlock), 0,
                       c.stream, int(P.inlet_ids.size()), c.inlet_ids, c.inlet_shape, hm, c.g, S);
    CHECK_LAUNCH();
  }

  // 1. tentative velocity: A_FF u*_F = (rho/dt) M u^n - G p^n - A_FD g
  double* b1 = c.w[8];
  double* x1 = c.w[9];
  if (P.params.advection == 1) {
    if ((rc = s1_explicit(c))) return rc;
  } else {
    const bool mf = P.params.advdiff == 0;
    if ((rc = mf ? prep_s1_mf(c, P.params.precision == 1) : build_s1(c))) return rc;
    double cm[4];
    for (int t = 0; t < 4; ++t) cm[t] = rho / dt * c.fc.m[t];
    klaunch<k_s1_rhs>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.emask,
                       c.flags, c.u, c.p, b1, S, sy, sz, cm[0], cm[1], cm[2], cm[3],
                       c.fc.g2[0], c.fc.g2[1], c.fc.g2[2]);
    if (c.nlift > 0 && mf)
      klaunch<(k_lift_rows<OpConv<double>>)>(c, dim3(blocks_lin(c.nlift)), dim3(kBlock), 0, c.stream, c.nlift,
                                              (const int32_t*)c.lift_rows, conv_op<double>(c, kFlagF),
                                              (const double*)c.g, b1);
    else if (c.nlift > 0)
      klaunch<k_s1_lift>(c, dim3(blocks_lin(c.nlift)), dim3(kBlock), 0, c.stream, c.nlift,
                         (const int32_t*)c.lift_rows, (const uint8_t*)c.flags, (const double*)c.coef64,
                         (const double*)c.g, b1, S, sy, sz);
    CHECK_LAUNCH();
    if (P.params.viscous == 1 && c.nlift > 0) {
      klaunch<k_strain_lift>(c, dim3(blocks_lin(c.nlift)), dim3(kBlock), 0, c.stream, c.nlift,
                         (const int32_t*)c.lift_rows, (const uint8_t*)c.emask, (const double*)c.g, b1, S,
                         P.params.mu, P.h, sy, sz);
      CHECK_LAUNCH();
    }
    klaunch<(k_masked_copy<double, double>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.flags, kFlagF, c.u, x1, 3, S);
    CHECK_LAUNCH();
    SolveOut so;
    auto solve = [&](const auto& op, const auto& op32) -> int {
      if (mixed)
        return run_refined(c, op, kFlagF, 3, b1, x1, c.v32[8], c.v32[9], rtol, so,
                           [&](const float* r32, float* d32, double tol, SolveOut& o) {
                             klaunch<k_zero<float>>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, d32, 3,
                                                S);
                             return run_bicgstab<float>(c, op32, r32, d32, c.v32, kScS1, tol, maxit, o, true);
                           });
      return run_bicgstab<double>(c, op, b1, x1, c.w, kScS1, rtol, maxit, so);
    };
    if (P.params.viscous == 1 && mf)
      rc = solve(conv_strain_op<double>(c, kFlagF), conv_strain_op<float>(c, kFlagF));
    else if (P.params.viscous == 1)
      rc = solve(strain_op<double>(c, c.coef64, kFlagF), strain_op<float>(c, c.coef32, kFlagF));
    else if (mf)
      rc = solve(conv_op<double>(c, kFlagF), conv_op<float>(c, kFlagF));
    else
      rc = solve(stencil_op<double>(c, c.coef64, kFlagF), stencil_op<float>(c, c.coef32, kFlagF));
    if (rc) return rc;
    c.stats.s1_iters = so.iters;
    c.stats.s1_res = so.res;
    c.stats.s1_outer = so.outer;
    c.stats.s1_restarts = so.restarts;
  }
  klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, x1, 1.0, c.g,
                     c.ustar, 3, S);
  CHECK_LAUNCH();

  // 2.-4. BCE-IB correction: G Lambda = U_B - I u*, u_ib = u* + I_F^T Lambda (FP64)
  klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, c.ustar,
                     0.0, c.ustar, c.uib, 3, S);
  CHECK_LAUNCH();
  c.stats.ib_iters = 0;
  c.stats.ib_res = 0.0;
  if (P.M > 0) {
    const int M = int(P.M);
    klaunch<k_ib_interp>(c, dim3(blocks_lin(int64_t(M) * 8)), dim3(kBlock), 0, c.stream, M, c.ib_idx, c.ib_w,
                       c.UB, c.ustar, S, c.ibv[0], c.mstride, 1);
    CHECK_LAUNCH();
    const bool warm = c.lam_warm;
    SolveOut so;
    c.lam_warm = false;
    if ((rc = run_ib_pcg(c, c.ibv[0], c.ibv[1], c.ibv[2], c.ibv[3], c.ibv[6], c.ibv[4], c.ibv[5], kScIB,
                         P.params.ib_rtol, maxit, !warm, so)))
      return rc;
    c.lam_warm = true;
    c.stats.ib_iters = so.iters;
    c.stats.ib_res = so.res;
    const int nn = c.n_sp;
    klaunch<k_ib_spread>(c, dim3(blocks_lin(nn)), dim3(kBlock), 0, c.stream, nn, c.sp_node,
                       c.sp_ptr, c.sp_pt, c.sp_wt, c.ibv[1], c.mstride, c.uib, S);
    CHECK_LAUNCH();
  }

  // 5. pressure increment: K_{P'P'} Phi = -(rho/dt) (B u_ib)_{P'}
  double* b3 = c.w[8];
  {
    klaunch<k_div>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.emask, c.flags,
                       kFlagPp, 0u, c.uib, b3, S, sy, sz, c.fc.g2[0], c.fc.g2[1], c.fc.g2[2], -rho / dt);
    CHECK_LAUNCH();
    if (P.n_floating > 0 && (rc = remove_slot_means(c, b3))) return rc;
    const double kc[4] = {c.fc.k[0], c.fc.k[1], c.fc.k[2], c.fc.k[3]};
    auto op = sym_op<double, 1>(c, kc, kFlagPp);
    SolveOut so;
    const bool mg = P.params.precond >= 1;  // multigrid or Chebyshev (one level)
    if (mixed) {
      auto op32 = sym_op<float, 1>(c, kc, kFlagPp);
      if (!c.phi_warm)
        klaunch<k_zero<double>>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.phi, 1, S);
      c.phi_warm = false;
      float* const* v = c.v32;
      rc = run_refined(c, op, kFlagPp, 1, b3, c.phi, v[8], v[9], rtol, so,
                       [&](const float* r32, float* d32, double tol, SolveOut& o) {
                         if (mg)
                           return run_pcg_mg<float>(c, op32, c.mg32, r32, d32, v[0], v[1], v[2], v[3], kScS3,
                                                    tol, maxit, o);
                         return run_cg<float>(c, op32, c.nl, r32, d32, v[0], v[1], v[2], kScS3,
                                              tol, maxit, true, o);
                       });
    } else if (mg) {
      rc = run_pcg_mg<double>(c, op, c.mg64, b3, c.phi, c.w[0], c.w[1], c.w[2], c.w[3], kScS3, rtol, maxit,
                              so);
    } else {
      rc = run_cg<double>(c, op, c.nl, b3, c.phi, c.w[0], c.w[1], c.w[2], kScS3, rtol, maxit,
                          true, so);
    }
    if (rc) return rc;
    c.stats.s3_iters = so.iters;
    c.stats.s3_res = so.res;
    c.stats.s3_outer = so.outer;
    if (P.n_floating > 0 && (rc = remove_slot_means(c, c.phi))) return rc;
    c.phi_warm = mixed;
  }

  // 6. correction: M_FF delta = (G Phi)_F, u^{n+1} = u_ib - (dt/rho) delta, p^{n+1} = p^n + Phi
  {
    const bool tensor = P.params.mass_precond == 1;
    double* b4 = c.w[8];
    double* delta = c.delta;
    klaunch<k_grad>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.emask, c.flags,
                       kFlagF, c.phi, b4, S, sy, sz, c.fc.g2[0], c.fc.g2[1], c.fc.g2[2]);
    CHECK_LAUNCH();
    const double mc[4] = {c.fc.m[0], c.fc.m[1], c.fc.m[2], c.fc.m[3]};
    auto op = sym_op<double, 3>(c, mc, kFlagF);
    SolveOut so;
    if (!c.delta_warm) klaunch<k_zero<double>>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, delta, 3, S);
    c.delta_warm = false;
    if (mixed) {
      float* const* v = c.v32;
      // the residual and the Chebyshev direction in walk order
      rc = run_refined(c, op, kFlagF, 3, b4, delta, c.rim, v[9], rtol, so,
                       [&](const float* r32, float* d32, double tol, SolveOut& o) {
                         if (tensor) {
                           o.iters = cheb_steps(tol, kTmLmin, kTmLmax);
                           return run_cheb_tm<float, 3, true>(c, mass_zop<float>(c), r32, d32, c.dim, o.iters,
                                                              [](float*) { return int(IBFE_OK); });
                         }
                         o.iters = mass_cheb_steps(tol);
                         if (c.batcher) return batched_cheb_mass(c, r32, d32, v[0], c.dim, o.iters);
                         return run_cheb_mass<float, true>(c, r32, d32, v[0], c.dim, o.iters);
                       }, true, tensor ? kTmInnerRtol : kInnerRtol);
    } else {
      // FP64: refinement sweeps whose corrections are FP64 Chebyshev solves
      double* r64 = c.w[3];
      so.iters = 0;
      so.outer = 0;
      for (int sweep = 0;; ++sweep) {
        double rr = 0, bb = 0;
        if ((rc = ir_residual(c, op, b4, delta, r64, rr, bb))) return rc;
        so.res = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        if (so.res <= rtol || sweep == 4) break;
        const double tol_in = std::max(rtol / std::max(so.res, 1e-300), 1e-15);
        const int it = tensor ? cheb_steps(tol_in, kTmLmin, kTmLmax) : mass_cheb_steps(tol_in);
        if (tensor)
          rc = run_cheb_tm<double, 3, false>(c, mass_zop<double>(c), (const double*)r64, c.w[0], c.w[2], it,
                                             [](double*) { return int(IBFE_OK); });
        else
          rc = run_cheb_mass<double>(c, (const double*)r64, c.w[0], c.w[1], c.w[2], it);
        if (rc) return rc;
        klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, delta, 1.0,
                           c.w[0], delta, 3, S);
        CHECK_LAUNCH();
        so.iters += it;
        so.outer += 1;
      }
      rc = so.res <= rtol ? IBFE_OK : fail(IBFE_ENOCONV, "mass correction did not converge");
    }
    if (rc) return rc;
    c.stats.s4_iters = so.iters;
    c.stats.s4_res = so.res;
    c.stats.s4_outer = so.outer;
    c.delta_warm = true;
    klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, c.uib,
                       -dt / rho, delta, c.u_next, 3, S);
    klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, c.p, 1.0,
                       c.phi, c.p_next, 1, S);
    CHECK_LAUNCH();
  }
  std::swap(c.u, c.u_next);
  std::swap(c.p, c.p_next);
  c.t = t1;
  c.steps += 1;
  c.stats.steps = c.steps;
  c.stats.t = c.t;
  return c.timing ? collect_kernel_times(c) : IBFE_OK;
}

// Tentative-velocity stencil of the composite mesh: fine-element part (rows of
// P and hanging nodes) into planes 0..26, coarse-element part into 27..53.
int build_s1_refined(ibfe_ctx& c) {
  const Plan& P = c.plan;
  const double rdt = P.params.rho / P.params.dt, mu = P.params.mu;
  double cf[4], cc[4];
  for (int t = 0; t < 4; ++t) {
    cf[t] = rdt * c.fc.m[t] + mu * c.fc.k[t];
    cc[t] = rdt * c.fcc.m[t] + mu * c.fcc.k[t];
  }
  const int nb = blocks_for(c.nchunks);
  const int64_t S = c.stride;
  klaunch<k_s1_build>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.emask, c.flags,
                     c.u, S, int(P.sy), int(P.sz), P.h, cf[0], cf[1], cf[2], cf[3], P.params.rho, c.coef64,
                     c.coef32, 1, kFlagP | kFlagHang);
  klaunch<k_s1_build>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.cmask, c.flags,
                     c.u, S, int(P.sy), int(P.sz), P.hb, cc[0], cc[1], cc[2], cc[3], P.params.rho,
                     c.coef64 + 27 * S, c.coef32 ? c.coef32 + 27 * S : nullptr, 2, kFlagP);
  CHECK_LAUNCH();
  return IBFE_OK;
}

// Tentative velocity with explicit advection on the composite mesh (see
// s1_explicit); the inputs u, p, g already hold their hanging values.
int s1_explicit_refined(ibfe_ctx& c) {
  const Plan& P = c.plan;
  const double rho = P.params.rho, dt = P.params.dt, mu = P.params.mu, rdt = rho / dt;
  const int nb = blocks_for(c.nchunks);
  const int64_t S = c.stride;
  double* b1 = c.w[8];
  double* x1 = c.w[9];
  klaunch<k_s1_build>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.emask, c.flags,
                     c.u, S, int(P.sy), int(P.sz), P.h, 0.0, 0.0, 0.0, 0.0, rho, c.coef64, (float*)nullptr, 1,
                     kFlagP | kFlagHang);
  klaunch<k_s1_build>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.cmask, c.flags,
                     c.u, S, int(P.sy), int(P.sz), P.hb, 0.0, 0.0, 0.0, 0.0, rho, c.coef64 + 27 * S,
                     (float*)nullptr, 2, kFlagP);
  CHECK_LAUNCH();
  int rc;
  S1RhsExplicitElem f{};
  f.mass = csym_op<double, 3>(c, rdt, 0.0, kFlagF, c.dinvM64);
  f.adv = cstencil_op<double>(c, c.coef64, kFlagF);
  f.aprime = csym_op<double, 3>(c, rdt, mu, kFlagF, c.dinvA64);
  f.grad = grad_elem(c, c.p);
  f.u = c.u;
  f.g = c.g;
  const bool strain = P.params.viscous == 1;
  if (strain) {
    S1RhsStrainElem<S1RhsExplicitElem> fs{};
    fs.base = f;
    fs.emask = c.emask;
    fs.cmask = c.cmask;
    fs.mu = mu;
    fs.hf = P.h;
    fs.hc = P.hb;
    fs.sy = int(P.sy);
    fs.sz = int(P.sz);
    fs.stride = c.stride;
    if ((rc = comp_rows<double>(c, fs, kFlagF, 0u, 1.0, b1))) return rc;
  } else if ((rc = comp_rows<double>(c, f, kFlagF, 0u, 1.0, b1))) {
    return rc;
  }
  klaunch<(k_masked_copy<double, double>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl,
                     c.flags, kFlagF, c.u, x1, 3, S);
  CHECK_LAUNCH();
  SolveOut so;
  const int maxit = P.params.max_iters;
  auto solve = [&](const auto& op, const auto& op32) -> int {
    if (P.params.precision == 1) {
      float* const* v = c.v32;
      return run_refined(c, op, kFlagF, 3, b1, x1, v[8], v[9], P.params.rtol, so,
                         [&](const float* r32, float* d32, double tol, SolveOut& o) {
                           return run_cg<float>(c, op32, c.nl, r32, d32, v[0], v[1], v[2], kScS1, tol,
                                                maxit, true, o);
                         });
    }
    return run_cg<double>(c, op, c.nl, b1, x1, c.w[0], c.w[1], c.w[2], kScS1, P.params.rtol, maxit,
                          false, so);
  };
  auto op = csym_op<double, 3>(c, rdt, mu, kFlagF, c.dinvA64);
  auto op32 = csym_op<float, 3>(c, rdt, mu, kFlagF, c.dinvA32);
  if (strain) {
    auto wrap = [&](const auto& base) {
      using T = std::remove_const_t<std::remove_reference_t<decltype(base.cf[0])>>;
      OpCSymStrain<T> o{};
      o.base = base;
      o.mu = T(mu);
      o.hf = T(P.h);
      o.hc = T(P.hb);
      o.stride = base.stride;
      o.yh = base.yh;
      return o;
    };
    rc = solve(wrap(op), wrap(op32));
  } else {
    rc = solve(op, op32);
  }
  if (rc) return rc;
  c.stats.s1_iters = so.iters;
  c.stats.s1_res = so.res;
  c.stats.s1_outer = so.outer;
  c.stats.s1_restarts = so.restarts;
  return IBFE_OK;
}

int step_once_refined(ibfe_ctx& c) {
  const Plan& P = c.plan;
  const double rho = P.params.rho, dt = P.params.dt;
  const double t1 = c.t + dt;
  const int nb = blocks_for(c.nchunks);
  const int64_t S = c.stride;
  const bool mixed = P.params.precision == 1;
  const double rtol = P.params.rtol;
  const int maxit = P.params.max_iters;
  int rc;

  if (!P.inlet_ids.empty()) {
    Harmonics hm{};
    hm.K = P.K;
    for (int k = 1; k <= P.K; ++k) {
      hm.c[k - 1] = std::cos(k * P.omega * t1);
      hm.s[k - 1] = std::sin(k * P.omega * t1);
    }
    klaunch<k_inlet>(c, dim3(blocks_lin(int64_t(P.inlet_ids.size()))), dim3(kBlock), 0,
                       c.stream, int(P.inlet_ids.size()), c.inlet_ids, c.inlet_shape, hm, c.g, S);
    CHECK_LAUNCH();
  }
  // the element forms read the hanging values C x of u^n, p^n and g
  if ((rc = fill_hanging<double>(c, c.u, 3)) || (rc = fill_hanging<double>(c, c.p, 1)) ||
      (rc = fill_hanging<double>(c, c.g, 3)))
    return rc;

  // 1. tentative velocity
  double* b1 = c.w[8];
  double* x1 = c.w[9];
  if (P.params.advection == 1) {
    if ((rc = s1_explicit_refined(c))) return rc;
  } else {
    const bool mf = P.params.advdiff == 0;
    const bool strain = P.params.viscous == 1;
    // b1 = (rho/dt) M u^n - G p^n - A g (and the strain-rate lifting)
    auto rhs = [&](auto A) -> int {
      S1RhsElemT<decltype(A)> f{};
      f.mass = csym_op<double, 3>(c, rho / dt, 0.0, kFlagF, c.dinvM64);
      f.A = A;
      f.grad = grad_elem(c, c.p);
      f.u = c.u;
      f.g = c.g;
      for (int a = 0; a < 3; ++a) {
        f.lo[a] = c.lift_lo[a];
        f.hi[a] = c.lift_hi[a];
      }
      if (!strain) return comp_rows<double>(c, f, kFlagF, 0u, 1.0, b1);
      S1RhsStrainElem<S1RhsElemT<decltype(A)>> fs{};
      fs.base = f;
      fs.emask = c.emask;
      fs.cmask = c.cmask;
      fs.mu = P.params.mu;
      fs.hf = P.h;
      fs.hc = P.hb;
      fs.sy = int(P.sy);
      fs.sz = int(P.sz);
      fs.stride = c.stride;
      return comp_rows<double>(c, fs, kFlagF, 0u, 1.0, b1);
    };
    if (mf) {
      if ((rc = prep_s1_mf(c, P.params.precision == 1)) || (rc = rhs(cconv_op<double>(c, kFlagF)))) return rc;
    } else {
      if ((rc = build_s1_refined(c)) || (rc = rhs(cstencil_op<double>(c, c.coef64, kFlagF)))) return rc;
    }
    klaunch<(k_masked_copy<double, double>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.flags, kFlagF, c.u, x1, 3, S);
    CHECK_LAUNCH();
    SolveOut so;
    auto solve = [&](const auto& op, const auto& op32) -> int {
      if (mixed)
        return run_refined(c, op, kFlagF, 3, b1, x1, c.v32[8], c.v32[9], rtol, so,
                           [&](const float* r32, float* d32, double tol, SolveOut& o) {
                             klaunch<k_zero<float>>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, d32, 3,
                                                S);
                             return run_bicgstab<float>(c, op32, r32, d32, c.v32, kScS1, tol, maxit, o, true);
                           });
      return run_bicgstab<double>(c, op, b1, x1, c.w, kScS1, rtol, maxit, so);
    };
    if (strain && mf)
      rc = solve(cconv_strain_op<double>(c, kFlagF), cconv_strain_op<float>(c, kFlagF));
    else if (strain)
      rc = solve(cstrain_op<double>(c, c.coef64, kFlagF), cstrain_op<float>(c, c.coef32, kFlagF));
    else if (mf)
      rc = solve(cconv_solver_op<double>(c, kFlagF), cconv_solver_op<float>(c, kFlagF));
    else
      rc = solve(cstencil_op<double>(c, c.coef64, kFlagF), cstencil_op<float>(c, c.coef32, kFlagF));
    if (rc) return rc;
    c.stats.s1_iters = so.iters;
    c.stats.s1_res = so.res;
    c.stats.s1_outer = so.outer;
    c.stats.s1_restarts = so.restarts;
  }
  klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, x1, 1.0, c.g,
                     c.ustar, 3, S);
  CHECK_LAUNCH();

  // 2.-4. BCE-IB correction (every support node is a fine, non-hanging node)
  klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, c.ustar,
                     0.0, c.ustar, c.uib, 3, S);
  CHECK_LAUNCH();
  c.stats.ib_iters = 0;
  c.stats.ib_res = 0.0;
  if (P.M > 0) {
    const int M = int(P.M);
    klaunch<k_ib_interp>(c, dim3(blocks_lin(int64_t(M) * 8)), dim3(kBlock), 0, c.stream, M, c.ib_idx, c.ib_w,
                       c.UB, c.ustar, S, c.ibv[0], c.mstride, 1);
    CHECK_LAUNCH();
    const bool warm = c.lam_warm;
    SolveOut so;
    c.lam_warm = false;
    if ((rc = run_ib_pcg(c, c.ibv[0], c.ibv[1], c.ibv[2], c.ibv[3], c.ibv[6], c.ibv[4], c.ibv[5], kScIB,
                         P.params.ib_rtol, maxit, !warm, so)))
      return rc;
    c.lam_warm = true;
    c.stats.ib_iters = so.iters;
    c.stats.ib_res = so.res;
    const int nn = c.n_sp;
    klaunch<k_ib_spread>(c, dim3(blocks_lin(nn)), dim3(kBlock), 0, c.stream, nn, c.sp_node,
                       c.sp_ptr, c.sp_pt, c.sp_wt, c.ibv[1], c.mstride, c.uib, S);
    CHECK_LAUNCH();
  }

  // 5. pressure increment
  double* b3 = c.w[8];
  {
    if ((rc = fill_hanging<double>(c, c.uib, 3))) return rc;
    DivElem f{};
    f.emask = c.emask;
    f.cmask = c.cmask;
    f.u = c.uib;
    f.stride = S;
    f.sy = int(P.sy);
    f.sz = int(P.sz);
    for (int k = 0; k < 3; ++k) {
      f.gf[k] = c.fc.g2[k];
      f.gc[k] = c.fcc.g2[k];
    }
    if ((rc = comp_rows<double>(c, f, kFlagPp, 0u, -rho / dt, b3))) return rc;
    if (P.n_floating > 0 && (rc = remove_slot_means(c, b3))) return rc;
    auto op = csym_op<double, 1>(c, 0.0, 1.0, kFlagPp, c.dinvK64);
    const bool mg = P.params.precond >= 1;  // multigrid or Chebyshev (one level)
    SolveOut so;
    if (mixed) {
      auto op32 = csym_op<float, 1>(c, 0.0, 1.0, kFlagPp, c.dinvK32);
      if (!c.phi_warm)
        klaunch<k_zero<double>>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, c.phi, 1, S);
      c.phi_warm = false;
      float* const* v = c.v32;
      rc = run_refined(c, op, kFlagPp, 1, b3, c.phi, v[8], v[9], rtol, so,
                       [&](const float* r32, float* d32, double tol, SolveOut& o) {
                         if (mg)
                           return run_pcg_mg<float>(c, op32, c.mg32, r32, d32, v[0], v[1], v[2], v[3], kScS3,
                                                    tol, maxit, o);
                         return run_cg<float>(c, op32, c.nl, r32, d32, v[0], v[1], v[2], kScS3,
                                              tol, maxit, true, o);
                       });
    } else if (mg) {
      rc = run_pcg_mg<double>(c, op, c.mg64, b3, c.phi, c.w[0], c.w[1], c.w[2], c.w[3], kScS3, rtol, maxit,
                              so);
    } else {
      rc = run_cg<double>(c, op, c.nl, b3, c.phi, c.w[0], c.w[1], c.w[2], kScS3, rtol, maxit,
                          true, so);
    }
    if (rc) return rc;
    c.stats.s3_iters = so.iters;
    c.stats.s3_res = so.res;
    c.stats.s3_outer = so.outer;
    if (P.n_floating > 0 && (rc = remove_slot_means(c, c.phi))) return rc;
    c.phi_warm = mixed;
  }

  // 6. correction: M_FF delta = (G Phi)_F with Chebyshev on [lmin, 27/8] of D'^-1 M
  // (mass_precond = 0) or on [kTmLmin, kTmLmax] of P M (mass_precond = 1)
  {
    const bool tensor = P.params.mass_precond == 1;
    double* b4 = c.w[8];
    double* delta = c.delta;
    if ((rc = fill_hanging<double>(c, c.phi, 1))) return rc;
    if ((rc = comp_rows<double>(c, grad_elem(c, c.phi), kFlagF, 0u, 1.0, b4))) return rc;
    auto op = csym_op<double, 3>(c, 1.0, 0.0, kFlagF, c.dinvM64);
    const double lmin = c.mass_lmin, lmax = kMassLmax;
    SolveOut so;
    if (!c.delta_warm) klaunch<k_zero<double>>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, delta, 3, S);
    c.delta_warm = false;
    if (mixed) {
      auto op32 = csym_op<float, 3>(c, 1.0, 0.0, kFlagF, c.dinvM32);
      float* const* v = c.v32;
      // the residual and the Chebyshev direction in walk order
      rc = run_refined(c, op, kFlagF, 3, b4, delta, c.rim, v[9], rtol, so,
                       [&](const float* r32, float* d32, double tol, SolveOut& o) {
                         if (tensor) {
                           o.iters = cheb_steps(tol, kTmLmin, kTmLmax);
                           return run_cheb_tm<float, 3, true>(c, zcomp_op(c, op32), r32, d32, c.dim, o.iters,
                                                              [&](float* x) {
                                                                int rp = pre_apply(c, op32, x, (const KScal*)nullptr);
                                                                if (!rp) launch_extra<float, 3>(c, op32, x, nullptr);
                                                                return rp;
                                                              });
                         }
                         o.iters = cheb_steps(tol, lmin, lmax);
                         return run_cheb_gen<float, decltype(op32), true>(c, op32, r32, d32, v[0], c.dim, o.iters,
                                                                          lmin, lmax);
                       }, true, tensor ? kTmInnerRtol : kInnerRtol);
    } else {
      double* r64 = c.w[3];
      so.iters = 0;
      so.outer = 0;
      for (int sweep = 0;; ++sweep) {
        double rr = 0, bb = 0;
        if ((rc = ir_residual(c, op, b4, delta, r64, rr, bb))) return rc;
        so.res = bb > 0.0 ? std::sqrt(rr / bb) : 0.0;
        if (so.res <= rtol || sweep == 4) break;
        const double tol_in = std::max(rtol / std::max(so.res, 1e-300), 1e-15);
        const int it = tensor ? cheb_steps(tol_in, kTmLmin, kTmLmax) : cheb_steps(tol_in, lmin, lmax);
        if (tensor)
          rc = run_cheb_tm<double, 3, false>(c, zcomp_op(c, op), (const double*)r64, c.w[0], c.w[2], it,
                                             [&](double* x) {
                                               int rp = pre_apply(c, op, x, (const KScal*)nullptr);
                                               if (!rp) launch_extra<double, 3>(c, op, x, nullptr);
                                               return rp;
                                             });
        else
          rc = run_cheb_gen<double>(c, op, (const double*)r64, c.w[0], c.w[1], c.w[2], it, lmin, lmax);
        if (rc) return rc;
        klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, delta, 1.0,
                           c.w[0], delta, 3, S);
        CHECK_LAUNCH();
        so.iters += it;
        so.outer += 1;
      }
      rc = so.res <= rtol ? IBFE_OK : fail(IBFE_ENOCONV, "mass correction did not converge");
    }
    if (rc) return rc;
    c.stats.s4_iters = so.iters;
    c.stats.s4_res = so.res;
    c.stats.s4_outer = so.outer;
    c.delta_warm = true;
    klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, c.uib,
                       -dt / rho, delta, c.u_next, 3, S);
    klaunch<k_axpby>(c, dim3(nb), dim3(kBlock), 0, c.stream, c.nl, 1.0, c.p, 1.0,
                       c.phi, c.p_next, 1, S);
    CHECK_LAUNCH();
  }
  std::swap(c.u, c.u_next);
  std::swap(c.p, c.p_next);
  c.t = t1;
  c.steps += 1;
  c.stats.steps = c.steps;
  c.stats.t = c.t;
  return c.timing ? collect_kernel_times(c) : IBFE_OK;
}

// FP32 work vectors for the verification applies of an FP64-mode context
// (allocated on first use).
int ensure_fp32_work(ibfe_ctx& C) {
  int rc;
  if (!C.v32[0])
    for (int i = 0; i < 10; ++i)
      if ((rc = C.field(&C.v32[i], 3))) return rc;
  return IBFE_OK;
}

// Verification applies on a refined lattice: rows and columns on all of P,
// C^T A C with the hanging-node constraint.
int apply_refined(ibfe_ctx& C, int op, int precision, double* xin, double* yout, int& nc_out) {
  const Plan& P = C.plan;
  const int nb = blocks_for(C.nchunks);
  const int64_t S = C.stride;
  int rc;
  switch (op) {
    case IBFE_OP_MASS:
    case IBFE_OP_STIFF: {
      const double a = op == IBFE_OP_MASS ? 1.0 : 0.0, b = 1.0 - a;
      nc_out = 1;
      if (precision == 0) {
        if ((rc = fill_hanging<double>(C, xin, 1))) return rc;
        auto o = csym_op<double, 1>(C, a, b, kFlagP, C.dinvM64);
        return comp_rows<double>(C, OpElem<double, OpCSym<double, 1>>{o, xin}, kFlagP, 0u, 1.0, yout);
      }
      if ((rc = ensure_fp32_work(C))) return rc;
      float* x32 = C.v32[0];
      float* y32 = C.v32[1];
      klaunch<(k_masked_copy<double, float>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, xin, x32, 1, S);
      CHECK_LAUNCH();
      if ((rc = fill_hanging<float>(C, x32, 1))) return rc;
      auto o = csym_op<float, 1>(C, a, b, kFlagP, C.dinvM32);
      if ((rc = comp_rows<float>(C, OpElem<float, OpCSym<float, 1>>{o, x32}, kFlagP, 0u, 1.0f, y32))) return rc;
      klaunch<(k_masked_copy<float, double>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, y32, yout, 1, S);
      CHECK_LAUNCH();
      return IBFE_OK;
    }
    case IBFE_OP_GRAD:
      nc_out = 3;
      if ((rc = fill_hanging<double>(C, xin, 1))) return rc;
      return comp_rows<double>(C, grad_elem(C, xin), kFlagP, 0u, 1.0, yout);
    case IBFE_OP_DIV: {
      nc_out = 1;
      if ((rc = fill_hanging<double>(C, xin, 3))) return rc;
      DivElem f{};
      f.emask = C.emask;
      f.cmask = C.cmask;
      f.u = xin;
      f.stride = S;
      f.sy = int(P.sy);
      f.sz = int(P.sz);
      for (int k = 0; k < 3; ++k) {
        f.gf[k] = C.fc.g2[k];
        f.gc[k] = C.fcc.g2[k];
      }
      return comp_rows<double>(C, f, kFlagP, 0u, 1.0, yout);
    }
    case IBFE_OP_ADVDIFF: {
      nc_out = 3;
      if (!C.coef64) {
        // matrix-free context
        if (precision == 1 && !C.w32) {
          if ((rc = C.field(&C.w32, 3)) || (rc = C.field(&C.dinvS32, 1))) return rc;
          if ((rc = ensure_fp32_work(C))) return rc;
        }
        if ((rc = fill_hanging<double>(C, C.u, 3))) return rc;
        if ((rc = prep_s1_mf(C, precision == 1 || P.params.precision == 1))) return rc;
        const bool strain = P.params.viscous == 1;
        if (precision == 0) {
          if ((rc = fill_hanging<double>(C, xin, 3))) return rc;
          if (strain)
            return comp_rows<double>(C, OpElem<double, OpCStencilStrain<double, OpCConv<double>>>{
                                            cconv_strain_op<double>(C, kFlagP), xin},
                                     kFlagP, 0u, 1.0, yout);
          return comp_rows<double>(C, OpElem<double, OpCConv<double>>{cconv_op<double>(C, kFlagP), xin}, kFlagP,
                                   0u, 1.0, yout);
        }
        float* x32 = C.v32[0];
        float* y32 = C.v32[1];
        klaunch<(k_masked_copy<double, float>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, xin, x32, 3, S);
        CHECK_LAUNCH();
        if ((rc = fill_hanging<float>(C, x32, 3))) return rc;
        if (strain)
          rc = comp_rows<float>(C, OpElem<float, OpCStencilStrain<float, OpCConv<float>>>{
                                       cconv_strain_op<float>(C, kFlagP), x32},
                                kFlagP, 0u, 1.0f, y32);
        else
          rc = comp_rows<float>(C, OpElem<float, OpCConv<float>>{cconv_op<float>(C, kFlagP), x32}, kFlagP, 0u,
                                1.0f, y32);
        if (rc) return rc;
        klaunch<(k_masked_copy<float, double>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, y32, yout, 3, S);
        CHECK_LAUNCH();
        return IBFE_OK;
      }
      if (precision == 1 && !C.coef32) {
        if ((rc = C.field(&C.coef32, 54))) return rc;
        if ((rc = ensure_fp32_work(C))) return rc;
      }
      if ((rc = fill_hanging<double>(C, C.u, 3))) return rc;
      if ((rc = build_s1_refined(C))) return rc;
      if (precision == 0) {
        if ((rc = fill_hanging<double>(C, xin, 3))) return rc;
        if (P.params.viscous == 1)
          return comp_rows<double>(C, OpElem<double, OpCStencilStrain<double>>{cstrain_op<double>(C, C.coef64, kFlagP), xin},
                                   kFlagP, 0u, 1.0, yout);
        auto o = cstencil_op<double>(C, C.coef64, kFlagP);
        return comp_rows<double>(C, OpElem<double, OpCStencil<double, 3>>{o, xin}, kFlagP, 0u, 1.0, yout);
      }
      float* x32 = C.v32[0];
      float* y32 = C.v32[1];
      klaunch<(k_masked_copy<double, float>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, xin, x32, 3, S);
      CHECK_LAUNCH();
      if ((rc = fill_hanging<float>(C, x32, 3))) return rc;
      if (P.params.viscous == 1)
        rc = comp_rows<float>(C, OpElem<float, OpCStencilStrain<float>>{cstrain_op<float>(C, C.coef32, kFlagP), x32},
                              kFlagP, 0u, 1.0f, y32);
      else
        rc = comp_rows<float>(C, OpElem<float, OpCStencil<float, 3>>{cstencil_op<float>(C, C.coef32, kFlagP), x32},
                              kFlagP, 0u, 1.0f, y32);
      if (rc) return rc;
      klaunch<(k_masked_copy<float, double>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, y32, yout, 3, S);
      CHECK_LAUNCH();
      return IBFE_OK;
    }
    default: return fail(IBFE_EINVAL, "unknown operator");
  }
}

// Smallest eigenvalue of D'^-1 C^T M C on the free rows of a refined lattice, by
// Lanczos: preconditioned CG on the FP64 composite mass from a pseudo-random
// right-hand side; its step lengths alpha_j and ratios beta_j give the Lanczos
// tridiagonal of the Jacobi-scaled operator (diagonal 1/alpha_j +
// beta_{j-1}/alpha_{j-1}, off-diagonal sqrt(beta_j)/alpha_j), whose smallest
// eigenvalue (bisection on the Sturm sequence) is a Ritz value and so lies
// above the true one.  The mass correction's Chebyshev interval starts at 0.9 of
// it, never below the proven bound (1/8) min a_nn / D'(n): error components
// below the interval are reduced less but not amplified, and the FP64
// refinement measures the true residual.
int estimate_mass_lmin(ibfe_ctx& c) {
  const Plan& P = c.plan;
  c.mass_lmin = P.mass_lmin;
  if (!P.refined || P.n_free == 0) return IBFE_OK;
  constexpr int kLanczos = 40;
  auto op = csym_op<double, 1>(c, 1.0, 0.0, kFlagF, c.dinvM64);
  double *b = c.w[0], *x = c.w[1], *r = c.w[2], *p = c.w[3], *q = c.w[4];
  const NodeList nl = c.nl;
  const int nb = blocks_for(nl.n), nr = red_blocks(nl.n);
  KScal* sc = &c.scal[kScMisc];
  klaunch<k_fill_hash>(c, dim3(nb), dim3(kBlock), 0, c.stream, nl, (const uint8_t*)c.flags, kFlagF, b);
  klaunch<(k_cg_init<double, decltype(op)>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, (const double*)b, x,
                                              r, p, c.partials, 1);
  klaunch<k_fin_cg_init>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr, sc, 0.0,
                         kLanczos);
  CHECK_LAUNCH();
  std::vector<double> alpha, beta;
  for (int j = 0; j < kLanczos; ++j) {
    int rc;
    if ((rc = pre_apply(c, op, p, (const KScal*)sc))) return rc;
    const int nq = launch_q<double>(c, op, nl, p, q, (const KScal*)sc);
    klaunch<k_fin_cg_q>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nq, sc);
    klaunch<(k_cg_xr<double, decltype(op)>)>(c, dim3(nr), dim3(kBlock), 0, c.stream, nl, op, x, r,
                                             (const double*)p, (const double*)q, c.partials, (const KScal*)sc);
    klaunch<k_fin_cg_xr>(c, dim3(1), dim3(kBlock), 0, c.stream, (const double*)c.partials, nr, sc);
    klaunch<(k_cg_p<double, decltype(op)>)>(c, dim3(nb), dim3(kBlock), 0, c.stream, nl, op, (const double*)r, p,
                                            (const KScal*)sc);
    CHECK_LAUNCH();
    KScal s{};
    if ((rc = poll(c, kScMisc, s))) return rc;
    if (s.status != 0 || !(s.alpha > 0.0) || !std::isfinite(s.beta)) break;
    alpha.push_back(s.alpha);
    beta.push_back(s.beta);
    if (s.done) break;
  }
  const int k = int(alpha.size());
  if (k < 8) return IBFE_OK;  // too few steps for an estimate: keep the bound
  std::vector<double> d(k), e(k, 0.0);
  for (int j = 0; j < k; ++j) {
    d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < k) e[j] = std::sqrt(beta[j]) / alpha[j];
  }
  // number of eigenvalues of the tridiagonal below s (Sturm sequence)
  auto below = [&](double s) {
    int cnt = 0;
    double qv = 1.0;
    for (int j = 0; j < k; ++j) {
      qv = d[j] - s - (j > 0 ? e[j - 1] * e[j - 1] / qv : 0.0);
      if (qv == 0.0) qv = -1e-300;
      if (qv < 0.0) ++cnt;
    }
    return cnt;
  };
  double lo = 0.0, hi = kMassLmax * 2.0;
  for (int it = 0; it < 100; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (below(mid) >= 1) hi = mid;
    else lo = mid;
  }
  const double ritz = 0.5 * (lo + hi);
  if (ritz > 0.0 && ritz < 1.0) c.mass_lmin = std::max(P.mass_lmin, 0.9 * ritz);
  return IBFE_OK;
}

int copy_in(ibfe_ctx& c, double* dense, int nc, const double* src, int on_device) {
  const int64_t n = c.nP;
  const double* comp = src;
  if (!on_device) {
    HIP_TRY(hipMemcpyAsync(c.compact, src, sizeof(double) * nc * n, hipMemcpyHostToDevice, c.stream));
    comp = c.compact;
  }
  HIP_TRY(hipMemsetAsync(dense - c.halo, 0, sizeof(double) * c.stride * nc, c.stream));
  klaunch<k_scatter>(c, dim3(blocks_lin(n)), dim3(kBlock), 0, c.stream, n, c.pids, comp, dense, nc,
                     c.stride);
  CHECK_LAUNCH();
  if (!on_device) HIP_TRY(hipStreamSynchronize(c.stream));
  return IBFE_OK;
}

int copy_out(ibfe_ctx& c, const double* dense, int nc, double* dst, int on_device) {
  const int64_t n = c.nP;
  double* comp = on_device ? dst : c.compact;
  klaunch<k_gather>(c, dim3(blocks_lin(n)), dim3(kBlock), 0, c.stream, n, c.pids, dense, comp, nc,
                     c.stride);
  CHECK_LAUNCH();
  if (!on_device) {
    HIP_TRY(hipMemcpyAsync(dst, c.compact, sizeof(double) * nc * n, hipMemcpyDeviceToHost, c.stream));
    HIP_TRY(hipStreamSynchronize(c.stream));
  }
  return IBFE_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================

extern "C" {

const char* ibfe_last_error(void) { return ibfe::last_error_message().c_str(); }

int ibfe_plan_create(const ibfe_grid* grid, const ibfe_ib* ib, const ibfe_params* params,
                     const ibfe_inlet* inlet, ibfe_plan** out) {
  if (!out) return fail(IBFE_EINVAL, "out is NULL");
  *out = nullptr;
  std::unique_ptr<ibfe_plan> pl(new (std::nothrow) ibfe_plan());
  if (!pl) return fail(IBFE_ENOMEM, "host allocation failed");
  std::string err;
  int rc = build_plan(grid, ib, params, inlet, pl->p, err);
  if (rc) return fail(rc, err);
  *out = pl.release();
  return IBFE_OK;
}

int ibfe_plan_sizes(const ibfe_plan* plan, int64_t* n_p, int64_t* n_free, int64_t* n_pfree,
                    int64_t* n_kept_cells, int64_t* n_floating) {
  if (!plan) return fail(IBFE_EINVAL, "plan is NULL");
  const Plan& P = plan->p;
  if (n_p) *n_p = int64_t(P.P_ids.size());
  if (n_free) *n_free = P.n_free;
  if (n_pfree) *n_pfree = P.n_pfree;
  if (n_kept_cells) *n_kept_cells = P.n_kept;
  if (n_floating) *n_floating = P.n_floating;
  return IBFE_OK;
}

int ibfe_plan_node_ids(const ibfe_plan* plan, int64_t* ids) {
  if (!plan || !ids) return fail(IBFE_EINVAL, "NULL argument");
  std::memcpy(ids, plan->p.P_ids.data(), sizeof(int64_t) * plan->p.P_ids.size());
  return IBFE_OK;
}

int ibfe_plan_node_flags(const ibfe_plan* plan, uint8_t* flags) {
  if (!plan || !flags) return fail(IBFE_EINVAL, "NULL argument");
  std::memcpy(flags, plan->p.flags.data(), plan->p.flags.size());
  return IBFE_OK;
}

void ibfe_plan_destroy(ibfe_plan* plan) { delete plan; }

int ibfe_create(const ibfe_grid* grid, const ibfe_ib* ib, const ibfe_params* params,
                const ibfe_inlet* inlet, const ibfe_alloc* alloc, void* hip_stream, ibfe_ctx** out) {
  if (!out) return fail(IBFE_EINVAL, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(IBFE_EHIP, "no HIP device");
  std::unique_ptr<ibfe_ctx> c(new (std::nothrow) ibfe_ctx());
  if (!c) return fail(IBFE_ENOMEM, "host allocation failed");
  std::string err;
  int rc = build_plan(grid, ib, params, inlet, c->plan, err);
  if (rc) return fail(rc, err);
  c->stream = reinterpret_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&c->device) != hipSuccess) return fail(IBFE_EHIP, "hipGetDevice failed");
  if (alloc && alloc->alloc && alloc->free) {
    c->alloc = *alloc;
    c->user_alloc = true;
  }
  if ((rc = setup_device(*c))) return rc;
  if ((rc = estimate_mass_lmin(*c))) return rc;
  *out = c.release();
  return IBFE_OK;
}

int ibfe_num_nodes(const ibfe_ctx* c, int64_t* n_u, int64_t* n_p) {
  if (!c) return fail(IBFE_EINVAL, "ctx is NULL");
  if (n_u) *n_u = c->nP;
  if (n_p) *n_p = c->nP;
  return IBFE_OK;
}

int ibfe_get_node_ids(const ibfe_ctx* c, int64_t* vel_ids, int64_t* p_ids) {
  if (!c) return fail(IBFE_EINVAL, "ctx is NULL");
  if (vel_ids) std::memcpy(vel_ids, c->plan.P_ids.data(), sizeof(int64_t) * c->nP);
  if (p_ids) std::memcpy(p_ids, c->plan.P_ids.data(), sizeof(int64_t) * c->nP);
  return IBFE_OK;
}

int ibfe_set_state(ibfe_ctx* c, const double* u, const double* p, double t, int on_device) {
  if (!c || !u || !p) return fail(IBFE_EINVAL, "NULL argument");
  if (!std::isfinite(t)) return fail(IBFE_EINVAL, "t must be finite");
  int rc;
  if ((rc = copy_in(*c, c->u, 3, u, on_device))) return rc;
  if ((rc = copy_in(*c, c->p, 1, p, on_device))) return rc;
  c->t = t;
  c->steps = 0;
  c->lam_warm = false;
  c->phi_warm = c->delta_warm = false;
  c->stats = ibfe_stats{};
  c->stats.t = t;
  return IBFE_OK;
}

int ibfe_step(ibfe_ctx* c, int nsteps) {
  if (!c || nsteps < 0) return fail(IBFE_EINVAL, "bad argument");
  if (!c->ib_valid) return fail(IBFE_EINVAL, "the Lagrangian points are not set (a failed ibfe_set_points)");
  for (int k = 0; k < nsteps; ++k) {
    const double t_save = c->t;
    int rc = c->plan.refined ? step_once_refined(*c) : step_once(*c);
    if (rc) {
      c->t = t_save;  // u, p were not swapped: the last completed state is intact
      return rc;
    }
  }
  return IBFE_OK;
}

}  // extern "C"

namespace {

// Scratch of one device rebuild of the IB operators for M points (np = 64 M
// support pairs): the positions, the (node, slot) pairs and their sorted copies,
// segment flags and positions, counters, the row lengths of G and the scan/sort
// work arrays.  Every section starts on a 256-byte boundary.
struct RebuildBufs {
  double* X = nullptr;
  uint32_t *keys = nullptr, *vals = nullptr, *skeys = nullptr, *svals = nullptr;
  int *flag = nullptr, *pos = nullptr, *counters = nullptr;
  int64_t* cnt = nullptr;
  uint32_t* hist = nullptr;
  void* sums = nullptr;
};

// Byte offsets of the sections (base may be null: then only the size is wanted).
size_t rebuild_layout(int64_t M, char* base, RebuildBufs* out) {
  const int64_t np = 64 * M;
  const int nb = scan_tiles(np);
  const int64_t sums_tiles = std::max<int64_t>({int64_t(scan_tiles(int64_t(kRadixBins) * nb)), int64_t(nb),
                                                int64_t(scan_tiles(M + 1)), int64_t(1)});
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return base ? base + o : nullptr;
  };
  RebuildBufs b;
  b.X = reinterpret_cast<double*>(take(sizeof(double) * 3 * M));
  b.keys = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * np));
  b.vals = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * np));
  b.skeys = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * np));
  b.svals = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * np));
  b.flag = reinterpret_cast<int*>(take(sizeof(int) * np));
  b.pos = reinterpret_cast<int*>(take(sizeof(int) * np));
  b.counters = reinterpret_cast<int*>(take(sizeof(int) * 8));
  b.cnt = reinterpret_cast<int64_t*>(take(sizeof(int64_t) * (M + 1)));
  b.hist = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t) * kRadixBins * size_t(nb)));
  b.sums = take(sizeof(int64_t) * size_t(sums_tiles));
  if (out) *out = b;
  return off;
}

// Exclusive prefix sums of n values (in may be out); sums holds scan_tiles(n) values.
template <typename T>
int exclusive_scan(ibfe_ctx& c, const T* in, T* out, int64_t n, T* sums) {
  const int nb = scan_tiles(n);
  if (nb == 0) return IBFE_OK;
  klaunch<k_tile_sums<T>>(c, dim3(nb), dim3(kBlock), 0, c.stream, in, n, sums);
  klaunch<k_scan_sums<T>>(c, dim3(1), dim3(kBlock), 0, c.stream, sums, nb);
  klaunch<k_scan_tiles<T>>(c, dim3(nb), dim3(kBlock), 0, c.stream, in, out, n, (const T*)sums);
  CHECK_LAUNCH();
  return IBFE_OK;
}

// Stable sort of n (key, value) pairs by the low `bits` bits of the key, 8 bits per
// pass; k0/v0 are overwritten, the result ends in k1/v1.
int radix_sort_pairs(ibfe_ctx& c, uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, int64_t n, int bits,
                     uint32_t* hist, uint32_t* sums) {
  const int nb = scan_tiles(n);
  if (nb == 0) return IBFE_OK;
  const int passes = std::max(1, (bits + 7) / 8);
  uint32_t *ki = k0, *vi = v0, *ko = k1, *vo = v1;
  int rc;
  for (int p = 0; p < passes; ++p) {
    klaunch<k_rs_hist>(c, dim3(nb), dim3(kBlock), 0, c.stream, (const uint32_t*)ki, n, 8 * p, hist, nb);
    if ((rc = exclusive_scan<uint32_t>(c, hist, hist, int64_t(kRadixBins) * nb, sums))) return rc;
    klaunch<k_rs_scatter>(c, dim3(nb), dim3(kBlock), 0, c.stream, (const uint32_t*)ki, (const uint32_t*)vi, ko, vo,
                          n, 8 * p, (const uint32_t*)hist, nb);
    CHECK_LAUNCH();
    std::swap(ki, ko);
    std::swap(vi, vo);
  }
  if (ki != k1) {
    HIP_TRY(hipMemcpyAsync(k1, ki, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c.stream));
    HIP_TRY(hipMemcpyAsync(v1, vi, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, c.stream));
  }
  return IBFE_OK;
}

// Rebuild buffers of ibfe_set_points, allocated on its first call.  The captured
// graphs are dropped: they may have been captured before the first rebuild.
int setup_moving(ibfe_ctx& C) {
  const int64_t M = C.plan.M;
  void* b = nullptr;
  int rc;
  if ((rc = C.dalloc(&b, rebuild_layout(M, nullptr, nullptr)))) return rc;
  RebuildBufs r;
  rebuild_layout(M, static_cast<char*>(b), &r);
  auto& mv = C.mv;
  mv.X = r.X;
  mv.keys = r.keys;
  mv.vals = r.vals;
  mv.skeys = r.skeys;
  mv.svals = r.svals;
  mv.flag = r.flag;
  mv.pos = r.pos;
  mv.counters = r.counters;
  mv.cnt = r.cnt;
  mv.hist = r.hist;
  mv.sums = r.sums;
  HIP_TRY(hipStreamSynchronize(C.stream));
  for (auto& kv : C.graph_cache) (void)hipGraphExecDestroy(kv.second);
  C.graph_cache.clear();
  mv.ready = true;
  return IBFE_OK;
}

// The device rebuild for new positions X (and velocities U_B, NULL = 0) into the
// context's IB operators, with the scratch B: stencils of Eq. 17, the spreading
// lists (pairs sorted by node), G = I_F I_F^T row by row and its block inverses.
// Synchronises the stream twice (error counts, the size of G).
int rebuild_points(ibfe_ctx& C, const RebuildBufs& B, const double* X, const double* U_B, int on_device) {
  const Plan& P = C.plan;
  const int64_t M = P.M;
  C.ib_valid = false;
  const size_t bytes = sizeof(double) * 3 * size_t(M);
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HIP_TRY(hipMemcpyAsync(B.X, X, bytes, kind, C.stream));
  if (U_B)
    HIP_TRY(hipMemcpyAsync(C.UB, U_B, bytes, kind, C.stream));
  else
    klaunch<k_fill_f64>(C, dim3(blocks_lin(3 * M)), dim3(kBlock), 0, C.stream, C.UB, int64_t(3 * M), 0.0);
  klaunch<k_fill_i32>(C, dim3(1), dim3(kBlock), 0, C.stream, B.counters, int64_t(8), 0);
  const int64_t np = 64 * M;
  const uint32_t N = uint32_t(P.N);
  GridGeom g{P.origin[0], P.origin[1], P.origin[2], P.h, P.nx, P.ny, P.nz, P.sy, P.sz};
  klaunch<k_ib_stencil>(C, dim3(blocks_lin(M)), dim3(kBlock), 0, C.stream, int(M), g, (const double*)B.X,
                        (const uint8_t*)C.flags, N, C.ib_idx, C.ib_w, B.keys, B.vals, B.counters,
                        (const uint8_t*)C.ib_band);
  CHECK_LAUNCH();
  int bits = 1;
  while (bits < 32 && (uint64_t(1) << bits) <= uint64_t(N)) ++bits;
  int rc;
  if ((rc = radix_sort_pairs(C, B.keys, B.vals, B.skeys, B.svals, np, bits, B.hist,
                             static_cast<uint32_t*>(B.sums))))
    return rc;
  const int nbp = int((np + kBlock - 1) / kBlock);
  klaunch<k_sp_flags>(C, dim3(nbp), dim3(kBlock), 0, C.stream, np, (const uint32_t*)B.skeys, N, B.flag);
  CHECK_LAUNCH();
  if ((rc = exclusive_scan<int>(C, B.flag, B.pos, np, static_cast<int*>(B.sums)))) return rc;
  klaunch<k_sp_fill>(C, dim3(nbp), dim3(kBlock), 0, C.stream, np, int(M), (const uint32_t*)B.skeys,
                     (const uint32_t*)B.svals, N, (const int*)B.flag, (const int*)B.pos, (const double*)C.ib_w,
                     C.sp_node, C.sp_ptr, C.sp_pt, C.sp_wt, B.counters);
  CHECK_LAUNCH();
  int hc[8];
  HIP_TRY(hipMemcpyAsync(hc, B.counters, sizeof(hc), hipMemcpyDeviceToHost, C.stream));
  HIP_TRY(hipStreamSynchronize(C.stream));
  if (hc[4] > 0)
    return fail(IBFE_EINVAL, std::to_string(hc[4]) +
                                 " support node(s) of the moved points leave the refined band (the closure of the "
                                 "flagged cells without the hanging nodes)");
  if (hc[0] > 0)
    return fail(IBFE_ESINGULAR, std::to_string(hc[0]) + " Lagrangian point(s) without a free support node");
  const int64_t nvalid = hc[3];
  klaunch<(k_gram_rows<false>)>(C, dim3(unsigned(M)), dim3(64), 0, C.stream, int(M), (const int32_t*)C.ib_idx,
                                (const double*)C.ib_w, (const uint8_t*)C.flags, (const uint32_t*)B.skeys, nvalid,
                                (const int32_t*)C.sp_pt, (const double*)C.sp_wt, B.cnt, (const int64_t*)nullptr,
                                (int32_t*)nullptr, (double*)nullptr, (double*)nullptr, B.counters);
  CHECK_LAUNCH();
  if ((rc = exclusive_scan<int64_t>(C, B.cnt, C.G_ptr, M + 1, static_cast<int64_t*>(B.sums)))) return rc;
  int64_t nnz = 0;
  HIP_TRY(hipMemcpyAsync(&nnz, C.G_ptr + M, sizeof(int64_t), hipMemcpyDeviceToHost, C.stream));
  HIP_TRY(hipMemcpyAsync(hc, B.counters, sizeof(hc), hipMemcpyDeviceToHost, C.stream));
  HIP_TRY(hipStreamSynchronize(C.stream));
  if (hc[1] > 0)
    return fail(IBFE_EINVAL, "a Lagrangian point overlaps more than " + std::to_string(kGramCap) +
                                 " support products: the points are too dense");
  if (nnz > C.mv.g_cap) return fail(IBFE_ENOMEM, "the force system exceeds its capacity");
  klaunch<(k_gram_rows<true>)>(C, dim3(unsigned(M)), dim3(64), 0, C.stream, int(M), (const int32_t*)C.ib_idx,
                               (const double*)C.ib_w, (const uint8_t*)C.flags, (const uint32_t*)B.skeys, nvalid,
                               (const int32_t*)C.sp_pt, (const double*)C.sp_wt, (int64_t*)nullptr,
                               (const int64_t*)C.G_ptr, C.G_col, C.G_val, C.G_diag, B.counters);
  const int nblk = int((M + kIBBlock - 1) / kIBBlock);
  klaunch<k_gram_block_inv>(C, dim3(nblk), dim3(kBlock), 0, C.stream, int(M), (const int64_t*)C.G_ptr,
                            (const int32_t*)C.G_col, (const double*)C.G_val, C.G_binv);
  CHECK_LAUNCH();
  C.n_sp = hc[2];
  C.ib_valid = true;
  return IBFE_OK;
}

int check_points(const ibfe_ctx& C, const double* X, const double* U_B, int on_device) {
  const Plan& P = C.plan;
  if (64 * P.M > int64_t(INT32_MAX) - 1) return fail(IBFE_EINVAL, "too many Lagrangian points to move");
  if (!on_device) {
    for (int64_t q = 0; q < 3 * P.M; ++q)
      if (!std::isfinite(X[q]) || (U_B && !std::isfinite(U_B[q])))
        return fail(IBFE_EINVAL, "X and U_B must be finite");
  }
  return IBFE_OK;
}

// The allocation-free rebuild takes its scratch from this array (one copy per
// device, held until the process ends); host code uses the per-device address
// from hipGetSymbolAddress, never the array's name.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Address of this device's scratch array (looked up once per device, with that
// device current).
int scratch_address(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return fail(IBFE_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    if (cur != device) HIP_TRY(hipSetDevice(device));
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) HIP_TRY(hipSetDevice(cur));
    if (e != hipSuccess || !p)
      return fail(IBFE_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[device] = p;
  }
  *out = g_scratch_ptr[device];
  return IBFE_OK;
}

}  // namespace

extern "C" {

int ibfe_set_points(ibfe_ctx* c, const double* X, const double* U_B, int on_device) {
  if (!c || !X) return fail(IBFE_EINVAL, "NULL argument");
  ibfe_ctx& C = *c;
  if (C.plan.M == 0) return IBFE_OK;
  int rc;
  if ((rc = check_points(C, X, U_B, on_device))) return rc;
  if (!C.mv.ready && (rc = setup_moving(C))) return rc;
  RebuildBufs B;
  B.X = C.mv.X;
  B.keys = C.mv.keys;
  B.vals = C.mv.vals;
  B.skeys = C.mv.skeys;
  B.svals = C.mv.svals;
  B.flag = C.mv.flag;
  B.pos = C.mv.pos;
  B.counters = C.mv.counters;
  B.cnt = C.mv.cnt;
  B.hist = C.mv.hist;
  B.sums = C.mv.sums;
  return rebuild_points(C, B, X, U_B, on_device);
}

int ibfe_set_points_noalloc(ibfe_ctx* c, const double* X, const double* U_B, int on_device) {
  if (!c || !X) return fail(IBFE_EINVAL, "NULL argument");
  ibfe_ctx& C = *c;
  const int64_t M = C.plan.M;
  if (M == 0) return IBFE_OK;
  int rc;
  if ((rc = check_points(C, X, U_B, on_device))) return rc;
  const size_t need = rebuild_layout(M, nullptr, nullptr);
  if (need > kNoAllocScratchBytes)
    return fail(IBFE_EINVAL, "ibfe_set_points_noalloc: " + std::to_string(M) + " points need " +
                                 std::to_string(need) + " bytes of scratch, more than its " +
                                 std::to_string(kNoAllocScratchBytes) + " (at most " +
                                 std::to_string(ibfe_set_points_noalloc_max_points()) + " points)");
  void* base = nullptr;
  if ((rc = scratch_address(C.device, &base))) return rc;
  RebuildBufs B;
  rebuild_layout(M, static_cast<char*>(base), &B);
  return rebuild_points(C, B, X, U_B, on_device);
}

int64_t ibfe_set_points_noalloc_max_points(void) {
  int64_t lo = 0, hi = int64_t(kNoAllocScratchBytes);
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) / 2;
    if (rebuild_layout(mid, nullptr, nullptr) <= kNoAllocScratchBytes) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

int ibfe_run_steady(ibfe_ctx* c, double tol, int64_t max_steps, int64_t* steps, double* nrmse) {
  if (!c || !steps || !nrmse) return fail(IBFE_EINVAL, "NULL argument");
  if (!(tol >= 0.0) || max_steps < 0) return fail(IBFE_EINVAL, "tol must be >= 0 and max_steps >= 0");
  ibfe_ctx& C = *c;
  *steps = 0;
  nrmse[0] = nrmse[1] = nrmse[2] = HUGE_VAL;
  if (!C.ib_valid) return fail(IBFE_EINVAL, "the Lagrangian points are not set (a failed ibfe_set_points)");
  // 9 partial rows per block within the kMaxRows x kRedBlocks buffer
  const int nr = std::max(1, std::min(red_blocks(C.nchunks), kMaxRows * kRedBlocks / 9));
  for (int64_t k = 0; k < max_steps; ++k) {
    const double t_save = C.t;
    int rc = C.plan.refined ? step_once_refined(C) : step_once(C);
    if (rc) {
      C.t = t_save;
      return rc;
    }
    *steps = k + 1;
    if (C.nP == 0) {
      nrmse[0] = nrmse[1] = nrmse[2] = 0.0;
    } else {
      // after the step c.u holds u^{n+1} and c.u_next the previous state
      klaunch<k_nrmse_part>(C, dim3(nr), dim3(kBlock), 0, C.stream, C.nl, (const uint8_t*)C.flags,
                         uint32_t(kFlagP), (const double*)C.u, (const double*)C.u_next, C.stride, C.partials);
      klaunch<k_fin_nrmse>(C, dim3(1), dim3(kBlock), 0, C.stream, (const double*)C.partials, nr,
                         double(C.nP), C.nrmse);
      CHECK_LAUNCH();
      HIP_TRY(hipMemcpyAsync(C.host_nrmse, C.nrmse, 3 * sizeof(double), hipMemcpyDeviceToHost, C.stream));
      HIP_TRY(hipStreamSynchronize(C.stream));
      for (int d = 0; d < 3; ++d) nrmse[d] = C.host_nrmse[d];
    }
    if (nrmse[0] < tol && nrmse[1] < tol && nrmse[2] < tol) break;
  }
  return IBFE_OK;
}

int ibfe_get_state(ibfe_ctx* c, double* u, double* p, double* t, int on_device) {
  if (!c) return fail(IBFE_EINVAL, "ctx is NULL");
  int rc;
  if (u && (rc = copy_out(*c, c->u, 3, u, on_device))) return rc;
  if (p && (rc = copy_out(*c, c->p, 1, p, on_device))) return rc;
  if (t) *t = c->t;
  return IBFE_OK;
}

}  // extern "C"

namespace {

// Checkpoint layout (host memory): header, then u (3 x n_p), p, Phi, delta (3 x n_p)
// and Lambda (3 x M) as FP64 in canonical order.
struct CkptHeader {
  char magic[8];
  int64_t n_p, M;
  double t;
  int64_t steps;
  int32_t warm;  // bit 0: Lambda, bit 1: Phi, bit 2: delta hold the last step's values
  int32_t reserved;
};
static_assert(sizeof(CkptHeader) == 48, "checkpoint header layout");
constexpr char kCkptMagic[8] = {'I', 'B', 'F', 'E', 'C', 'K', 'P', '1'};

size_t ckpt_bytes(const ibfe_ctx& c) {
  return sizeof(CkptHeader) + sizeof(double) * (size_t(8) * size_t(c.nP) + size_t(3) * size_t(c.plan.M));
}

}  // namespace

extern "C" {

int ibfe_checkpoint_size(const ibfe_ctx* c, size_t* bytes) {
  if (!c || !bytes) return fail(IBFE_EINVAL, "NULL argument");
  *bytes = ckpt_bytes(*c);
  return IBFE_OK;
}

int ibfe_checkpoint_save(ibfe_ctx* c, void* buf, size_t bytes) {
  if (!c || !buf) return fail(IBFE_EINVAL, "NULL argument");
  if (bytes < ckpt_bytes(*c)) return fail(IBFE_EINVAL, "checkpoint buffer too small");
  CkptHeader h{};
  std::memcpy(h.magic, kCkptMagic, 8);
  h.n_p = c->nP;
  h.M = c->plan.M;
  h.t = c->t;
  h.steps = c->steps;
  h.warm = (c->lam_warm ? 1 : 0) | (c->phi_warm ? 2 : 0) | (c->delta_warm ? 4 : 0);
  std::memcpy(buf, &h, sizeof(h));
  double* d = reinterpret_cast<double*>(static_cast<char*>(buf) + sizeof(h));
  const int64_t n = c->nP;
  int rc;
  if ((rc = copy_out(*c, c->u, 3, d, 0))) return rc;
  if ((rc = copy_out(*c, c->p, 1, d + 3 * n, 0))) return rc;
  if ((rc = copy_out(*c, c->phi, 1, d + 4 * n, 0))) return rc;
  if ((rc = copy_out(*c, c->delta, 3, d + 5 * n, 0))) return rc;
  double* lam = d + 8 * n;
  for (int k = 0; k < 3 && c->plan.M > 0; ++k)
    HIP_TRY(hipMemcpyAsync(lam + k * c->plan.M, c->ibv[1] + k * c->mstride, sizeof(double) * c->plan.M,
                           hipMemcpyDeviceToHost, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return IBFE_OK;
}

int ibfe_checkpoint_load(ibfe_ctx* c, const void* buf, size_t bytes) {
  if (!c || !buf) return fail(IBFE_EINVAL, "NULL argument");
  if (bytes < sizeof(CkptHeader)) return fail(IBFE_EINVAL, "checkpoint buffer too small");
  CkptHeader h;
  std::memcpy(&h, buf, sizeof(h));
  if (std::memcmp(h.magic, kCkptMagic, 8) != 0) return fail(IBFE_EINVAL, "not a checkpoint");
  if (h.n_p != c->nP || h.M != c->plan.M)
    return fail(IBFE_EINVAL, "checkpoint sizes do not match the context");
  if (bytes < ckpt_bytes(*c)) return fail(IBFE_EINVAL, "checkpoint buffer too small");
  if (!std::isfinite(h.t) || h.steps < 0) return fail(IBFE_EINVAL, "bad checkpoint header");
  const double* d = reinterpret_cast<const double*>(static_cast<const char*>(buf) + sizeof(h));
  const int64_t n = c->nP;
  int rc;
  if ((rc = copy_in(*c, c->u, 3, d, 0))) return rc;
  if ((rc = copy_in(*c, c->p, 1, d + 3 * n, 0))) return rc;
  if ((rc = copy_in(*c, c->phi, 1, d + 4 * n, 0))) return rc;
  if ((rc = copy_in(*c, c->delta, 3, d + 5 * n, 0))) return rc;
  const double* lam = d + 8 * n;
  for (int k = 0; k < 3 && c->plan.M > 0; ++k)
    HIP_TRY(hipMemcpyAsync(c->ibv[1] + k * c->mstride, lam + k * c->plan.M, sizeof(double) * c->plan.M,
                           hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  c->t = h.t;
  c->steps = h.steps;
  c->lam_warm = (h.warm & 1) != 0;
  c->phi_warm = (h.warm & 2) != 0;
  c->delta_warm = (h.warm & 4) != 0;
  c->stats = ibfe_stats{};
  c->stats.steps = c->steps;
  c->stats.t = c->t;
  return IBFE_OK;
}

int ibfe_inject_breakdown(ibfe_ctx* c, int iteration) {
  if (!c || iteration < 0) return fail(IBFE_EINVAL, "bad argument");
  const int32_t v = iteration;
  HIP_TRY(hipMemcpyAsync(&c->scal[kScS1].brk_at, &v, sizeof(v), hipMemcpyHostToDevice, c->stream));
  HIP_TRY(hipStreamSynchronize(c->stream));
  return IBFE_OK;
}

int ibfe_get_stats(const ibfe_ctx* c, ibfe_stats* stats) {
  if (!c || !stats) return fail(IBFE_EINVAL, "NULL argument");
  *stats = c->stats;
  return IBFE_OK;
}

int ibfe_set_kernel_timing(ibfe_ctx* c, int enable) {
  if (!c) return fail(IBFE_EINVAL, "ctx is NULL");
  int rc_;
  if (c->timing && (rc_ = collect_kernel_times(*c))) return rc_;
  c->timing = enable != 0;
  c->kt.acc.clear();
  c->stats.poisson_apply_ms = 0.0;
  c->stats.poisson_applies = 0;
  c->stats.mass_apply_ms = 0.0;
  c->stats.mass_applies = 0;
  return IBFE_OK;
}

int ibfe_set_kernel_timing_filter(ibfe_ctx* c, const char* kernel) {
  if (!c) return fail(IBFE_EINVAL, "ctx is NULL");
  int rc;
  if ((rc = collect_kernel_times(*c))) return rc;
  c->kt.only = kernel ? std::string(kernel) : std::string();
  return IBFE_OK;
}

int ibfe_get_kernel_times(ibfe_ctx* c, ibfe_kernel_time* out, int32_t cap, int32_t* n) {
  if (!c || !n || cap < 0 || (cap > 0 && !out)) return fail(IBFE_EINVAL, "bad argument");
  int rc;
  if ((rc = collect_kernel_times(*c))) return rc;
  std::vector<std::pair<std::string, KTimer::Acc>> v(c->kt.acc.begin(), c->kt.acc.end());
  std::sort(v.begin(), v.end(), [](const auto& a, const auto& b) { return a.second.ms > b.second.ms; });
  *n = int32_t(v.size());
  for (int32_t i = 0; i < cap && i < int32_t(v.size()); ++i) {
    std::memset(out[i].name, 0, sizeof(out[i].name));
    std::strncpy(out[i].name, v[i].first.c_str(), sizeof(out[i].name) - 1);
    out[i].total_ms = v[i].second.ms;
    out[i].launches = v[i].second.launches;
  }
  return IBFE_OK;
}

int ibfe_set_graphs(ibfe_ctx* c, int enable) {
  if (!c) return fail(IBFE_EINVAL, "ctx is NULL");
  if ((enable != 0) != c->graphs) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& kv : c->graph_cache) (void)hipGraphExecDestroy(kv.second);
    c->graph_cache.clear();
  }
  c->graphs = enable != 0;
  return IBFE_OK;
}

int ibfe_get_field(ibfe_ctx* c, int which, double* out, int on_device) {
  if (!c || !out) return fail(IBFE_EINVAL, "NULL argument");
  switch (which) {
    case IBFE_FIELD_USTAR: return copy_out(*c, c->ustar, 3, out, on_device);
    case IBFE_FIELD_UIB: return copy_out(*c, c->uib, 3, out, on_device);
    case IBFE_FIELD_PHI: return copy_out(*c, c->phi, 1, out, on_device);
    default: return fail(IBFE_EINVAL, "unknown field");
  }
}

int ibfe_wall_shear(ibfe_ctx* c, const double* normals, double* tau, int on_device) {
  if (!c || !normals || !tau) return fail(IBFE_EINVAL, "NULL argument");
  ibfe_ctx& C = *c;
  const Plan& P = C.plan;
  if (P.M == 0) return fail(IBFE_EINVAL, "no Lagrangian points");
  const int M = int(P.M);
  const size_t bytes = sizeof(double) * 3 * size_t(M);
  // scratch: the strain planes in two 3-plane work fields, normals and result in
  // the IB vectors that do not hold the force of the last step
  double* ed = C.w[6];
  double* eo = C.w[7];
  const double* nrm = normals;
  if (!on_device) {
    HIP_TRY(hipMemcpyAsync(C.ibv[0], normals, bytes, hipMemcpyHostToDevice, C.stream));
    nrm = C.ibv[0];
  }
  double* out = on_device ? tau : C.ibv[2];
  if (P.refined) {
    // composite weak gradients of each component: hanging entries filled with the
    // parents' mean, hanging rows gathered into their parents
    double* uc = C.w[5];
    const int nb = blocks_for(C.nchunks);
    klaunch<k_axpby>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, 1.0, (const double*)C.u, 0.0,
                       (const double*)C.u, uc, 3, C.stride);
    CHECK_LAUNCH();
    int rc;
    if ((rc = fill_hanging<double>(C, uc, 3))) return rc;
    double* g[3] = {C.w[2], C.w[3], C.w[4]};
    for (int d = 0; d < 3; ++d)
      if ((rc = comp_rows<double>(C, grad_elem(C, uc + d * C.stride), kFlagP, 0u, 1.0, g[d]))) return rc;
    klaunch<k_strain_from_grad>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, (const uint8_t*)C.flags,
                       (const double*)g[0], (const double*)g[1], (const double*)g[2], (const double*)C.lmass64,
                       C.stride, ed, eo);
  } else {
    klaunch<k_nodal_strain>(C, dim3(blocks_for(C.nchunks)), dim3(kBlock), 0, C.stream, C.nl,
                       (const uint8_t*)C.emask, (const uint8_t*)C.flags, (const double*)C.u, C.stride, P.h,
                       C.fc.g2[0], C.fc.g2[1], C.fc.g2[2], int(P.sy), int(P.sz), ed, eo);
  }
  klaunch<k_wall_shear>(C, dim3(blocks_lin(M)), dim3(kBlock), 0, C.stream, M, (const int32_t*)C.ib_idx,
                     (const double*)C.ib_w, (const double*)ed, (const double*)eo, C.stride, nrm, P.params.mu,
                     out);
  CHECK_LAUNCH();
  if (!on_device) HIP_TRY(hipMemcpyAsync(tau, C.ibv[2], bytes, hipMemcpyDeviceToHost, C.stream));
  HIP_TRY(hipStreamSynchronize(C.stream));
  return IBFE_OK;
}

int ibfe_apply(ibfe_ctx* c, int op, int precision, const double* x, double* y, int on_device) {
  if (!c || !x || !y) return fail(IBFE_EINVAL, "NULL argument");
  if (precision != 0 && precision != 1) return fail(IBFE_EINVAL, "precision must be 0 or 1");
  if (precision == 1 && op != IBFE_OP_MASS && op != IBFE_OP_STIFF && op != IBFE_OP_ADVDIFF)
    return fail(IBFE_EINVAL, "FP32 is available for MASS, STIFF and ADVDIFF only");
  ibfe_ctx& C = *c;
  C.lam_warm = false;  // the IB applies use the force buffer
  const Plan& P = C.plan;
  const int nb = blocks_for(C.nchunks);
  const int sy = int(P.sy), sz = int(P.sz);
  const int64_t S = C.stride;
  double* xin = C.w[0];
  double* yout = C.w[1];
  int rc;
  const int nc_in = (op == IBFE_OP_DIV || op == IBFE_OP_ADVDIFF || op == IBFE_OP_INTERP) ? 3 : 1;
  if (op == IBFE_OP_SPREAD) {
    if (P.M == 0) return fail(IBFE_EINVAL, "no Lagrangian points");
    // x is M x 3 row major -> planes of mstride
    std::vector<double> h(3 * C.mstride, 0.0);
    std::vector<double> hx(3 * P.M);
    if (on_device) {
      HIP_TRY(hipMemcpyAsync(hx.data(), x, sizeof(double) * 3 * P.M, hipMemcpyDeviceToHost, C.stream));
      HIP_TRY(hipStreamSynchronize(C.stream));
    } else {
      std::memcpy(hx.data(), x, sizeof(double) * 3 * P.M);
    }
    for (int64_t i = 0; i < P.M; ++i)
      for (int d = 0; d < 3; ++d) h[d * C.mstride + i] = hx[3 * i + d];
    HIP_TRY(hipMemcpyAsync(C.ibv[1], h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, C.stream));
    HIP_TRY(hipMemsetAsync(yout - C.halo, 0, sizeof(double) * 3 * S, C.stream));
    const int nn = C.n_sp;
    klaunch<k_ib_spread>(C, dim3(blocks_lin(nn)), dim3(kBlock), 0, C.stream, nn, C.sp_node, C.sp_ptr,
                       C.sp_pt, C.sp_wt, C.ibv[1], C.mstride, yout, S);
    CHECK_LAUNCH();
    return copy_out(C, yout, 3, y, on_device);
  }
  if ((rc = copy_in(C, xin, nc_in, x, on_device))) return rc;
  if (P.refined && op != IBFE_OP_INTERP) {
    int nc_out = 1;
    if ((rc = apply_refined(C, op, precision, xin, yout, nc_out))) return rc;
    return copy_out(C, yout, nc_out, y, on_device);
  }
  switch (op) {
    case IBFE_OP_MASS:
    case IBFE_OP_STIFF: {
      const double* f = op == IBFE_OP_MASS ? C.fc.m : C.fc.k;
      const double cf[4] = {f[0], f[1], f[2], f[3]};
      if (precision == 0) {
        auto o = sym_op<double, 1>(C, cf, kFlagP);
        klaunch<(k_apply<double, 1, OpSym<double, 1>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream,
                           C.nl, o, xin, yout);
      } else {
        if ((rc = ensure_fp32_work(C))) return rc;
        float* x32 = C.v32[0];
        float* y32 = C.v32[1];
        klaunch<(k_masked_copy<double, float>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, xin, x32, 1, S);
        auto o = sym_op<float, 1>(C, cf, kFlagP);
        klaunch<(k_apply<float, 1, OpSym<float, 1>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream,
                           C.nl, o, x32, y32);
        klaunch<(k_masked_copy<float, double>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, y32, yout, 1, S);
      }
      CHECK_LAUNCH();
      return copy_out(C, yout, 1, y, on_device);
    }
    case IBFE_OP_GRAD:
      klaunch<k_grad>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.emask, C.flags,
                         kFlagP, xin, yout, S, sy, sz, C.fc.g2[0], C.fc.g2[1], C.fc.g2[2]);
      CHECK_LAUNCH();
      return copy_out(C, yout, 3, y, on_device);
    case IBFE_OP_DIV:
      klaunch<k_div>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.emask, C.flags,
                         kFlagP, 0u, xin, yout, S, sy, sz, C.fc.g2[0], C.fc.g2[1], C.fc.g2[2], 1.0);
      CHECK_LAUNCH();
      return copy_out(C, yout, 1, y, on_device);
    case IBFE_OP_ADVDIFF: {
      if (!C.coef64) {
        // matrix-free context
        if (precision == 1 && !C.w32) {
          if ((rc = C.field(&C.w32, 3)) || (rc = C.field(&C.dinvS32, 1))) return rc;
          if ((rc = ensure_fp32_work(C))) return rc;
        }
        if ((rc = prep_s1_mf(C, precision == 1 || P.params.precision == 1))) return rc;
        const bool strain = P.params.viscous == 1;
        if (precision == 0) {
          if (strain)
            klaunch<(k_apply<double, 3, OpConvStrain<double>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl,
                                                                 conv_strain_op<double>(C, kFlagP), xin, yout);
          else
            klaunch<(k_apply<double, 3, OpConv<double>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl,
                                                           conv_op<double>(C, kFlagP), xin, yout);
        } else {
          float* x32 = C.v32[0];
          float* y32 = C.v32[1];
          klaunch<(k_masked_copy<double, float>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, xin, x32, 3, S);
          if (strain)
            klaunch<(k_apply<float, 3, OpConvStrain<float>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl,
                                                               conv_strain_op<float>(C, kFlagP), x32, y32);
          else
            klaunch<(k_apply<float, 3, OpConv<float>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl,
                                                         conv_op<float>(C, kFlagP), x32, y32);
          klaunch<(k_masked_copy<float, double>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, y32, yout, 3, S);
        }
        CHECK_LAUNCH();
        return copy_out(C, yout, 3, y, on_device);
      }
      float* c32 = C.coef32;
      if (precision == 1 && !c32) {
        // FP64-mode context: build an FP32 copy of the stencil in extra work space
        if ((rc = C.field(&C.coef32, 27))) return rc;
        if ((rc = ensure_fp32_work(C))) return rc;
        c32 = C.coef32;
      }
      if ((rc = build_s1(C))) return rc;
      const bool strain = P.params.viscous == 1;
      if (precision == 0) {
        if (strain)
          klaunch<(k_apply<double, 3, OpStencilStrain<double>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream,
                             C.nl, strain_op<double>(C, C.coef64, kFlagP), xin, yout);
        else
          klaunch<(k_apply<double, 3, OpStencil<double, 3>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream,
                             C.nl, stencil_op<double>(C, C.coef64, kFlagP), xin, yout);
      } else {
        float* x32 = C.v32[0];
        float* y32 = C.v32[1];
        klaunch<(k_masked_copy<double, float>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, xin, x32, 3, S);
        if (strain)
          klaunch<(k_apply<float, 3, OpStencilStrain<float>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream,
                             C.nl, strain_op<float>(C, c32, kFlagP), x32, y32);
        else
          klaunch<(k_apply<float, 3, OpStencil<float, 3>>)>(C, dim3(nb), dim3(kBlock), 0, C.stream,
                             C.nl, stencil_op<float>(C, c32, kFlagP), x32, y32);
        klaunch<(k_masked_copy<float, double>)>(C, dim3(nb), dim3(kBlock), 0, C.stream, C.nl, C.flags, kFlagP, y32, yout, 3, S);
      }
      CHECK_LAUNCH();
      return copy_out(C, yout, 3, y, on_device);
    }
    case IBFE_OP_INTERP: {
      if (P.M == 0) return fail(IBFE_EINVAL, "no Lagrangian points");
      const int M = int(P.M);
      klaunch<k_ib_interp>(C, dim3(blocks_lin(int64_t(M) * 8)), dim3(kBlock), 0, C.stream, M, C.ib_idx, C.ib_w,
                         C.UB, xin, S, C.ibv[0], C.mstride, 0);
      CHECK_LAUNCH();
      std::vector<double> h(3 * C.mstride);
      HIP_TRY(hipMemcpyAsync(h.data(), C.ibv[0], sizeof(double) * h.size(), hipMemcpyDeviceToHost, C.stream));
      HIP_TRY(hipStreamSynchronize(C.stream));
      std::vector<double> o(3 * M);
      for (int i = 0; i < M; ++i)
        for (int d = 0; d < 3; ++d) o[3 * i + d] = -h[d * C.mstride + i];
      if (on_device) {
        HIP_TRY(hipMemcpyAsync(y, o.data(), sizeof(double) * o.size(), hipMemcpyHostToDevice, C.stream));
        HIP_TRY(hipStreamSynchronize(C.stream));
      } else {
        std::memcpy(y, o.data(), sizeof(double) * o.size());
      }
      return IBFE_OK;
    }
    default: return fail(IBFE_EINVAL, "unknown operator");
  }
}

void ibfe_destroy(ibfe_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  (void)ibfe_attach_batcher(c, nullptr);
  delete c;
}

int ibfe_batcher_create(double window_us, ibfe_batcher** out) {
  if (!out || !(window_us >= 0.0)) return fail(IBFE_EINVAL, "need window_us >= 0 and an output pointer");
  *out = nullptr;
  std::unique_ptr<ibfe_batcher> B(new (std::nothrow) ibfe_batcher());
  if (!B) return fail(IBFE_ENOMEM, "host allocation failed");
  HIP_TRY(hipGetDevice(&B->device));
  HIP_TRY(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking));
  B->window_us = window_us;
  *out = B.release();
  return IBFE_OK;
}

int ibfe_attach_batcher(ibfe_ctx* c, ibfe_batcher* b) {
  if (!c) return fail(IBFE_EINVAL, "NULL context");
  if (b && b->device != c->device) return fail(IBFE_EINVAL, "batcher and context are on different devices");
  if (c->batcher == b) return IBFE_OK;
  if (c->batcher) {
    (void)hipStreamSynchronize(c->stream);
    std::lock_guard<std::mutex> lk(c->batcher->mu);
    c->batcher->members -= 1;
    c->batcher->cv.notify_all();
    c->batcher = nullptr;
  }
  if (!b) return IBFE_OK;
  if (!c->ev_ready) HIP_TRY(hipEventCreateWithFlags(&c->ev_ready, hipEventDisableTiming));
  if (!c->ev_done) HIP_TRY(hipEventCreateWithFlags(&c->ev_done, hipEventDisableTiming));
  std::lock_guard<std::mutex> lk(b->mu);
  b->members += 1;
  c->batcher = b;
  return IBFE_OK;
}

int ibfe_batcher_stats(ibfe_batcher* b, int64_t* batches, int64_t* members, int32_t* widest) {
  if (!b) return fail(IBFE_EINVAL, "NULL batcher");
  std::lock_guard<std::mutex> lk(b->mu);
  if (batches) *batches = b->batches;
  if (members) *members = b->jobs;
  if (widest) *widest = b->widest;
  return IBFE_OK;
}

int ibfe_batcher_destroy(ibfe_batcher* b) {
  if (!b) return IBFE_OK;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->members != 0) return fail(IBFE_EINVAL, "contexts are still attached to the batcher");
  }
  (void)hipStreamSynchronize(b->stream);
  (void)hipStreamDestroy(b->stream);
  delete b;
  return IBFE_OK;
}

}  // extern "C"
