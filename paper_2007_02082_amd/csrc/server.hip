// Serving loop: independent flow solves admitted first-in first-out by device
// footprint into a fixed number of worker slots.  Each slot owns a HIP stream
// and drives one request at a time through the C ABI (create, step, read,
// destroy); slots run concurrently, so the kernels of admitted requests overlap
// on the GPU.  With batching on, the running requests share a batcher that
// joins their mass-correction Chebyshev steps into single launches over all of
// their column items.  A request's arithmetic does not depend on what else
// runs, so its result is identical alone and in a mix.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "ibfe.h"

namespace ibfe {
std::string& last_error_message();
}

namespace {

int sfail(int code, const std::string& msg) {
  ibfe::last_error_message() = msg;
  return code;
}

// Deep copy of a request's inputs.
struct Job {
  int64_t id = 0;
  ibfe_grid grid{};
  ibfe_ib ib{};
  ibfe_params params{};
  ibfe_inlet inlet{};
  int32_t nsteps = 0;
  double t0 = 0.0;
  std::vector<uint8_t> mask, tag, refine;
  std::vector<double> X, UB, shape;
  std::vector<int64_t> inlet_ids;
  size_t footprint = 0;
  // results
  ibfe_result res{};
  std::vector<double> u, p;
  std::vector<int64_t> ids;
};

size_t footprint_of(const ibfe_grid& g, int64_t M, const ibfe_params& pr) {
  const bool ref = g.refine_cell != nullptr;
  const int64_t f = ref ? 2 : 1;
  const int64_t sy = f * g.nx + 1, sz = sy * (f * g.ny + 1);
  const int64_t N = sz * (f * g.nz + 1);
  const int64_t halo = ((f * (sz + sy + 1) + 63) / 64) * 64;
  const int64_t stride = 2 * halo + ((N + 63) / 64) * 64;
  // the assembled advection-diffusion stencil (27 planes, 54 when refined, FP64
  // and in mixed mode FP32) or, matrix-free, the inverse diagonals and u^n in FP32
  const bool stencil = pr.advdiff == 1 || pr.advection == 1;
  const double planes = ref ? 54.0 : 27.0;
  double bytes = double(stride) * (48.0 * 8.0 + 3.0);              // FP64 fields, node bytes
  if (pr.precision == 1) bytes += double(stride) * 30.0 * 4.0;     // FP32 work space
  if (stencil) {
    bytes += double(stride) * planes * 8.0;
    if (pr.precision == 1) bytes += double(stride) * planes * 4.0;
  } else {
    bytes += double(stride) * (32.0 + (pr.precision == 1 ? 16.0 : 0.0));
  }
  // refined: coarse cell bits, parent slots, inverse diagonals
  if (ref) bytes += double(stride) * (1.0 + 4.0 + 24.0);
  // the tensor-preconditioned mass correction: scaled residual (and its rows with
  // coarse cells), 3 planes each
  if (pr.mass_precond == 1) bytes += double(stride) * 3.0 * (ref ? 2.0 : 1.0) * (pr.precision == 1 ? 4.0 : 8.0);
  // the tentative-velocity BiCGStab's six node-list-order vectors (at most one
  // entry per lattice position and component)
  if (pr.advection == 0) bytes += double(stride) * 18.0 * (pr.precision == 1 ? 4.0 : 8.0);
  if (pr.precond >= 1) bytes += 0.15 * double(stride) * (5.0 * (pr.precision == 1 ? 4 : 8) + 2.0);
  // IB arrays: stencils, spreading lists and G, held at the sizes a rebuild for
  // moved points may need (64 pairs per point, four times G's entries)
  bytes += double(M) * (64.0 * 12.0 + 64.0 * 24.0 + 4.0 * 150.0 * 12.0 + 15.0 * 8.0 + 64.0);
  if (ref && M > 0) bytes += double(N);  // the band of allowed support nodes
  bytes += 3.0 * 8.0 * double(N + M) + 8.0 * 2048.0 * 8.0;         // compact copies, partials
  return size_t(bytes * 1.05) + (16u << 20);
}

double now_s(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

}  // namespace

struct ibfe_server {
  int device = 0;
  ibfe_batcher* batcher = nullptr;  // joins the running requests' mass-correction kernels
  size_t budget = 0, used = 0;
  int32_t running = 0, peak = 0;
  bool stop = false;
  int64_t next_id = 1;
  std::chrono::steady_clock::time_point t0;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::shared_ptr<Job>> queue;
  std::map<int64_t, std::shared_ptr<Job>> jobs;
  std::vector<std::thread> workers;
};

namespace {

void run_job(Job& J, hipStream_t stream, ibfe_batcher* batcher) {
  ibfe_ctx* ctx = nullptr;
  int rc = ibfe_create(&J.grid, &J.ib, &J.params, &J.inlet, nullptr, stream, &ctx);
  if (rc == IBFE_OK && batcher) rc = ibfe_attach_batcher(ctx, batcher);
  if (rc == IBFE_OK) {
    int64_t nu = 0, np = 0;
    ibfe_num_nodes(ctx, &nu, &np);
    std::vector<double> u0(3 * nu, 0.0), p0(np, 0.0);
    rc = ibfe_set_state(ctx, u0.data(), p0.data(), J.t0, 0);
    if (rc == IBFE_OK) rc = ibfe_step(ctx, J.nsteps);
    if (rc == IBFE_OK) {
      J.u.resize(3 * nu);
      J.p.resize(np);
      J.ids.resize(nu);
      rc = ibfe_get_state(ctx, J.u.data(), J.p.data(), nullptr, 0);
      if (rc == IBFE_OK) rc = ibfe_get_node_ids(ctx, J.ids.data(), nullptr);
      J.res.n_u = nu;
      J.res.n_p = np;
    }
    ibfe_get_stats(ctx, &J.res.stats);
  }
  if (rc != IBFE_OK) J.res.error = rc;
  if (ctx) ibfe_destroy(ctx);
}

void worker_loop(ibfe_server* S) {
  (void)hipSetDevice(S->device);
  hipStream_t stream = nullptr;
  if (hipStreamCreateWithFlags(&stream, hipStreamNonBlocking) != hipSuccess) stream = nullptr;
  while (true) {
    std::shared_ptr<Job> job;
    {
      std::unique_lock<std::mutex> lk(S->mu);
      S->cv.wait(lk, [&] {
        return S->stop || (!S->queue.empty() && S->used + S->queue.front()->footprint <= S->budget);
      });
      if (S->stop) break;
      job = S->queue.front();
      S->queue.pop_front();
      S->used += job->footprint;
      S->running += 1;
      S->peak = std::max(S->peak, S->running);
      job->res.status = IBFE_REQ_RUNNING;
      job->res.t_admit = now_s(S->t0);
    }
    run_job(*job, stream, S->batcher);
    {
      std::lock_guard<std::mutex> lk(S->mu);
      S->used -= job->footprint;
      S->running -= 1;
      job->res.t_done = now_s(S->t0);
      job->res.status = job->res.error ? IBFE_REQ_FAILED : IBFE_REQ_DONE;
    }
    S->cv.notify_all();
  }
  if (stream) (void)hipStreamDestroy(stream);
}

}  // namespace

extern "C" {

int ibfe_request_footprint(const ibfe_request* req, size_t* bytes) {
  if (!req || !req->grid || !req->params || !bytes) return sfail(IBFE_EINVAL, "NULL argument");
  *bytes = footprint_of(*req->grid, req->ib ? req->ib->M : 0, *req->params);
  return IBFE_OK;
}

int ibfe_server_create(size_t budget_bytes, int32_t max_slots, ibfe_server** out) {
  if (!out || max_slots < 1 || max_slots > 16) return sfail(IBFE_EINVAL, "need 1 <= max_slots <= 16");
  *out = nullptr;
  std::unique_ptr<ibfe_server> S(new (std::nothrow) ibfe_server());
  if (!S) return sfail(IBFE_ENOMEM, "host allocation failed");
  if (hipGetDevice(&S->device) != hipSuccess) return sfail(IBFE_EHIP, "no HIP device");
  if (budget_bytes == 0) {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) return sfail(IBFE_EHIP, "hipMemGetInfo failed");
    budget_bytes = size_t(0.9 * double(fr));
  }
  S->budget = budget_bytes;
  S->t0 = std::chrono::steady_clock::now();
  for (int i = 0; i < max_slots; ++i) S->workers.emplace_back(worker_loop, S.get());
  *out = S.release();
  return IBFE_OK;
}

int ibfe_server_submit(ibfe_server* S, const ibfe_request* req, int64_t* id) {
  if (!S || !req || !req->grid || !req->params || !id) return sfail(IBFE_EINVAL, "NULL argument");
  const ibfe_grid& g = *req->grid;
  if (g.nx < 1 || g.ny < 1 || g.nz < 1 || !g.node_mask) return sfail(IBFE_EINVAL, "bad grid");
  if (req->nsteps < 0) return sfail(IBFE_EINVAL, "nsteps must be >= 0");
  auto J = std::make_shared<Job>();
  const int64_t f = g.refine_cell ? 2 : 1;  // refined: node arrays live on the fine lattice
  const int64_t N = (f * g.nx + 1) * (f * g.ny + 1) * (f * g.nz + 1);
  J->grid = g;
  if (g.refine_cell) {
    J->refine.assign(g.refine_cell, g.refine_cell + int64_t(g.nx) * g.ny * g.nz);
    J->grid.refine_cell = J->refine.data();
  }
  J->mask.assign(g.node_mask, g.node_mask + N);
  J->grid.node_mask = J->mask.data();
  if (g.bc_tag) {
    J->tag.assign(g.bc_tag, g.bc_tag + N);
    J->grid.bc_tag = J->tag.data();
  }
  J->params = *req->params;
  if (req->ib) {
    J->ib = *req->ib;
    if (J->ib.M < 0 || (J->ib.M > 0 && !J->ib.X)) return sfail(IBFE_EINVAL, "bad Lagrangian points");
    if (J->ib.M > 0) {
      J->X.assign(J->ib.X, J->ib.X + 3 * J->ib.M);
      J->ib.X = J->X.data();
      if (J->ib.U_B) {
        J->UB.assign(J->ib.U_B, J->ib.U_B + 3 * J->ib.M);
        J->ib.U_B = J->UB.data();
      }
    }
  }
  if (req->inlet) {
    J->inlet = *req->inlet;
    if (J->inlet.n > 0) {
      if (!J->inlet.node_ids || !J->inlet.shape || J->inlet.K < 0)
        return sfail(IBFE_EINVAL, "bad inlet table");
      J->inlet_ids.assign(J->inlet.node_ids, J->inlet.node_ids + J->inlet.n);
      J->shape.assign(J->inlet.shape, J->inlet.shape + size_t(2 * J->inlet.K + 1) * J->inlet.n * 3);
      J->inlet.node_ids = J->inlet_ids.data();
      J->inlet.shape = J->shape.data();
    }
  }
  J->nsteps = req->nsteps;
  J->t0 = req->t0;
  J->footprint = footprint_of(J->grid, J->ib.M, J->params);
  {
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->stop) return sfail(IBFE_EINVAL, "server is shutting down");
    J->id = S->next_id++;
    J->res.footprint = J->footprint;
    J->res.t_submit = now_s(S->t0);
    S->jobs[J->id] = J;
    if (J->footprint > S->budget) {
      J->res.status = IBFE_REQ_FAILED;
      J->res.error = IBFE_ENOMEM;
      J->res.t_done = J->res.t_submit;
    } else {
      J->res.status = IBFE_REQ_QUEUED;
      S->queue.push_back(J);
    }
    *id = J->id;
  }
  S->cv.notify_all();
  return IBFE_OK;
}

int ibfe_server_poll(ibfe_server* S, int64_t id, ibfe_result* out) {
  if (!S || !out) return sfail(IBFE_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return sfail(IBFE_EINVAL, "unknown request id");
  *out = it->second->res;
  return IBFE_OK;
}

int ibfe_server_wait(ibfe_server* S, int64_t id, double timeout_s, ibfe_result* out) {
  if (!S || !out) return sfail(IBFE_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->jobs.find(id);
  if (it == S->jobs.end()) return sfail(IBFE_EINVAL, "unknown request id");
  std::shared_ptr<Job> J = it->second;
  auto finished = [&] { return J->res.status == IBFE_REQ_DONE || J->res.status == IBFE_REQ_FAILED; };
  if (timeout_s < 0)
    S->cv.wait(lk, finished);
  else
    S->cv.wait_for(lk, std::chrono::duration<double>(timeout_s), finished);
  *out = J->res;
  return IBFE_OK;
}

int ibfe_server_fetch(ibfe_server* S, int64_t id, double* u, double* p, int64_t* node_ids) {
  if (!S) return sfail(IBFE_EINVAL, "NULL argument");
  std::shared_ptr<Job> J;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->jobs.find(id);
    if (it == S->jobs.end()) return sfail(IBFE_EINVAL, "unknown request id");
    J = it->second;
    if (J->res.status != IBFE_REQ_DONE) return sfail(IBFE_EINVAL, "request is not done");
    S->jobs.erase(it);
  }
  if (u) std::memcpy(u, J->u.data(), sizeof(double) * J->u.size());
  if (p) std::memcpy(p, J->p.data(), sizeof(double) * J->p.size());
  if (node_ids) std::memcpy(node_ids, J->ids.data(), sizeof(int64_t) * J->ids.size());
  return IBFE_OK;
}

int ibfe_server_set_batching(ibfe_server* S, double window_us) {
  if (!S) return sfail(IBFE_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->batcher) return sfail(IBFE_EINVAL, "batching is already on");
  if (S->running != 0 || !S->queue.empty()) return sfail(IBFE_EINVAL, "set batching before submitting");
  return ibfe_batcher_create(window_us, &S->batcher);
}

int ibfe_server_batch_stats(ibfe_server* S, int64_t* batches, int64_t* members, int32_t* widest) {
  if (!S) return sfail(IBFE_EINVAL, "NULL argument");
  if (!S->batcher) {
    if (batches) *batches = 0;
    if (members) *members = 0;
    if (widest) *widest = 0;
    return IBFE_OK;
  }
  return ibfe_batcher_stats(S->batcher, batches, members, widest);
}

int ibfe_server_peak_concurrency(const ibfe_server* S, int32_t* peak) {
  if (!S || !peak) return sfail(IBFE_EINVAL, "NULL argument");
  *peak = S->peak;
  return IBFE_OK;
}

void ibfe_server_destroy(ibfe_server* S) {
  if (!S) return;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    // let running requests finish; fail the ones still queued
    for (auto& J : S->queue) {
      J->res.status = IBFE_REQ_FAILED;
      J->res.error = IBFE_EINVAL;
    }
    S->queue.clear();
    S->cv.wait(lk, [&] { return S->running == 0; });
    S->stop = true;
  }
  S->cv.notify_all();
  for (auto& t : S->workers) t.join();
  if (S->batcher) (void)ibfe_batcher_destroy(S->batcher);
  delete S;
}

}  // extern "C"
