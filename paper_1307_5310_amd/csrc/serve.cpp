// Serving loop: independent cavity solves, each marched slab by slab
// (Section 2.2, time slabs; each slab solved as in stdg_slab_solve), admitted
// by device footprint into one arena and advanced concurrently.
//
// One server thread owns the device work.  Each admitted request holds a
// contiguous reservation of the arena (its mesh tables, state, load and
// Krylov vectors are bump-allocated from it), its own stream and a resumable
// SlabSolver.  The thread polls the requests' events and, for every request
// whose last step has completed, runs the host part of that step and enqueues
// the next one, so the device always holds work of every active request and
// new requests join between steps (continuous batching at the granularity of
// one GMRES iteration).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "solver.h"

extern "C" int stdg_project_modes(const stdg_mesh* mesh, int32_t n_modes, const int32_t* mnl, const double* abc,
                                  double* state_dev, void* stream);
extern "C" int stdg_load_assemble(const stdg_mesh* mesh, const stdg_source* src, double t0, double dt,
                                  double* load_dev, void* stream);
extern "C" int stdg_energy(const stdg_mesh* mesh, const double* state_dev, double* energy_out, void* stream);

namespace stdg {

namespace {

using Clock = std::chrono::steady_clock;

struct Request {
  uint64_t ticket = 0;
  stdg_mesh* mesh = nullptr;  // analysed on the submitting thread, uploaded at admission
  std::vector<double> init;
  std::vector<int32_t> mnl;
  std::vector<double> abc;
  int64_t ne = 0;
  double t0 = 0.0, dt = 0.0;
  int n_slabs = 0;
  stdg_source src{};
  double c_diss = 0.0;
  int64_t n_unk = 0, n_trial = 0, n_state = 0;
  size_t footprint = 0;
  double t_submit = 0.0;
};

struct Finished {
  stdg_result res{};
  std::vector<double> state;
};

struct Active {
  Request* rq = nullptr;
  size_t off = 0;
  Ctx ctx{};
  stdg_mesh* mesh = nullptr;
  hipStream_t stream = nullptr;
  double* state = nullptr;
  double* load = nullptr;
  SlabSolver solver;
  bool solver_ready = false;
  int slab = 0;
  bool finishing = false;
  hipEvent_t done_ev = nullptr;
  double eta2 = 0.0;  // accumulated iteration-error bound (inexact solves)
  double pend_since = -1.0;  // server clock when its pending restart cycle was left for a batch
  Finished out;
};

// First-fit allocator over [0, size) with coalescing of free ranges.
class Arena {
 public:
  void reset(size_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) & ~(size_t)255;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes, noff = it->first + bytes;
        free_.erase(it);
        if (rest) free_[noff] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) & ~(size_t)255;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

}  // namespace

struct Server {
  Ctx* ctx = nullptr;
  stdg_serve_opts opts{};
  SlabOpts so;
  char* arena_mem = nullptr;
  size_t arena_size = 0;
  Arena arena;
  Clock::time_point t_start;
  std::mutex mu;
  std::condition_variable cv;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, Finished> finished;
  std::unordered_map<uint64_t, bool> known;  // submitted and not yet polled
  uint64_t next_ticket = 1;
  std::atomic<bool> stop{false};
  std::vector<Active*> active;  // server thread only
  std::thread th;
  // batched restart cycles: streams (round-robin) and their events
  static constexpr int kBatchStreams = 4;
  hipStream_t bstream[kBatchStreams] = {};
  hipEvent_t bev[kBatchStreams] = {};
  int bnext = 0;

  double now() const { return std::chrono::duration<double>(Clock::now() - t_start).count(); }
  void run();
  bool admit_one();
  int start(Active* a);
  int start_slab(Active* a);
  int step(Active* a, bool* finished_now);
  void retire(Active* a, int status);
  void launch_pending_cycles();
};

namespace {

size_t footprint_of(const Request& r, const SlabOpts& so) {
  auto r256 = [](size_t b) { return (b + 255) & ~(size_t)255; };
  const Mesh& m = r.mesh->m;
  size_t b = mesh_device_bytes(m);
  // preconditioner scratch of meshes with a non-diagonal metric or local time
  // steps (the P^{-1} pre-pass; FP32 then FP64)
  if (m.n_diag != m.ne || !m.lt.empty()) b += r256(sizeof(float) * r.n_unk) + r256(sizeof(double) * r.n_unk);
  // state, load, projection inputs
  b += r256(sizeof(double) * r.n_state) + (r.src.kind ? r256(sizeof(double) * r.n_unk) : 0) +
       2 * r256(sizeof(double) * 3 * (r.mnl.size() / 3 + 1));
  b += slab_solver_bytes(r.n_unk, r.n_trial, r.ne, so);
  b += r256(sizeof(double) * (r.ne + 1));  // energy of the initial field (inexact solves)
  if (r.c_diss > 0.0)  // D_h coefficients, FP64 and FP32
    b += r256(sizeof(double) * Mesh::kDissWords * r.ne) + r256(sizeof(float) * Mesh::kDissWords * r.ne);
  return b + 16384;  // alignment of the individual allocations
}

}  // namespace

int Server::start(Active* a) {
  Request* r = a->rq;
  a->ctx.device = ctx->device;
  a->ctx.budget = r->footprint;
  a->ctx.used = 0;
  a->ctx.chunk = arena_mem + a->off;
  a->ctx.chunk_size = r->footprint;
  a->ctx.chunk_off = 0;
  a->out.res.t_submit = r->t_submit;
  a->out.res.t_admit = now();
  a->out.res.device_bytes = (int64_t)r->footprint;
  a->out.res.state_size = r->n_state;
  STDG_HIP(hipStreamCreateWithFlags(&a->stream, hipStreamNonBlocking));
  STDG_HIP(hipEventCreateWithFlags(&a->done_ev, hipEventDisableTiming));
  a->mesh = r->mesh;
  r->mesh = nullptr;
  int rc = upload_mesh(&a->ctx, &a->mesh->m);
  if (rc != STDG_OK) return rc;
  Mesh& m = a->mesh->m;
  if (r->c_diss > 0.0 && (rc = set_dissipation(&m, r->c_diss)) != STDG_OK) return rc;
  if ((rc = dev_alloc(&a->ctx, (void**)&a->state, sizeof(double) * r->n_state)) != STDG_OK) return rc;
  if (r->src.kind && (rc = dev_alloc(&a->ctx, (void**)&a->load, sizeof(double) * r->n_unk)) != STDG_OK) return rc;
  if (!r->init.empty()) {
    STDG_HIP(hipMemcpyAsync(a->state, r->init.data(), sizeof(double) * r->n_state, hipMemcpyHostToDevice,
                            a->stream));
  } else {
    STDG_HIP(hipMemsetAsync(a->state, 0, sizeof(double) * r->n_state, a->stream));
    if (!r->mnl.empty() &&
        (rc = stdg_project_modes(a->mesh, (int32_t)(r->mnl.size() / 3), r->mnl.data(), r->abc.data(), a->state,
                                 a->stream)) != STDG_OK)
      return rc;
  }
  SlabOpts ro = so;
  if (opts.eta_rel > 0.0) {
    // per-slab budget of the iteration-error bound, relative to the initial energy
    double e0 = 0.0;
    if ((rc = stdg_energy(a->mesh, a->state, &e0, a->stream)) != STDG_OK) return rc;
    ro.eta_t_final = r->n_slabs * r->dt;
    ro.eta_tol = opts.eta_rel * std::sqrt(2.0 * e0) / std::sqrt((double)r->n_slabs);
    if (!(ro.eta_tol > 0.0)) ro.eta_tol = 0.0;  // zero field: solve to rtol
  }
  if ((rc = a->solver.init(&m, ro, a->stream)) != STDG_OK) return rc;
  a->solver.set_defer_cycles(true);  // launched by launch_pending_cycles, alone or batched
  a->solver_ready = true;
  return start_slab(a);
}

int Server::start_slab(Active* a) {
  Request* r = a->rq;
  const double ts = r->t0 + a->slab * r->dt;
  int rc;
  if (r->src.kind && (rc = stdg_load_assemble(a->mesh, &r->src, ts, r->dt, a->load, a->stream)) != STDG_OK) return rc;
  return a->solver.begin(r->dt, r->src.kind ? a->load : nullptr, a->state, nullptr);
}

// advance one request whose event has completed
int Server::step(Active* a, bool* finished_now) {
  *finished_now = false;
  if (a->finishing) {
    a->out.res.t_done = now();
    *finished_now = true;
    return STDG_OK;
  }
  bool done = false;
  int rc = a->solver.advance(&done);
  if (rc != STDG_OK) return rc;
  if (!done) return STDG_OK;
  stdg_result& res = a->out.res;
  if (a->slab == 0) res.energy_start = a->solver.energy_start;
  res.energy_end = a->solver.energy_end;
  res.iters += a->solver.iters;
  res.max_rel_res = std::max(res.max_rel_res, a->solver.rel_res);
  a->eta2 += a->solver.eta2;
  res.eta_it = std::sqrt(a->eta2);
  if (a->solver.status != STDG_OK) res.status = a->solver.status;
  res.slabs_done = ++a->slab;
  if (a->slab < a->rq->n_slabs) return start_slab(a);
  res.batched_cycles = a->solver.batched_cycles;
  // final state to the host, then done
  a->out.state.resize((size_t)a->rq->n_state);
  STDG_HIP(hipMemcpyAsync(a->out.state.data(), a->state, sizeof(double) * a->rq->n_state, hipMemcpyDeviceToHost,
                          a->stream));
  STDG_HIP(hipEventRecord(a->done_ev, a->stream));
  a->finishing = true;
  return STDG_OK;
}

void Server::retire(Active* a, int status) {
  if (a->stream) (void)hipStreamSynchronize(a->stream);
  if (status != STDG_OK)  // a batched cycle may still reach its vectors
    for (int k = 0; k < kBatchStreams; ++k)
      if (bstream[k]) (void)hipStreamSynchronize(bstream[k]);
  if (status != STDG_OK) {
    a->out.res.status = status;
    a->out.state.clear();
    if (a->out.res.t_done == 0.0) a->out.res.t_done = now();
  }
  if (a->solver_ready) a->solver.release();
  if (a->mesh) {
    release_mesh(&a->mesh->m);
    delete a->mesh;
  }
  if (a->done_ev) (void)hipEventDestroy(a->done_ev);
  if (a->stream) (void)hipStreamDestroy(a->stream);
  arena.release(a->off, a->rq->footprint);
  {
    std::lock_guard<std::mutex> lk(mu);
    finished[a->rq->ticket] = std::move(a->out);
  }
  if (a->rq->mesh) {
    release_mesh(&a->rq->mesh->m);
    delete a->rq->mesh;
  }
  delete a->rq;
  delete a;
}

bool Server::admit_one() {
  Request* r = nullptr;
  size_t off = 0;
  {
    std::lock_guard<std::mutex> lk(mu);
    if (pending.empty() || (int)active.size() >= opts.max_active) return false;
    if (!arena.alloc(pending.front()->footprint, &off)) return false;  // FIFO: wait for memory
    r = pending.front();
    pending.pop_front();
  }
  Active* a = new Active;
  a->rq = r;
  a->off = off;
  int rc = start(a);
  if (rc != STDG_OK) {
    retire(a, rc);
    return true;
  }
  active.push_back(a);
  return true;
}

// Restart cycles left pending by this tick's steps.  Requests that can share
// batched cycles (same batch key) are launched together, up to kMaxBatch per
// launch sequence; a pending cycle waits up to kBatchWait seconds while other
// requests of its key still have a step in flight (their true residuals end
// moments later), so that batches re-form after every cycle.  Everything
// else runs alone.
void Server::launch_pending_cycles() {
  constexpr double kBatchWait = 0.5e-3;
  const double t = now();
  std::map<int, std::vector<Active*>> by_key;
  std::vector<std::pair<Active*, int>> failed;
  std::map<int, int> in_flight;  // per key: requests with a step in flight
  for (Active* a : active) {
    if (a->finishing || !a->solver_ready) continue;
    const int key = opts.batch_cycles ? a->solver.batch_key() : -1;
    if (a->solver.cycle_pending()) {
      if (a->pend_since < 0.0) a->pend_since = t;
      if (key < 0) {
        int rc = a->solver.launch_pending_cycle();
        a->pend_since = -1.0;
        if (rc != STDG_OK) failed.push_back({a, rc});
      } else {
        by_key[key].push_back(a);
      }
    } else if (key >= 0) {
      in_flight[key] += 1;
    }
  }
  for (auto& kv : by_key) {
    std::vector<Active*>& v = kv.second;
    double oldest = t;
    for (Active* a : v) oldest = std::min(oldest, a->pend_since);
    // hold for partners still in flight (bounded wait)
    if (in_flight[kv.first] > 0 && (int)v.size() < kMaxBatch && t - oldest < kBatchWait) continue;
    for (size_t i0 = 0; i0 < v.size(); i0 += kMaxBatch) {
      const int n = (int)std::min<size_t>(kMaxBatch, v.size() - i0);
      int rc = STDG_OK;
      if (n == 1) {
        rc = v[i0]->solver.launch_pending_cycle();
      } else {
        if (!bstream[bnext]) {
          if (hipStreamCreateWithFlags(&bstream[bnext], hipStreamNonBlocking) != hipSuccess ||
              hipEventCreateWithFlags(&bev[bnext], hipEventDisableTiming) != hipSuccess)
            rc = fail(STDG_E_DEVICE, "serve: cannot create a batch stream");
        }
        SlabSolver* ss[kMaxBatch];
        for (int k = 0; k < n; ++k) ss[k] = &v[i0 + k]->solver;
        if (rc == STDG_OK) rc = SlabSolver::launch_cycles_batched(ss, n, bstream[bnext], bev[bnext]);
        bnext = (bnext + 1) % kBatchStreams;
      }
      for (int k = 0; k < n; ++k) {
        v[i0 + k]->pend_since = -1.0;
        if (rc != STDG_OK) failed.push_back({v[i0 + k], rc});
      }
    }
  }
  for (auto& f : failed) {
    auto it = std::find(active.begin(), active.end(), f.first);
    if (it != active.end()) active.erase(it);
    retire(f.first, f.second);
  }
}

void Server::run() {
  (void)hipSetDevice(ctx->device);
  while (!stop.load()) {
    bool progressed = false;
    while (admit_one()) progressed = true;
    for (size_t i = 0; i < active.size();) {
      Active* a = active[i];
      if (!a->finishing && a->solver_ready && a->solver.cycle_pending()) {
        ++i;  // no step in flight: its cycle waits for launch_pending_cycles
        continue;
      }
      hipError_t e = hipEventQuery(a->finishing ? a->done_ev : a->solver.event());
      if (e == hipErrorNotReady) {
        ++i;
        continue;
      }
      progressed = true;
      int rc = e == hipSuccess ? STDG_OK : hip_fail(e, "serve: device step");
      bool fin = false;
      if (rc == STDG_OK) rc = step(a, &fin);
      if (rc != STDG_OK || fin) {
        active.erase(active.begin() + (long)i);
        retire(a, rc);
        continue;
      }
      ++i;
    }
    launch_pending_cycles();
    if (!progressed) {
      if (active.empty()) {
        std::unique_lock<std::mutex> lk(mu);
        cv.wait_for(lk, std::chrono::milliseconds(2), [&] { return stop.load() || !pending.empty(); });
      } else {
        std::this_thread::yield();
      }
    }
  }
  for (Active* a : active) retire(a, STDG_E_CANCELLED);
  active.clear();
  for (int k = 0; k < kBatchStreams; ++k) {
    if (bstream[k]) (void)hipStreamSynchronize(bstream[k]);
    if (bstream[k]) (void)hipStreamDestroy(bstream[k]);
    if (bev[k]) (void)hipEventDestroy(bev[k]);
    bstream[k] = nullptr;
    bev[k] = nullptr;
  }
  std::lock_guard<std::mutex> lk(mu);
  for (Request* r : pending) {
    finished[r->ticket].res.status = STDG_E_CANCELLED;
    delete r->mesh;
    delete r;
  }
  pending.clear();
}

}  // namespace stdg

struct stdg_server {
  stdg::Server s;
};

using namespace stdg;

extern "C" {

int stdg_serve_start(stdg_ctx* ctx, const stdg_serve_opts* opts, stdg_server** out) {
  if (!ctx || !out) return fail(STDG_E_ARG, "stdg_serve_start: NULL argument");
  *out = nullptr;
  stdg_serve_opts o{};
  if (opts) o = *opts;
  if (o.hbm_budget == 0) o.hbm_budget = (size_t)16 << 30;
  if (o.max_active <= 0) o.max_active = 16;
  if (o.eta_rel < 0.0) return fail(STDG_E_ARG, "stdg_serve_start: eta_rel must be >= 0");
  stdg_solve_opts so{o.inner_prec, o.restart, o.max_iters, o.max_refine, o.rtol, o.inner_rtol, o.krylov_prec, 0.0,
                     0.0, o.use_graph};
  SlabOpts sop;
  int rc = slab_opts_from(&so, &sop);
  if (rc != STDG_OK) return rc;
  STDG_HIP(hipSetDevice(ctx->c.device));
  stdg_server* sv = new (std::nothrow) stdg_server;
  if (!sv) return fail(STDG_E_NOMEM, "stdg_serve_start: host allocation failed");
  Server& S = sv->s;
  S.ctx = &ctx->c;
  S.opts = o;
  S.so = sop;
  S.arena_size = (o.hbm_budget + 255) & ~(size_t)255;
  if ((rc = dev_alloc(S.ctx, (void**)&S.arena_mem, S.arena_size)) != STDG_OK) {
    delete sv;
    return rc;
  }
  S.arena.reset(S.arena_size);
  S.t_start = Clock::now();
  try {
    S.th = std::thread([&S] { S.run(); });
  } catch (...) {
    dev_free(S.ctx, S.arena_mem, S.arena_size);
    delete sv;
    return fail(STDG_E_NOMEM, "stdg_serve_start: cannot start the server thread");
  }
  *out = sv;
  return STDG_OK;
}

int stdg_serve_submit(stdg_server* server, const stdg_request* req, uint64_t* ticket) {
  if (!server || !req || !ticket) return fail(STDG_E_ARG, "stdg_serve_submit: NULL argument");
  Server& S = server->s;
  const double t_in = S.now();
  const stdg_mesh_desc& d = req->mesh;
  if (d.n_elements <= 0 || d.n_vertices <= 0 || !d.vertices || !d.hexes || !d.p || !d.q || !d.eps || !d.mu)
    return fail(STDG_E_ARG, "stdg_serve_submit: empty mesh or NULL array");
  if (d.n_elements > (int64_t)INT32_MAX) return fail(STDG_E_ARG, "stdg_serve_submit: too many elements");
  if (!(req->dt > 0.0) || req->n_slabs < 1) return fail(STDG_E_ARG, "stdg_serve_submit: need dt > 0 and n_slabs >= 1");
  if (req->source.kind != 0 && req->source.kind != 1) return fail(STDG_E_ARG, "stdg_serve_submit: unknown source kind");
  if (req->n_modes < 0 || (req->n_modes > 0 && (!req->mnl || !req->abc)))
    return fail(STDG_E_ARG, "stdg_serve_submit: invalid mode list");
  if (!(req->c_diss >= 0.0) || !std::isfinite(req->c_diss))
    return fail(STDG_E_ARG, "stdg_serve_submit: c_diss must be finite and >= 0");
  Request* r = new (std::nothrow) Request;
  if (!r) return fail(STDG_E_NOMEM, "stdg_serve_submit: host allocation failed");
  int rc;
  try {
    r->mesh = new stdg_mesh;
    rc = build_mesh_host(&d, &r->mesh->m);
    if (rc == STDG_OK) {
      const Mesh& m = r->mesh->m;
      r->ne = m.ne;
      r->n_unk = m.unk_off.back();
      r->n_trial = m.trial_off.back();
      r->n_state = m.state_off.back();
      if (req->n_modes > 0) {
        if (m.n_nonaffine > 0) rc = fail(STDG_E_UNSUPPORTED, "stdg_serve_submit: mode projection needs affine elements");
        r->mnl.assign(req->mnl, req->mnl + 3 * req->n_modes);
        r->abc.assign(req->abc, req->abc + 3 * req->n_modes);
      }
      if (req->init_state) {
        if (req->init_state_size != r->n_state)
          rc = fail(STDG_E_ARG, "stdg_serve_submit: init_state_size " + std::to_string(req->init_state_size) +
                                    " != the mesh's state size " + std::to_string(r->n_state));
        else
          r->init.assign(req->init_state, req->init_state + r->n_state);
      }
    }
  } catch (const std::bad_alloc&) {
    rc = fail(STDG_E_NOMEM, "stdg_serve_submit: host allocation failed");
  }
  if (rc != STDG_OK) {
    delete r->mesh;
    delete r;
    return rc;
  }
  r->t0 = req->t0;
  r->dt = req->dt;
  r->n_slabs = req->n_slabs;
  r->src = req->source;
  r->c_diss = req->c_diss;
  r->footprint = footprint_of(*r, S.so);
  if (r->footprint > S.arena_size) {
    const size_t fp = r->footprint;
    delete r->mesh;
    delete r;
    return fail(STDG_E_CAPACITY, "stdg_serve_submit: request needs " + std::to_string(fp) +
                                     " device bytes, the arena holds " + std::to_string(S.arena_size));
  }
  {
    std::lock_guard<std::mutex> lk(S.mu);
    r->ticket = S.next_ticket++;
    r->t_submit = t_in;
    S.known[r->ticket] = true;
    S.pending.push_back(r);
    *ticket = r->ticket;
  }
  S.cv.notify_one();
  return STDG_OK;
}

int stdg_serve_poll(stdg_server* server, uint64_t ticket, stdg_result* out) {
  if (!server || !out) return fail(STDG_E_ARG, "stdg_serve_poll: NULL argument");
  Server& S = server->s;
  std::lock_guard<std::mutex> lk(S.mu);
  if (!S.known.count(ticket)) return fail(STDG_E_ARG, "stdg_serve_poll: unknown or released ticket");
  auto it = S.finished.find(ticket);
  if (it == S.finished.end()) return STDG_E_NOT_READY;
  Finished& f = it->second;
  if (out->state && !f.state.empty()) {
    if (out->state_capacity < (int64_t)f.state.size())
      return fail(STDG_E_ARG, "stdg_serve_poll: state buffer too small");
    std::memcpy(out->state, f.state.data(), sizeof(double) * f.state.size());
  }
  double* keep = out->state;
  const int64_t cap = out->state_capacity;
  *out = f.res;
  out->state = keep;
  out->state_capacity = cap;
  S.finished.erase(it);
  S.known.erase(ticket);
  return STDG_OK;
}

double stdg_serve_clock(const stdg_server* server) { return server ? server->s.now() : 0.0; }

int stdg_serve_stop(stdg_server* server) {
  if (!server) return fail(STDG_E_ARG, "stdg_serve_stop: NULL argument");
  Server& S = server->s;
  S.stop.store(true);
  S.cv.notify_all();
  if (S.th.joinable()) S.th.join();
  dev_free(S.ctx, S.arena_mem, S.arena_size);
  delete server;
  return STDG_OK;
}

}  // extern "C"
