// Slab solve: find U with the l_0 block fixed to the state at t0 such that
// B_h(U, V) = L(V) for every test function (Section 3, eq. weakform;
// Section 4, eq. weakform_stabilized), by restarted GMRES preconditioned from
// the right with P = the time-derivative terms (Section 5.4,
// eq. preconditioner; block diagonal, exact on affine elements, from the
// metric at the element centre on trilinear ones).
//
// Every restart cycle starts from the true residual L - B U evaluated in
// FP64.  Inner applies run in FP64 (the plain path) or in FP32 with FP64
// orthogonalisation (classical Gram-Schmidt applied twice, the second
// projection delayed into the next iteration: two passes over the basis per
// iteration, krylov.hip); with FP32 applies each cycle is one step of
// iterative refinement.  The basis is stored in FP64, or optionally in FP32
// (all sums still FP64).  The Hessenberg least-squares problem is updated on
// the device, so the host waits once per restart cycle.
// The end-of-slab state is the l_1 block of the solution (continuity in time:
// l_1(1) = 1, every other trial function vanishes at the slab end).
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstring>
#include <string>

#include <new>

#include "solver.h"

namespace stdg {

namespace {
// device scalars (mirrored to pinned host memory at every step): ||r||^2 of
// the true residual, the energies, the dual norms of the residual
constexpr int kBeta = 0, kE0 = 1, kE1 = 2, kDE = 3, kDH = 4, kMirror = 5, kScalars = 8;
// bytes of CycleCtl copied each way: the parameters (host to device), and
// the parameters with the counters (device to host)
constexpr size_t kCtlParams = offsetof(CycleCtl, active), kCtlHead = offsetof(CycleCtl, nu);

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

int slab_opts_from(const stdg_solve_opts* o, SlabOpts* out) {
  if (o->inner_prec != STDG_FP64 && o->inner_prec != STDG_FP32)
    return fail(STDG_E_ARG, "stdg_slab_solve: unknown inner precision");
  if (o->krylov_prec != STDG_FP64 && o->krylov_prec != STDG_FP32)
    return fail(STDG_E_ARG, "stdg_slab_solve: unknown Krylov basis precision");
  if (o->krylov_prec == STDG_FP32 && o->inner_prec != STDG_FP32)
    return fail(STDG_E_ARG, "stdg_slab_solve: an FP32 Krylov basis needs FP32 inner applies");
  SlabOpts r;
  r.f32 = o->inner_prec == STDG_FP32;
  r.v32 = o->krylov_prec == STDG_FP32;
  r.restart = o->restart > 0 ? o->restart : 10;
  if (r.restart + 1 > kMaxBasis) return fail(STDG_E_ARG, "stdg_slab_solve: restart must be <= 15");
  r.max_iters = o->max_iters > 0 ? o->max_iters : 500;
  r.max_refine = o->max_refine > 0 ? o->max_refine : 100;
  r.rtol = o->rtol > 0 ? o->rtol : 1e-10;
  r.inner_rtol = o->inner_rtol > 0 ? o->inner_rtol : 1e-4;
  if (o->eta_tol < 0.0 || (o->eta_tol > 0.0 && !(o->eta_t_final > 0.0)))
    return fail(STDG_E_ARG, "stdg_slab_solve: eta_tol needs eta_t_final > 0");
  r.eta_tol = o->eta_tol;
  r.eta_t_final = o->eta_t_final;
  r.use_graph = o->use_graph != 0;
  *out = r;
  return STDG_OK;
}

size_t slab_solver_bytes(int64_t n, int64_t nt, int64_t ne, const SlabOpts& o) {
  const size_t n8 = round256(sizeof(double) * n), n4 = round256(sizeof(float) * n);
  const int64_t ld = (n + 63) / 64 * 64;
  size_t b = round256((o.v32 ? sizeof(float) : sizeof(double)) * ld * (o.restart + 1));
  b += o.v32 ? n4 : n8;              // pending vector
  b += o.f32 ? n4 : n8;              // apply output
  if (o.f32 && !o.v32) b += n4;      // FP32 copy of the apply input
  b += 3 * n8 + round256(sizeof(double) * nt);  // iterate, correction, scaled correction; trial vector
  if (o.v32) b += n8;                // residual before it becomes the FP32 start vector
  b += round256(sizeof(double) * kMaxBasis * kMaxDotBlocks) + round256(sizeof(unsigned) * 4) +
       round256(sizeof(double) * kScalars) + round256(sizeof(double) * (2 * ne + 4)) + round256(sizeof(CycleCtl));
  return b;
}

int SlabSolver::init(Mesh* m, const SlabOpts& o, hipStream_t s) {
  m_ = m;
  o_ = o;
  s_ = s;
  int rc = ensure_state_off(m);
  if (rc != STDG_OK) return rc;
  n_ = m->unk_off.back();
  ld_ = (n_ + 63) / 64 * 64;
  const int64_t nt = m->trial_off.back();
  const size_t n8 = sizeof(double) * n_, n4 = sizeof(float) * n_;
  Ctx* c = m->ctx;
  if ((rc = dev_alloc(c, &V_, (o.v32 ? 4 : 8) * (size_t)ld_ * (o.restart + 1))) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, &w_, o.v32 ? n4 : n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, &z_, o.f32 ? n4 : n8)) != STDG_OK) return rc;
  if (o.f32 && !o.v32 && (rc = dev_alloc(c, (void**)&w32_, n4)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&x_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&d_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&pd_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&U_, sizeof(double) * nt)) != STDG_OK) return rc;
  if (o.v32 && (rc = dev_alloc(c, (void**)&r_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&dw_.partial, sizeof(double) * kMaxBasis * kMaxDotBlocks)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&dw_.counter, sizeof(unsigned) * 4)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&hv_, sizeof(double) * kScalars)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&etmp_, sizeof(double) * (2 * m->ne + 4))) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&ctl_, sizeof(CycleCtl))) != STDG_OK) return rc;
  STDG_HIP(hipMemsetAsync(dw_.counter, 0, sizeof(unsigned) * 4, s_));
  STDG_HIP(hipMemsetAsync(hv_, 0, sizeof(double) * kScalars, s_));
  STDG_HIP(hipMemsetAsync(ctl_, 0, sizeof(CycleCtl), s_));
  STDG_HIP(hipHostMalloc((void**)&hb_, sizeof(double) * kScalars, hipHostMallocDefault));
  std::memset(hb_, 0, sizeof(double) * kScalars);
  STDG_HIP(hipHostMalloc((void**)&hctl_, kCtlHead, hipHostMallocDefault));
  std::memset(hctl_, 0, kCtlHead);
  STDG_HIP(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
  return STDG_OK;
}

void SlabSolver::drop_graphs() {
  if (gexec_) (void)hipGraphExecDestroy(gexec_);
  gexec_ = nullptr;
  seen_ = false;
}

void SlabSolver::release() {
  if (!m_) return;
  drop_graphs();
  if (cap_) (void)hipStreamDestroy(cap_);
  cap_ = nullptr;
  Ctx* c = m_->ctx;
  const size_t n8 = sizeof(double) * n_, n4 = sizeof(float) * n_;
  dev_free(c, V_, (o_.v32 ? 4 : 8) * (size_t)ld_ * (o_.restart + 1));
  dev_free(c, w_, o_.v32 ? n4 : n8);
  dev_free(c, z_, o_.f32 ? n4 : n8);
  dev_free(c, w32_, n4);
  dev_free(c, x_, n8);
  dev_free(c, d_, n8);
  dev_free(c, pd_, n8);
  dev_free(c, U_, sizeof(double) * m_->trial_off.back());
  dev_free(c, r_, n8);
  dev_free(c, dw_.partial, sizeof(double) * kMaxBasis * kMaxDotBlocks);
  dev_free(c, dw_.counter, sizeof(unsigned) * 4);
  dev_free(c, hv_, sizeof(double) * kScalars);
  dev_free(c, etmp_, sizeof(double) * (2 * m_->ne + 4));
  dev_free(c, ctl_, sizeof(CycleCtl));
  if (hb_) (void)hipHostFree(hb_);
  if (hctl_) (void)hipHostFree(hctl_);
  if (ev_) (void)hipEventDestroy(ev_);
  V_ = w_ = z_ = nullptr;
  w32_ = nullptr;
  x_ = r_ = U_ = d_ = pd_ = hv_ = etmp_ = hb_ = nullptr;
  ctl_ = hctl_ = nullptr;
  dw_ = DotWork();
  ev_ = nullptr;
  m_ = nullptr;
  phase_ = kIdle;
}

int SlabSolver::rebind(const SlabOpts& o, hipStream_t s) {
  o_ = o;
  s_ = s;
  phase_ = kIdle;
  STDG_HIP(hipMemsetAsync(dw_.counter, 0, sizeof(unsigned) * 4, s_));
  STDG_HIP(hipMemsetAsync(hv_, 0, sizeof(double) * kScalars, s_));
  return STDG_OK;
}

void release_cached_solver(Mesh* m) {
  if (!m->solver) return;
  m->solver->release();
  delete m->solver;
  m->solver = nullptr;
}

// r' = B U(x) - L in FP64 (into the first basis slot when the basis is FP64),
// ||r'||^2 and (inexact solves) its dual norms into the scalars, the scalars
// and the cycle counters to the host, and the step's event; the Krylov
// residual is r = -r'
int SlabSolver::launch_true_residual() {
  int rc;
  if ((rc = layout_embed(m_, U_, x_, state_, s_)) != STDG_OK) return rc;
  double* res = o_.v32 ? r_ : (double*)basis(0);
  ApplyArgs a{m_, dt_, STDG_FP64, STDG_RESIDUAL, U_, load_, res, s_};
  if ((rc = launch_residual(a)) != STDG_OK) return rc;
  if ((rc = vec_dot(res, res, n_, hv_ + kBeta, dw_, s_)) != STDG_OK) return rc;
  if (o_.eta_tol > 0.0 && (rc = dual_norms_async(m_, dt_, res, etmp_, hv_ + kDE, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_, hv_, sizeof(double) * kMirror, hipMemcpyDeviceToHost, s_));
  STDG_HIP(hipMemcpyAsync(hctl_, ctl_, kCtlHead, hipMemcpyDeviceToHost, s_));
  STDG_HIP(hipEventRecord(ev_, s_));
  return STDG_OK;
}

// the slab's term of the iteration-error bound (eq. a_posteriori:iteration, as printed):
// 4 [(2 t_N / eps_min + dt^2 / (2 t_N eps_min)) ||R_E||^2 + (same with mu) ||R_H||^2]
double SlabSolver::eta_term() const {
  const double tN = o_.eta_t_final, dt = dt_;
  const double cE = 2.0 * tN / m_->eps_min + dt * dt / (2.0 * tN * m_->eps_min);
  const double cH = 2.0 * tN / m_->mu_min + dt * dt / (2.0 * tN * m_->mu_min);
  return 4.0 * (cE * hb_[kDE] + cH * hb_[kDH]);
}

int SlabSolver::begin(double dt, const double* load, double* state, double* slab_U) {
  dt_ = dt;
  load_ = load;
  state_ = state;
  slabU_ = slab_U;
  status = STDG_OK;
  iters = refinements = cycles_ = 0;
  rel_res = energy_start = energy_end = eta2 = 0.0;
  converged_ = false;
  int rc;
  // the slab's iteration counter starts at zero (the whole head of the control block)
  std::memset(hctl_, 0, kCtlHead);
  STDG_HIP(hipMemcpyAsync(ctl_, hctl_, kCtlHead, hipMemcpyHostToDevice, s_));
  if ((rc = energy_async(m_, state_, etmp_, hv_ + kE0, s_)) != STDG_OK) return rc;
  if ((rc = layout_guess(m_, x_, state_, s_)) != STDG_OK) return rc;
  if ((rc = launch_true_residual()) != STDG_OK) return rc;
  phase_ = kWaitStart;
  return STDG_OK;
}

// One restart cycle on the device: V_0 = r' / |r'|, up to `restart` Arnoldi
// iterations on B P^{-1} (each: the preconditioned apply of the pending
// vector, pass 1, pass 2; kernels of iterations past the cycle's end return
// at once), y = R^{-1} g, correction d = -sum_l y_l V_l (the sign undoes
// r' = -r), x += P^{-1} d.  Every argument is a fixed device address of this
// solver (or dt), so the sequence can be captured once and replayed.
int SlabSolver::enqueue_cycle() {
  int rc;
  const bool f32 = o_.f32, v32 = o_.v32;
  const double* res = v32 ? r_ : (const double*)basis(0);
  if ((rc = cycle_start(res, hv_ + kBeta, basis(0), v32, (f32 && !v32) ? w32_ : nullptr, n_, ctl_, s_)) != STDG_OK)
    return rc;
  for (int j = 0; j < o_.restart; ++j) {
    const void* in = j == 0 ? ((f32 && !v32) ? (const void*)w32_ : basis(0))
                            : ((f32 && !v32) ? (const void*)w32_ : (const void*)w_);
    ApplyArgs a{m_, dt_, f32 ? STDG_FP32 : STDG_FP64, STDG_OPERATOR_PRECOND, in, nullptr, z_, s_};
    a.skip = &ctl_->active;
    if ((rc = launch_residual(a)) != STDG_OK) return rc;
    if ((rc = arnoldi_pass1(V_, v32, ld_, j, z_, f32, w_, n_, ctl_, dw_, s_)) != STDG_OK) return rc;
    if ((rc = arnoldi_pass2(V_, v32, ld_, j, z_, f32, w_, (f32 && !v32) ? w32_ : nullptr, n_, ctl_, dw_, s_)) !=
        STDG_OK)
      return rc;
  }
  if ((rc = cycle_least_squares(ctl_, s_)) != STDG_OK) return rc;
  if ((rc = basis_combine(d_, V_, v32, ld_, o_.restart, &ctl_->k, ctl_->y, n_, s_)) != STDG_OK) return rc;
  if ((rc = launch_precond_scale(m_, STDG_FP64, d_, pd_, s_)) != STDG_OK) return rc;
  if ((rc = blas_axpy(x_, pd_, 1.0, n_, s_)) != STDG_OK) return rc;
  return STDG_OK;
}

int SlabSolver::launch_cycle() {
  int rc = prepare_cycle();
  if (rc != STDG_OK) return rc;
  if (defer_) {
    phase_ = kWantCycle;
    return STDG_OK;
  }
  return run_cycle();
}

int SlabSolver::launch_pending_cycle() {
  if (phase_ != kWantCycle) return fail(STDG_E_ARG, "slab solver: no restart cycle pending");
  return run_cycle();
}

int SlabSolver::batch_key() const {
  if (!o_.f32 || !batchable_mesh(m_)) return -1;
  for (const Group& g : m_->groups)
    if (g.count > 0) return ((g.a * 8 + g.q) * 2 + (o_.v32 ? 1 : 0)) * 64 + o_.restart;
  return -1;
}

int SlabSolver::launch_cycles_batched(SlabSolver* const* S, int count, hipStream_t bs, hipEvent_t bev) {
  if (count < 1 || count > kMaxBatch) return fail(STDG_E_ARG, "batched cycles: 1 to kMaxBatch solvers");
  const int key = S[0]->batch_key();
  for (int i = 0; i < count; ++i)
    if (!S[i]->cycle_pending() || key < 0 || S[i]->batch_key() != key)
      return fail(STDG_E_ARG, "batched cycles: solvers not pending or not of one batch key");
  const SlabOpts& o = S[0]->o_;
  const bool f32 = o.f32, v32 = o.v32;
  CycleSeg seg[kMaxBatch];
  BatchApplyArgs app[kMaxBatch];
  for (int i = 0; i < count; ++i) {
    SlabSolver& t = *S[i];
    // the solver's previous step has completed (its event was seen): the wait is for order only
    STDG_HIP(hipStreamWaitEvent(bs, t.ev_, 0));
    STDG_HIP(hipMemcpyAsync(t.ctl_, t.hctl_, kCtlParams, hipMemcpyHostToDevice, bs));
    CycleSeg& c = seg[i];
    c.V = t.V_;
    c.ldv = t.ld_;
    c.z = t.z_;
    c.w = t.w_;
    c.w32 = (f32 && !v32) ? t.w32_ : nullptr;
    c.r = v32 ? t.r_ : (const double*)t.basis(0);
    c.norm2 = t.hv_ + kBeta;
    c.out = t.d_;
    c.n = t.n_;
    c.ctl = t.ctl_;
    c.dw = t.dw_;
    app[i] = BatchApplyArgs{t.m_, t.dt_, nullptr, t.z_, &t.ctl_->active};
  }
  // the steps of enqueue_cycle, each one launch for all solvers
  int rc;
  if ((rc = cycle_start_batch(seg, count, v32, bs)) != STDG_OK) return rc;
  for (int j = 0; j < o.restart; ++j) {
    for (int i = 0; i < count; ++i) {
      SlabSolver& t = *S[i];
      app[i].x = (f32 && !v32) ? (const void*)t.w32_ : (j == 0 ? t.basis(0) : (const void*)t.w_);
    }
    if ((rc = launch_residual_batch(app, count, f32 ? STDG_FP32 : STDG_FP64, bs)) != STDG_OK) return rc;
    if ((rc = arnoldi_pass1_batch(seg, count, v32, f32, j, bs)) != STDG_OK) return rc;
    if ((rc = arnoldi_pass2_batch(seg, count, v32, f32, j, bs)) != STDG_OK) return rc;
  }
  if ((rc = cycle_least_squares_batch(seg, count, bs)) != STDG_OK) return rc;
  if ((rc = basis_combine_batch(seg, count, v32, o.restart, bs)) != STDG_OK) return rc;
  for (int i = 0; i < count; ++i) {
    SlabSolver& t = *S[i];
    if ((rc = launch_precond_scale(t.m_, STDG_FP64, t.d_, t.pd_, bs)) != STDG_OK) return rc;
    if ((rc = blas_axpy(t.x_, t.pd_, 1.0, t.n_, bs)) != STDG_OK) return rc;
  }
  STDG_HIP(hipEventRecord(bev, bs));
  for (int i = 0; i < count; ++i) {
    SlabSolver& t = *S[i];
    STDG_HIP(hipStreamWaitEvent(t.s_, bev, 0));
    if ((rc = t.launch_true_residual()) != STDG_OK) return rc;
    t.phase_ = kWaitCycle;
    t.batched_cycles += 1;
  }
  return STDG_OK;
}

int SlabSolver::prepare_cycle() {
  ++cycles_;
  // the inner target: rtol of the initial residual (FP64 applies), or for
  // FP32 applies inner_rtol of this cycle's residual, but never below the
  // outer target (each cycle is one step of iterative refinement)
  const double target = o_.rtol * beta0_;
  double inner = o_.f32 ? std::max(o_.inner_rtol * beta_, target) : target;
  if (o_.eta_tol > 0.0) {
    // ||R||_{W'}^2 <= ||R||_2^2 max_K 1 / (dt lambda_min(G_K)): a Euclidean residual
    // below this keeps the slab's eta term below eta_tol^2 (checked exactly at the cycle end)
    const double tN = o_.eta_t_final, dt = dt_;
    const double cmax = std::max(2.0 * tN / m_->eps_min + dt * dt / (2.0 * tN * m_->eps_min),
                                 2.0 * tN / m_->mu_min + dt * dt / (2.0 * tN * m_->mu_min));
    inner = std::max(inner, o_.eta_tol / std::sqrt(4.0 * cmax * m_->inv_gmin / dt));
  }
  hctl_->target = inner;
  hctl_->restart = o_.restart;
  hctl_->max_iters = o_.max_iters;
  return STDG_OK;
}

int SlabSolver::run_cycle() {
  STDG_HIP(hipMemcpyAsync(ctl_, hctl_, kCtlParams, hipMemcpyHostToDevice, s_));
  int rc;
  // the whole cycle as one captured graph, from the second cycle on (the first
  // runs directly: it also sizes any lazily allocated scratch)
  if (o_.use_graph && (graph_dt_ != dt_ || graph_epoch_ != m_->epoch)) {
    // a new dt, or a mesh change that moved or replaced what the captured
    // launches read (D_h coefficients, work lists, launch variants, scratch)
    drop_graphs();
    graph_dt_ = dt_;
    graph_epoch_ = m_->epoch;
  }
  if (o_.use_graph && seen_) {
    if (!gexec_) {
      // captured on a stream of the solver's own, launched on the caller's
      if (!cap_) STDG_HIP(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      const hipStream_t caller = s_;
      STDG_HIP(hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal));
      s_ = cap_;
      rc = enqueue_cycle();
      s_ = caller;
      hipError_t e = hipStreamEndCapture(cap_, &g);
      if (rc != STDG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return hip_fail(e, "slab solver: capturing a restart cycle");
      e = hipGraphInstantiate(&gexec_, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        gexec_ = nullptr;
        return hip_fail(e, "slab solver: instantiating a restart cycle");
      }
    }
    STDG_HIP(hipGraphLaunch(gexec_, s_));
  } else {
    if ((rc = enqueue_cycle()) != STDG_OK) return rc;
    seen_ = true;
  }
  if ((rc = launch_true_residual()) != STDG_OK) return rc;
  phase_ = kWaitCycle;
  return STDG_OK;
}

int SlabSolver::launch_slab_end() {
  int rc;
  if (slabU_ && (rc = layout_embed(m_, slabU_, x_, state_, s_)) != STDG_OK) return rc;
  if ((rc = layout_level(m_, state_, x_, 1, s_)) != STDG_OK) return rc;
  if ((rc = energy_async(m_, state_, etmp_, hv_ + kE1, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_, hv_, sizeof(double) * kMirror, hipMemcpyDeviceToHost, s_));
  STDG_HIP(hipEventRecord(ev_, s_));
  phase_ = kWaitEnd;
  return STDG_OK;
}

int SlabSolver::advance(bool* done) {
  *done = false;
  switch (phase_) {
    case kWaitStart: {
      energy_start = hb_[kE0];
      beta0_ = beta_ = std::sqrt(hb_[kBeta]);
      refinements = 1;
      if (!std::isfinite(beta0_)) return fail(STDG_E_ARG, "stdg_slab_solve: non-finite initial residual");
      converged_ = beta0_ == 0.0;
      if (o_.eta_tol > 0.0) {
        eta2 = eta_term();
        converged_ = converged_ || eta2 <= o_.eta_tol * o_.eta_tol;
      }
      if (converged_ || iters >= o_.max_iters) return launch_slab_end();
      return launch_cycle();
    }
    case kWaitCycle: {
      iters = hctl_->iters;
      if (hctl_->bad) return fail(STDG_E_NOT_CONVERGED, "stdg_slab_solve: non-finite Krylov vector");
      beta_ = std::sqrt(hb_[kBeta]);
      refinements += 1;
      if (!std::isfinite(beta_)) return fail(STDG_E_NOT_CONVERGED, "stdg_slab_solve: non-finite residual");
      converged_ = beta_ <= o_.rtol * beta0_;
      if (o_.eta_tol > 0.0) {
        eta2 = eta_term();
        converged_ = converged_ || eta2 <= o_.eta_tol * o_.eta_tol;
      }
      if (converged_ || iters >= o_.max_iters || (o_.f32 && cycles_ >= o_.max_refine) || beta_ == 0.0)
        return launch_slab_end();
      return launch_cycle();
    }
    case kWaitEnd: {
      energy_end = hb_[kE1];
      rel_res = beta0_ > 0 ? beta_ / beta0_ : 0.0;
      status = converged_ ? STDG_OK : STDG_E_NOT_CONVERGED;
      phase_ = kIdle;
      *done = true;
      return STDG_OK;
    }
    default:
      return fail(STDG_E_ARG, "slab solver: advance() without a step in flight");
  }
}

}  // namespace stdg

using namespace stdg;

extern "C" int stdg_slab_solve(const stdg_mesh* mesh, double t0, double dt, const double* load_dev,
                               const stdg_solve_opts* opts, double* state_dev, double* slab_U_dev,
                               stdg_solve_info* info, void* stream) {
  (void)t0;
  if (!mesh || !opts || !state_dev || !info) return fail(STDG_E_ARG, "stdg_slab_solve: NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(STDG_E_ARG, "stdg_slab_solve: dt must be finite and > 0");
  SlabOpts o;
  int rc = slab_opts_from(opts, &o);
  if (rc != STDG_OK) return rc;
  std::memset(info, 0, sizeof(*info));
  Mesh* m = const_cast<Mesh*>(&mesh->m);
  hipStream_t s = (hipStream_t)stream;
  // the mesh's cached solver (allocated on the first call, kept until the
  // mesh is freed or the precisions / restart change), or a private one if
  // another thread holds it
  SlabSolver own;
  SlabSolver* S = &own;
  bool expected = false;
  const bool cached = m->solver_busy.compare_exchange_strong(expected, true);
  if (cached) {
    if (m->solver && !m->solver->compatible(o)) release_cached_solver(m);
    if (m->solver) {
      rc = m->solver->rebind(o, s);
    } else {
      m->solver = new (std::nothrow) SlabSolver;
      rc = m->solver ? m->solver->init(m, o, s) : fail(STDG_E_NOMEM, "stdg_slab_solve: host allocation failed");
      if (rc != STDG_OK) release_cached_solver(m);
    }
    S = m->solver;
  } else {
    rc = own.init(m, o, s);
  }
  if (rc == STDG_OK) rc = S->begin(dt, load_dev, state_dev, slab_U_dev);
  bool done = false;
  while (rc == STDG_OK && !done) {
    hipError_t e = hipEventSynchronize(S->event());
    if (e != hipSuccess) {
      rc = hip_fail(e, "stdg_slab_solve: waiting for the device");
      break;
    }
    rc = S->advance(&done);
  }
  if (S) {
    info->iters = S->iters;
    info->refinements = S->refinements;
    info->rel_res = S->rel_res;
    info->energy_start = S->energy_start;
    info->energy_end = S->energy_end;
    info->eta2 = S->eta2;
    if (rc == STDG_OK && S->status != STDG_OK)
      rc = fail(S->status, "stdg_slab_solve: relative residual " + std::to_string(S->rel_res) + " after " +
                               std::to_string(S->iters) + " iterations");
  }
  (void)hipStreamSynchronize(s);
  if (cached) {
    // a solver left mid-step by an error is not reused
    if (rc != STDG_OK && rc != STDG_E_NOT_CONVERGED) release_cached_solver(m);
    m->solver_busy.store(false);
  } else {
    own.release();
  }
  return rc;
}
