// Slab solve: find U with the l_0 block fixed to the state at t0 such that
// B_h(U, V) = L(V) for every test function (Section 3, eq. weakform;
// Section 4, eq. weakform_stabilized), by restarted GMRES preconditioned from
// the right with P = the time-derivative terms (Section 5.4,
// eq. preconditioner; block diagonal, exact on affine elements, from the
// metric at the element centre on trilinear ones).
//
// Every restart cycle starts from the true residual L - B U evaluated in
// FP64.  Inner applies run in FP64 (the plain path) or in FP32 with FP64
// orthogonalisation (classical Gram-Schmidt applied twice, fused into three
// passes over the basis, krylov.hip); with FP32 applies each cycle is one step
// of iterative refinement.  The basis is stored in FP64, or optionally in FP32
// (all sums still FP64).
// The end-of-slab state is the l_1 block of the solution (continuity in time:
// l_1(1) = 1, every other trial function vanishes at the slab end).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include <new>

#include "solver.h"

namespace stdg {

namespace {
// device scalars (mirrored to pinned host memory after each step): h and c of
// the two Gram-Schmidt passes, ||Vt_{j+1}||^2, ||r||^2, basis scales s_j, the
// correction coefficients, and the energies
constexpr int kH1 = 0, kC1 = kMaxBasis, kH2 = 2 * kMaxBasis, kC2 = 3 * kMaxBasis, kHN = 4 * kMaxBasis,
              kBeta = kHN + 1, kE0 = kHN + 2, kE1 = kHN + 3, kDE = kHN + 4, kDH = kHN + 5,
              kMirror = kHN + 6,  // entries copied back
              kS = kMirror, kY = kS + kMaxBasis + 1, kScalars = kY + kMaxBasis;

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
  if (r.restart + 1 > kMaxBasis) return fail(STDG_E_ARG, "stdg_slab_solve: restart must be <= 31");
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
  size_t b = round256((o.v32 ? sizeof(float) : sizeof(double)) * ld * (o.restart + 1)) + 4 * n8 +
             round256(sizeof(double) * nt);
  if (o.v32) b += n8;                 // residual before rounding into the basis
  if (o.f32) b += (o.v32 ? 1 : 2) * n4;
  b += round256(sizeof(double) * kMaxBasis * kMaxDotBlocks) + round256(sizeof(unsigned) * 4) +
       round256(sizeof(double) * kScalars) + round256(sizeof(double) * (2 * ne + 4));
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
  if ((rc = dev_alloc(c, (void**)&w_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&x_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&d_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&pd_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&U_, sizeof(double) * nt)) != STDG_OK) return rc;
  if (o.v32 && (rc = dev_alloc(c, (void**)&r_, n8)) != STDG_OK) return rc;
  if (o.f32) {
    if (!o.v32 && (rc = dev_alloc(c, (void**)&v32_, n4)) != STDG_OK) return rc;
    if ((rc = dev_alloc(c, (void**)&w32_, n4)) != STDG_OK) return rc;
  }
  if ((rc = dev_alloc(c, (void**)&dw_.partial, sizeof(double) * kMaxBasis * kMaxDotBlocks)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&dw_.counter, sizeof(unsigned) * 4)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&hv_, sizeof(double) * kScalars)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&etmp_, sizeof(double) * (2 * m->ne + 4))) != STDG_OK) return rc;
  STDG_HIP(hipMemsetAsync(dw_.counter, 0, sizeof(unsigned) * 4, s_));
  STDG_HIP(hipMemsetAsync(hv_, 0, sizeof(double) * kScalars, s_));
  STDG_HIP(hipHostMalloc((void**)&hb_, sizeof(double) * kScalars, hipHostMallocDefault));
  std::memset(hb_, 0, sizeof(double) * kScalars);
  STDG_HIP(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
  return STDG_OK;
}

void SlabSolver::drop_graphs() {
  for (int j = 0; j < kMaxBasis; ++j) {
    if (gexec_[j]) (void)hipGraphExecDestroy(gexec_[j]);
    gexec_[j] = nullptr;
    seen_[j] = false;
  }
}

void SlabSolver::release() {
  if (!m_) return;
  drop_graphs();
  if (cap_) (void)hipStreamDestroy(cap_);
  cap_ = nullptr;
  Ctx* c = m_->ctx;
  const size_t n8 = sizeof(double) * n_, n4 = sizeof(float) * n_;
  dev_free(c, V_, (o_.v32 ? 4 : 8) * (size_t)ld_ * (o_.restart + 1));
  dev_free(c, w_, n8);
  dev_free(c, x_, n8);
  dev_free(c, d_, n8);
  dev_free(c, pd_, n8);
  dev_free(c, U_, sizeof(double) * m_->trial_off.back());
  dev_free(c, r_, n8);
  dev_free(c, v32_, n4);
  dev_free(c, w32_, n4);
  dev_free(c, dw_.partial, sizeof(double) * kMaxBasis * kMaxDotBlocks);
  dev_free(c, dw_.counter, sizeof(unsigned) * 4);
  dev_free(c, hv_, sizeof(double) * kScalars);
  dev_free(c, etmp_, sizeof(double) * (2 * m_->ne + 4));
  if (hb_) (void)hipHostFree(hb_);
  if (ev_) (void)hipEventDestroy(ev_);
  V_ = nullptr;
  w_ = x_ = r_ = U_ = d_ = pd_ = hv_ = etmp_ = hb_ = nullptr;
  v32_ = w32_ = nullptr;
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
// and ||r'||^2 into the scalars; the Krylov residual is r = -r'
int SlabSolver::launch_true_residual() {
  int rc;
  if ((rc = layout_embed(m_, U_, x_, state_, s_)) != STDG_OK) return rc;
  double* res = o_.v32 ? r_ : (double*)basis(0);
  ApplyArgs a{m_, dt_, STDG_FP64, STDG_RESIDUAL, U_, load_, res, s_};
  if ((rc = launch_residual(a)) != STDG_OK) return rc;
  if ((rc = vec_dot(res, res, n_, hv_ + kBeta, dw_, s_)) != STDG_OK) return rc;
  if (o_.eta_tol > 0.0 && (rc = dual_norms_async(m_, dt_, res, etmp_, hv_ + kDE, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_, hv_, sizeof(double) * kMirror, hipMemcpyDeviceToHost, s_));
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
  if ((rc = energy_async(m_, state_, etmp_, hv_ + kE0, s_)) != STDG_OK) return rc;
  if ((rc = layout_guess(m_, x_, state_, s_)) != STDG_OK) return rc;
  if ((rc = launch_true_residual()) != STDG_OK) return rc;
  STDG_HIP(hipEventRecord(ev_, s_));
  phase_ = kWaitStart;
  return STDG_OK;
}

// GMRES on B P^{-1} z' = r' (z' = -z, r' = -r): V_0 = r' / beta, Vt_0 = r', s_0 = 1 / beta
int SlabSolver::start_cycle() {
  ++cycles_;
  int rc;
  if (o_.v32 && (rc = vec_store(basis(0), true, r_, n_, s_)) != STDG_OK) return rc;
  hs_[0] = 1.0 / beta_;
  hb_[kS] = hs_[0];
  STDG_HIP(hipMemcpyAsync(hv_ + kS, hb_ + kS, sizeof(double), hipMemcpyHostToDevice, s_));
  for (int i = 0; i <= o_.restart; ++i) g_[i] = 0.0;
  g_[0] = beta_;
  const double target = o_.rtol * beta0_;
  inner_target_ = o_.f32 ? std::max(o_.inner_rtol * beta_, target) : target;
  if (o_.eta_tol > 0.0) {
    // ||R||_{W'}^2 <= ||R||_2^2 max_K 1 / (dt lambda_min(G_K)): a Euclidean residual
    // below this keeps the slab's eta term below eta_tol^2 (checked exactly at the cycle end)
    const double tN = o_.eta_t_final, dt = dt_;
    const double cmax = std::max(2.0 * tN / m_->eps_min + dt * dt / (2.0 * tN * m_->eps_min),
                                 2.0 * tN / m_->mu_min + dt * dt / (2.0 * tN * m_->mu_min));
    inner_target_ = std::max(inner_target_, o_.eta_tol / std::sqrt(4.0 * cmax * m_->inv_gmin / dt));
  }
  j_ = 0;
  return launch_iteration();
}

// one Arnoldi step on w~ = B P^{-1} Vt_j (the true w is s_j w~)
// One Arnoldi iteration with basis index j: the preconditioned apply of V_j,
// the CGS2 passes producing V_{j+1}, the copy of the new scalars to the host.
// Every argument is a fixed device address of this solver (or dt), so the
// sequence can be captured once per j and replayed.
int SlabSolver::enqueue_iteration(int j) {
  int rc;
  const void* wsrc;
  if (o_.f32) {
    const float* in = (const float*)basis(j);
    if (!o_.v32) {
      if ((rc = vec_store(v32_, true, (const double*)basis(j), n_, s_)) != STDG_OK) return rc;
      in = v32_;
    }
    ApplyArgs a{m_, dt_, STDG_FP32, STDG_OPERATOR_PRECOND, in, nullptr, w32_, s_};
    if ((rc = launch_residual(a)) != STDG_OK) return rc;
    wsrc = w32_;
  } else {
    ApplyArgs a{m_, dt_, STDG_FP64, STDG_OPERATOR_PRECOND, basis(j), nullptr, w_, s_};
    if ((rc = launch_residual(a)) != STDG_OK) return rc;
    wsrc = w_;
  }
  const bool v32 = o_.v32, w32 = o_.f32;
  if ((rc = arnoldi_dot(V_, v32, ld_, j + 1, wsrc, w32, n_, hv_ + kS, hv_ + kH1, hv_ + kC1, dw_, s_)) != STDG_OK)
    return rc;
  if ((rc = arnoldi_update_dot(V_, v32, ld_, j + 1, wsrc, w32, hv_ + kC1, w_, n_, hv_ + kS, hv_ + kH2, hv_ + kC2,
                               dw_, s_)) != STDG_OK)
    return rc;
  if ((rc = arnoldi_update_norm(V_, v32, ld_, j + 1, w_, hv_ + kC2, basis(j + 1), n_, hv_ + kHN, hv_ + kS + j + 1,
                                dw_, s_)) != STDG_OK)
    return rc;
  STDG_HIP(hipMemcpyAsync(hb_, hv_, sizeof(double) * kMirror, hipMemcpyDeviceToHost, s_));
  return STDG_OK;
}

int SlabSolver::launch_iteration() {
  int rc;
  const int j = j_;
  // graphs for meshes with one kernel group (no side-stream fork); the first
  // use of an index runs directly (it also sizes any lazily allocated scratch)
  const bool graph = o_.use_graph && m_->groups.size() == 1;
  if (graph && (graph_dt_ != dt_ || graph_epoch_ != m_->epoch)) {
    // a new dt, or a mesh change that moved or replaced what the captured
    // launches read (D_h coefficients, work lists, scratch): recapture
    drop_graphs();
    graph_dt_ = dt_;
    graph_epoch_ = m_->epoch;
  }
  if (graph && seen_[j]) {
    if (!gexec_[j]) {
      // captured on a stream of the solver's own, launched on the caller's
      if (!cap_) STDG_HIP(hipStreamCreateWithFlags(&cap_, hipStreamNonBlocking));
      hipGraph_t g = nullptr;
      const hipStream_t caller = s_;
      STDG_HIP(hipStreamBeginCapture(cap_, hipStreamCaptureModeThreadLocal));
      s_ = cap_;
      rc = enqueue_iteration(j);
      s_ = caller;
      hipError_t e = hipStreamEndCapture(cap_, &g);
      if (rc != STDG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
      }
      if (e != hipSuccess) return hip_fail(e, "slab solver: capturing an Arnoldi iteration");
      e = hipGraphInstantiate(&gexec_[j], g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (e != hipSuccess) {
        gexec_[j] = nullptr;
        return hip_fail(e, "slab solver: instantiating an Arnoldi iteration");
      }
    }
    STDG_HIP(hipGraphLaunch(gexec_[j], s_));
  } else {
    if ((rc = enqueue_iteration(j)) != STDG_OK) return rc;
    seen_[j] = true;
  }
  ++iters;
  STDG_HIP(hipEventRecord(ev_, s_));
  phase_ = kWaitIter;
  return STDG_OK;
}

// y = H^{-1} g, correction d = -sum_j y_j V_j = -sum_j (y_j s_j) Vt_j (the sign
// undoes r' = -r), x += P^{-1} d, then the true residual
int SlabSolver::launch_cycle_end() {
  const int k = j_;
  double y[kMaxBasis];
  for (int i = k - 1; i >= 0; --i) {
    double t = g_[i];
    for (int l = i + 1; l < k; ++l) t -= H_[i * kMaxBasis + l] * y[l];
    y[i] = t / H_[i * kMaxBasis + i];
  }
  for (int i = 0; i < k; ++i) hb_[kY + i] = -y[i] * hs_[i];
  int rc;
  STDG_HIP(hipMemcpyAsync(hv_ + kY, hb_ + kY, sizeof(double) * k, hipMemcpyHostToDevice, s_));
  if ((rc = basis_combine(d_, V_, o_.v32, ld_, k, hv_ + kY, n_, s_)) != STDG_OK) return rc;
  if ((rc = launch_precond_scale(m_, STDG_FP64, d_, pd_, s_)) != STDG_OK) return rc;
  if ((rc = blas_axpy(x_, pd_, 1.0, n_, s_)) != STDG_OK) return rc;
  if ((rc = launch_true_residual()) != STDG_OK) return rc;
  STDG_HIP(hipEventRecord(ev_, s_));
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
      return start_cycle();
    }
    case kWaitIter: {
      const int j = j_;
      const double sj = hs_[j];
      double hcol[kMaxBasis + 1];
      const double nrm = std::sqrt(hb_[kHN]);
      for (int i = 0; i <= j; ++i) hcol[i] = sj * (hb_[kH1 + i] + hb_[kH2 + i]);
      const double hnext = sj * nrm;
      hcol[j + 1] = hnext;
      hs_[j + 1] = nrm > 0.0 ? 1.0 / nrm : 0.0;
      if (!std::isfinite(hnext)) return fail(STDG_E_NOT_CONVERGED, "stdg_slab_solve: non-finite Krylov vector");
      // Givens rotations
      for (int i = 0; i < j; ++i) {
        const double t = cs_[i] * hcol[i] + sn_[i] * hcol[i + 1];
        hcol[i + 1] = -sn_[i] * hcol[i] + cs_[i] * hcol[i + 1];
        hcol[i] = t;
      }
      const double den = std::hypot(hcol[j], hcol[j + 1]);
      cs_[j] = den > 0 ? hcol[j] / den : 1.0;
      sn_[j] = den > 0 ? hcol[j + 1] / den : 0.0;
      hcol[j] = den;
      g_[j + 1] = -sn_[j] * g_[j];
      g_[j] = cs_[j] * g_[j];
      for (int i = 0; i <= j; ++i) H_[i * kMaxBasis + j] = hcol[i];
      j_ = j + 1;
      if (std::fabs(g_[j + 1]) <= inner_target_ || hnext == 0.0 || j_ >= o_.restart || iters >= o_.max_iters)
        return launch_cycle_end();
      return launch_iteration();
    }
    case kWaitCycle: {
      beta_ = std::sqrt(hb_[kBeta]);
      refinements += 1;
      converged_ = beta_ <= o_.rtol * beta0_;
      if (o_.eta_tol > 0.0) {
        eta2 = eta_term();
        converged_ = converged_ || eta2 <= o_.eta_tol * o_.eta_tol;
      }
      if (converged_ || iters >= o_.max_iters || (o_.f32 && cycles_ >= o_.max_refine)) return launch_slab_end();
      return start_cycle();
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
