// Slab solve: find U with the l_0 block fixed to the state at t0 such that
// B_h(U, V) = L(V) for every test function (Section 3, eq. weakform;
// Section 4, eq. weakform_stabilized), by restarted GMRES preconditioned from
// the right with P = the time-derivative terms (Section 5.4,
// eq. preconditioner; block diagonal, exact on affine elements, from the
// metric at the element centre on trilinear ones).
//
// Every restart cycle starts from the true residual L - B U evaluated in
// FP64.  Inner applies run in FP64 (the plain path) or in FP32 with FP64
// Krylov vectors and FP64 orthogonalisation (classical Gram-Schmidt applied
// twice); with FP32 applies each cycle is one step of iterative refinement.
// The end-of-slab state is the l_1 block of the solution (continuity in time:
// l_1(1) = 1, every other trial function vanishes at the slab end).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>

#include "solver.h"

namespace stdg {

namespace {
// pinned host scalars: h of the two Gram-Schmidt passes, ||w||^2, ||r||^2,
// the energies, and the GMRES coefficients y on their way to the device
constexpr int kH1 = 0, kH2 = kMaxBasis, kHN = 2 * kMaxBasis, kBeta = kHN + 1, kE0 = kHN + 2, kE1 = kHN + 3,
              kY = kHN + 4, kHostScalars = kY + kMaxBasis;

size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

int slab_opts_from(const stdg_solve_opts* o, SlabOpts* out) {
  if (o->inner_prec != STDG_FP64 && o->inner_prec != STDG_FP32)
    return fail(STDG_E_ARG, "stdg_slab_solve: unknown inner precision");
  SlabOpts r;
  r.f32 = o->inner_prec == STDG_FP32;
  r.restart = o->restart > 0 ? o->restart : 10;
  if (r.restart + 1 > kMaxBasis) return fail(STDG_E_ARG, "stdg_slab_solve: restart must be <= 31");
  r.max_iters = o->max_iters > 0 ? o->max_iters : 500;
  r.max_refine = o->max_refine > 0 ? o->max_refine : 100;
  r.rtol = o->rtol > 0 ? o->rtol : 1e-10;
  r.inner_rtol = o->inner_rtol > 0 ? o->inner_rtol : 1e-4;
  *out = r;
  return STDG_OK;
}

size_t slab_solver_bytes(int64_t n, int64_t nt, int64_t ne, const SlabOpts& o) {
  const size_t n8 = round256(sizeof(double) * n), n4 = round256(sizeof(float) * n);
  size_t b = round256(sizeof(double) * n * (o.restart + 1)) + 5 * n8 + round256(sizeof(double) * nt);
  if (o.f32) b += 2 * n4;
  b += round256(sizeof(double) * kDotBlocks * kMaxBasis) + round256(sizeof(double) * kMaxBasis) +
       round256(sizeof(double) * (ne + 2));
  return b;
}

int SlabSolver::init(Mesh* m, const SlabOpts& o, hipStream_t s) {
  m_ = m;
  o_ = o;
  s_ = s;
  int rc = ensure_state_off(m);
  if (rc != STDG_OK) return rc;
  n_ = m->unk_off.back();
  const int64_t nt = m->trial_off.back();
  const size_t n8 = sizeof(double) * n_, n4 = sizeof(float) * n_;
  Ctx* c = m->ctx;
  if ((rc = dev_alloc(c, (void**)&V_, n8 * (o.restart + 1))) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&w_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&x_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&r_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&d_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&pd_, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&U_, sizeof(double) * nt)) != STDG_OK) return rc;
  if (o.f32) {
    if ((rc = dev_alloc(c, (void**)&v32_, n4)) != STDG_OK) return rc;
    if ((rc = dev_alloc(c, (void**)&w32_, n4)) != STDG_OK) return rc;
  }
  if ((rc = dev_alloc(c, (void**)&partial_, sizeof(double) * kDotBlocks * kMaxBasis)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&hdev_, sizeof(double) * kMaxBasis)) != STDG_OK) return rc;
  if ((rc = dev_alloc(c, (void**)&etmp_, sizeof(double) * (m->ne + 2))) != STDG_OK) return rc;
  STDG_HIP(hipHostMalloc((void**)&hb_, sizeof(double) * kHostScalars, hipHostMallocDefault));
  std::memset(hb_, 0, sizeof(double) * kHostScalars);
  STDG_HIP(hipEventCreateWithFlags(&ev_, hipEventDisableTiming));
  return STDG_OK;
}

void SlabSolver::release() {
  if (!m_) return;
  Ctx* c = m_->ctx;
  const size_t n8 = sizeof(double) * n_, n4 = sizeof(float) * n_;
  dev_free(c, V_, n8 * (o_.restart + 1));
  dev_free(c, w_, n8);
  dev_free(c, x_, n8);
  dev_free(c, r_, n8);
  dev_free(c, d_, n8);
  dev_free(c, pd_, n8);
  dev_free(c, U_, sizeof(double) * m_->trial_off.back());
  dev_free(c, v32_, n4);
  dev_free(c, w32_, n4);
  dev_free(c, partial_, sizeof(double) * kDotBlocks * kMaxBasis);
  dev_free(c, hdev_, sizeof(double) * kMaxBasis);
  dev_free(c, etmp_, sizeof(double) * (m_->ne + 2));
  if (hb_) (void)hipHostFree(hb_);
  if (ev_) (void)hipEventDestroy(ev_);
  V_ = w_ = x_ = r_ = U_ = d_ = pd_ = partial_ = hdev_ = etmp_ = hb_ = nullptr;
  v32_ = w32_ = nullptr;
  ev_ = nullptr;
  m_ = nullptr;
  phase_ = kIdle;
}

// r = L - B U(x) in FP64, and ||r||^2 into the pinned scalars
int SlabSolver::launch_true_residual() {
  int rc;
  if ((rc = layout_embed(m_, U_, x_, state_, s_)) != STDG_OK) return rc;
  ApplyArgs a{m_, dt_, STDG_FP64, STDG_RESIDUAL, U_, load_, r_, s_};
  if ((rc = launch_residual(a)) != STDG_OK) return rc;
  if ((rc = blas_scale(r_, r_, -1.0, n_, s_)) != STDG_OK) return rc;
  if ((rc = blas_multi_dot(r_, n_, 1, r_, false, n_, partial_, hdev_, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_ + kBeta, hdev_, sizeof(double), hipMemcpyDeviceToHost, s_));
  return STDG_OK;
}

int SlabSolver::begin(double dt, const double* load, double* state, double* slab_U) {
  dt_ = dt;
  load_ = load;
  state_ = state;
  slabU_ = slab_U;
  status = STDG_OK;
  iters = refinements = cycles_ = 0;
  rel_res = energy_start = energy_end = 0.0;
  converged_ = false;
  int rc;
  if ((rc = energy_async(m_, state_, etmp_, etmp_ + m_->ne, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_ + kE0, etmp_ + m_->ne, sizeof(double), hipMemcpyDeviceToHost, s_));
  if ((rc = layout_guess(m_, x_, state_, s_)) != STDG_OK) return rc;
  if ((rc = launch_true_residual()) != STDG_OK) return rc;
  STDG_HIP(hipEventRecord(ev_, s_));
  phase_ = kWaitStart;
  return STDG_OK;
}

int SlabSolver::start_cycle() {
  ++cycles_;
  int rc;
  if ((rc = blas_scale(V_, r_, 1.0 / beta_, n_, s_)) != STDG_OK) return rc;
  for (int i = 0; i <= o_.restart; ++i) g_[i] = 0.0;
  g_[0] = beta_;
  const double target = o_.rtol * beta0_;
  inner_target_ = o_.f32 ? std::max(o_.inner_rtol * beta_, target) : target;
  j_ = 0;
  return launch_iteration();
}

int SlabSolver::launch_iteration() {
  int rc;
  const int j = j_;
  double* Vj = V_ + (int64_t)j * n_;
  const void* wsrc;
  if (o_.f32) {
    if ((rc = blas_to_f32(v32_, Vj, 1.0, n_, s_)) != STDG_OK) return rc;
    ApplyArgs a{m_, dt_, STDG_FP32, STDG_OPERATOR_PRECOND, v32_, nullptr, w32_, s_};
    if ((rc = launch_residual(a)) != STDG_OK) return rc;
    wsrc = w32_;
  } else {
    ApplyArgs a{m_, dt_, STDG_FP64, STDG_OPERATOR_PRECOND, Vj, nullptr, w_, s_};
    if ((rc = launch_residual(a)) != STDG_OK) return rc;
    wsrc = w_;
  }
  ++iters;
  // classical Gram-Schmidt, twice
  if ((rc = blas_multi_dot(V_, n_, j + 1, wsrc, o_.f32, n_, partial_, hdev_, s_)) != STDG_OK) return rc;
  if ((rc = blas_update(w_, wsrc, o_.f32, V_, n_, j + 1, hdev_, n_, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_ + kH1, hdev_, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s_));
  if ((rc = blas_multi_dot(V_, n_, j + 1, w_, false, n_, partial_, hdev_, s_)) != STDG_OK) return rc;
  if ((rc = blas_update(w_, w_, false, V_, n_, j + 1, hdev_, n_, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_ + kH2, hdev_, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s_));
  if ((rc = blas_multi_dot(w_, n_, 1, w_, false, n_, partial_, hdev_, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_ + kHN, hdev_, sizeof(double), hipMemcpyDeviceToHost, s_));
  STDG_HIP(hipEventRecord(ev_, s_));
  phase_ = kWaitIter;
  return STDG_OK;
}

// y = H^{-1} g, correction d = sum_j y_j V_j, x += P^{-1} d, then the true residual
int SlabSolver::launch_cycle_end() {
  const int k = j_;
  double* y = hb_ + kY;
  for (int i = k - 1; i >= 0; --i) {
    double t = g_[i];
    for (int l = i + 1; l < k; ++l) t -= H_[i * kMaxBasis + l] * y[l];
    y[i] = t / H_[i * kMaxBasis + i];
  }
  int rc;
  STDG_HIP(hipMemcpyAsync(hdev_, y, sizeof(double) * k, hipMemcpyHostToDevice, s_));
  if ((rc = blas_lincomb(d_, false, V_, n_, k, hdev_, n_, s_)) != STDG_OK) return rc;
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
  if ((rc = energy_async(m_, state_, etmp_, etmp_ + m_->ne, s_)) != STDG_OK) return rc;
  STDG_HIP(hipMemcpyAsync(hb_ + kE1, etmp_ + m_->ne, sizeof(double), hipMemcpyDeviceToHost, s_));
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
      if (converged_ || iters >= o_.max_iters) return launch_slab_end();
      return start_cycle();
    }
    case kWaitIter: {
      const int j = j_;
      double hcol[kMaxBasis + 1];
      const double hnext = std::sqrt(hb_[kHN]);
      for (int i = 0; i <= j; ++i) hcol[i] = hb_[kH1 + i] + hb_[kH2 + i];
      hcol[j + 1] = hnext;
      if (!std::isfinite(hnext)) return fail(STDG_E_NOT_CONVERGED, "stdg_slab_solve: non-finite Krylov vector");
      int rc;
      if (hnext > 0.0 && (rc = blas_scale(V_ + (int64_t)(j + 1) * n_, w_, 1.0 / hnext, n_, s_)) != STDG_OK) return rc;
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
  SlabSolver S;
  rc = S.init(m, o, s);
  if (rc == STDG_OK) rc = S.begin(dt, load_dev, state_dev, slab_U_dev);
  bool done = false;
  while (rc == STDG_OK && !done) {
    hipError_t e = hipEventSynchronize(S.event());
    if (e != hipSuccess) {
      rc = hip_fail(e, "stdg_slab_solve: waiting for the device");
      break;
    }
    rc = S.advance(&done);
  }
  info->iters = S.iters;
  info->refinements = S.refinements;
  info->rel_res = S.rel_res;
  info->energy_start = S.energy_start;
  info->energy_end = S.energy_end;
  if (rc == STDG_OK && S.status != STDG_OK)
    rc = fail(S.status, "stdg_slab_solve: relative residual " + std::to_string(S.rel_res) + " after " +
                            std::to_string(S.iters) + " iterations");
  (void)hipStreamSynchronize(s);
  S.release();
  return rc;
}
