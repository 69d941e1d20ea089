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
#include <cmath>
#include <cstring>
#include <vector>

#include "solver.h"

namespace stdg {

namespace {

struct Work {
  int64_t n = 0, nt = 0, ne = 0;
  int restart = 0;
  bool f32 = false;
  double *V = nullptr, *w = nullptr, *x = nullptr, *r = nullptr, *U = nullptr, *d = nullptr, *pd = nullptr;
  float *v32 = nullptr, *w32 = nullptr;
  double *partial = nullptr, *hdev = nullptr, *etmp = nullptr;
  size_t bytes = 0;
};

void free_work(Ctx* ctx, Work& W) {
  auto fr = [&](void* p, size_t b) { dev_free(ctx, p, b); };
  const size_t n8 = sizeof(double) * W.n, n4 = sizeof(float) * W.n;
  fr(W.V, n8 * (W.restart + 1));
  fr(W.w, n8);
  fr(W.x, n8);
  fr(W.r, n8);
  fr(W.d, n8);
  fr(W.pd, n8);
  fr(W.U, sizeof(double) * W.nt);
  if (W.v32) fr(W.v32, n4);
  if (W.w32) fr(W.w32, n4);
  fr(W.partial, sizeof(double) * kDotBlocks * kMaxBasis);
  fr(W.hdev, sizeof(double) * kMaxBasis);
  fr(W.etmp, sizeof(double) * (W.ne + 2));
  W = Work();
}

int alloc_work(Ctx* ctx, Work& W, int64_t n, int64_t nt, int64_t ne, int restart, bool f32) {
  W.n = n;
  W.nt = nt;
  W.ne = ne;
  W.restart = restart;
  W.f32 = f32;
  const size_t n8 = sizeof(double) * n, n4 = sizeof(float) * n;
  int rc;
  if ((rc = dev_alloc(ctx, (void**)&W.V, n8 * (restart + 1))) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&W.w, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&W.x, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&W.r, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&W.d, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&W.pd, n8)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&W.U, sizeof(double) * nt)) != STDG_OK) return rc;
  if (f32) {
    if ((rc = dev_alloc(ctx, (void**)&W.v32, n4)) != STDG_OK) return rc;
    if ((rc = dev_alloc(ctx, (void**)&W.w32, n4)) != STDG_OK) return rc;
  }
  if ((rc = dev_alloc(ctx, (void**)&W.partial, sizeof(double) * kDotBlocks * kMaxBasis)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&W.hdev, sizeof(double) * kMaxBasis)) != STDG_OK) return rc;
  if ((rc = dev_alloc(ctx, (void**)&W.etmp, sizeof(double) * (ne + 2))) != STDG_OK) return rc;
  return STDG_OK;
}

// true residual r = L - B U(x) in FP64, returns ||r|| (synchronises)
int true_residual(const Mesh* m, double dt, const double* load, const double* state, Work& W, hipStream_t s,
                  double* norm) {
  int rc;
  if ((rc = layout_embed(m, W.U, W.x, state, s)) != STDG_OK) return rc;
  ApplyArgs a{m, dt, STDG_FP64, STDG_RESIDUAL, W.U, load, W.r, s};
  if ((rc = launch_residual(a)) != STDG_OK) return rc;
  if ((rc = blas_scale(W.r, W.r, -1.0, W.n, s)) != STDG_OK) return rc;
  if ((rc = blas_multi_dot(W.r, W.n, 1, W.r, false, W.n, W.partial, W.hdev, s)) != STDG_OK) return rc;
  double nn = 0.0;
  STDG_HIP(hipMemcpyAsync(&nn, W.hdev, sizeof(double), hipMemcpyDeviceToHost, s));
  STDG_HIP(hipStreamSynchronize(s));
  *norm = std::sqrt(nn);
  return STDG_OK;
}

}  // namespace

}  // namespace stdg

using namespace stdg;

extern "C" int stdg_slab_solve(const stdg_mesh* mesh, double t0, double dt, const double* load_dev,
                               const stdg_solve_opts* opts, double* state_dev, double* slab_U_dev,
                               stdg_solve_info* info, void* stream) {
  (void)t0;
  if (!mesh || !opts || !state_dev || !info) return fail(STDG_E_ARG, "stdg_slab_solve: NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(STDG_E_ARG, "stdg_slab_solve: dt must be finite and > 0");
  if (opts->inner_prec != STDG_FP64 && opts->inner_prec != STDG_FP32)
    return fail(STDG_E_ARG, "stdg_slab_solve: unknown inner precision");
  const int restart = opts->restart > 0 ? opts->restart : 10;
  if (restart + 1 > kMaxBasis) return fail(STDG_E_ARG, "stdg_slab_solve: restart must be <= 31");
  const int max_iters = opts->max_iters > 0 ? opts->max_iters : 500;
  const int max_refine = opts->max_refine > 0 ? opts->max_refine : 100;
  const double rtol = opts->rtol > 0 ? opts->rtol : 1e-10;
  const double inner_rtol = opts->inner_rtol > 0 ? opts->inner_rtol : 1e-4;
  const bool f32 = opts->inner_prec == STDG_FP32;
  std::memset(info, 0, sizeof(*info));

  Mesh* m = const_cast<Mesh*>(&mesh->m);
  hipStream_t s = (hipStream_t)stream;
  int rc = ensure_state_off(m);
  if (rc != STDG_OK) return rc;
  const int64_t n = m->unk_off.back();
  Work W;
  rc = alloc_work(m->ctx, W, n, m->trial_off.back(), m->ne, restart, f32);
  if (rc != STDG_OK) {
    free_work(m->ctx, W);
    return rc;
  }
  auto done = [&](int code) {
    free_work(m->ctx, W);
    return code;
  };
#define TRY(call)                       \
  do {                                  \
    int rc_ = (call);                   \
    if (rc_ != STDG_OK) return done(rc_); \
  } while (0)

  // energy at the slab start
  TRY(energy_async(m, state_dev, W.etmp, W.etmp + m->ne, s));
  double e0 = 0.0;
  if (hipMemcpyAsync(&e0, W.etmp + m->ne, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return done(fail(STDG_E_DEVICE, "energy copy"));

  TRY(layout_guess(m, W.x, state_dev, s));
  double beta0 = 0.0, beta = 0.0;
  TRY(true_residual(m, dt, load_dev, state_dev, W, s, &beta0));
  beta = beta0;
  info->refinements = 1;
  int iters = 0;
  bool converged = !(beta0 > 0.0) || beta0 == 0.0;
  if (!std::isfinite(beta0)) return done(fail(STDG_E_ARG, "stdg_slab_solve: non-finite initial residual"));
  std::vector<double> H((restart + 1) * restart), cs(restart), sn(restart), g(restart + 1), hcol(kMaxBasis),
      y(restart);
  int cycles = 0;
  while (!converged && iters < max_iters && (!f32 || cycles < max_refine)) {
    ++cycles;
    // V_0 = r / beta
    TRY(blas_scale(W.V, W.r, 1.0 / beta, n, s));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    const double target = rtol * beta0;
    const double inner_target = f32 ? std::max(inner_rtol * beta, target) : target;
    int k = 0;
    for (int j = 0; j < restart && iters < max_iters; ++j) {
      double* Vj = W.V + (int64_t)j * n;
      const void* wsrc;
      if (f32) {
        TRY(blas_to_f32(W.v32, Vj, 1.0, n, s));
        ApplyArgs a{m, dt, STDG_FP32, STDG_OPERATOR_PRECOND, W.v32, nullptr, W.w32, s};
        TRY(launch_residual(a));
        wsrc = W.w32;
      } else {
        ApplyArgs a{m, dt, STDG_FP64, STDG_OPERATOR_PRECOND, Vj, nullptr, W.w, s};
        TRY(launch_residual(a));
        wsrc = W.w;
      }
      ++iters;
      // classical Gram-Schmidt, twice
      TRY(blas_multi_dot(W.V, n, j + 1, wsrc, f32, n, W.partial, W.hdev, s));
      TRY(blas_update(W.w, wsrc, f32, W.V, n, j + 1, W.hdev, n, s));
      std::vector<double> h1(j + 1), h2(j + 1);
      if (hipMemcpyAsync(h1.data(), W.hdev, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s) != hipSuccess)
        return done(fail(STDG_E_DEVICE, "copy h"));
      TRY(blas_multi_dot(W.V, n, j + 1, W.w, false, n, W.partial, W.hdev, s));
      TRY(blas_update(W.w, W.w, false, W.V, n, j + 1, W.hdev, n, s));
      if (hipMemcpyAsync(h2.data(), W.hdev, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s) != hipSuccess)
        return done(fail(STDG_E_DEVICE, "copy h"));
      TRY(blas_multi_dot(W.w, n, 1, W.w, false, n, W.partial, W.hdev, s));
      double hn2 = 0.0;
      if (hipMemcpyAsync(&hn2, W.hdev, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
        return done(fail(STDG_E_DEVICE, "copy norm"));
      if (hipStreamSynchronize(s) != hipSuccess) return done(fail(STDG_E_DEVICE, "sync"));
      const double hnext = std::sqrt(hn2);
      for (int i = 0; i <= j; ++i) hcol[i] = h1[i] + h2[i];
      hcol[j + 1] = hnext;
      if (!std::isfinite(hnext)) return done(fail(STDG_E_NOT_CONVERGED, "stdg_slab_solve: non-finite Krylov vector"));
      if (hnext > 0.0) TRY(blas_scale(W.V + (int64_t)(j + 1) * n, W.w, 1.0 / hnext, n, s));
      // Givens rotations
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * hcol[i] + sn[i] * hcol[i + 1];
        hcol[i + 1] = -sn[i] * hcol[i] + cs[i] * hcol[i + 1];
        hcol[i] = t;
      }
      const double den = std::hypot(hcol[j], hcol[j + 1]);
      cs[j] = den > 0 ? hcol[j] / den : 1.0;
      sn[j] = den > 0 ? hcol[j + 1] / den : 0.0;
      hcol[j] = den;
      hcol[j + 1] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      for (int i = 0; i <= j; ++i) H[i * restart + j] = hcol[i];
      k = j + 1;
      if (std::fabs(g[j + 1]) <= inner_target || hnext == 0.0) break;
    }
    // y = H^{-1} g, correction d = sum y_j V_j, x += P^{-1} d
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int l = i + 1; l < k; ++l) t -= H[i * restart + l] * y[l];
      y[i] = t / H[i * restart + i];
    }
    if (hipMemcpyAsync(W.hdev, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s) != hipSuccess)
      return done(fail(STDG_E_DEVICE, "copy y"));
    TRY(blas_lincomb(W.d, false, W.V, n, k, W.hdev, n, s));
    TRY(launch_precond_scale(m, STDG_FP64, W.d, W.pd, s));
    TRY(blas_axpy(W.x, W.pd, 1.0, n, s));
    TRY(true_residual(m, dt, load_dev, state_dev, W, s, &beta));
    info->refinements += 1;
    converged = beta <= rtol * beta0;
  }
  info->iters = iters;
  info->rel_res = beta0 > 0 ? beta / beta0 : 0.0;
  if (slab_U_dev) {
    TRY(layout_embed(m, slab_U_dev, W.x, state_dev, s));
  }
  TRY(layout_level(m, state_dev, W.x, 1, s));
  TRY(energy_async(m, state_dev, W.etmp, W.etmp + m->ne, s));
  double e1 = 0.0;
  if (hipMemcpyAsync(&e1, W.etmp + m->ne, sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess)
    return done(fail(STDG_E_DEVICE, "energy copy"));
  if (hipStreamSynchronize(s) != hipSuccess) return done(fail(STDG_E_DEVICE, "sync"));
  info->energy_start = e0;
  info->energy_end = e1;
  if (!converged)
    return done(fail(STDG_E_NOT_CONVERGED, "stdg_slab_solve: relative residual " + std::to_string(info->rel_res) +
                                                " after " + std::to_string(iters) + " iterations"));
  return done(STDG_OK);
#undef TRY
}
