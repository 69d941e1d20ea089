// Slab-solver internals: device vector kernels, layout conversions, the fused
// Arnoldi kernels and the resumable GMRES state machine.
#pragma once

#include "internal.h"

namespace stdg {

constexpr int kMaxBasis = 32;   // restart + 1 <= 32
constexpr int kMaxDotBlocks = 1024;

// Scratch of the deterministic reductions: kMaxBasis * kMaxDotBlocks partials
// and a counter that must be zero before the first use (kernels leave it zero).
struct DotWork {
  double* partial = nullptr;
  unsigned* counter = nullptr;
};
// Fused Arnoldi kernels (krylov.hip); V holds k basis vectors of length n
// (leading dimension ld) in FP32 (v32) or FP64, w in FP32 (w32) or FP64.
int arnoldi_dot(const void* V, bool v32, int64_t ld, int k, const void* w, bool w32, int64_t n, const double* s,
                double* h, double* c, const DotWork& dw, hipStream_t st);
int arnoldi_update_dot(const void* V, bool v32, int64_t ld, int k, const void* w, bool w32, const double* cin,
                       double* wout, int64_t n, const double* s, double* h, double* c, const DotWork& dw,
                       hipStream_t st);
int arnoldi_update_norm(const void* V, bool v32, int64_t ld, int k, const double* w, const double* cin, void* vout,
                        int64_t n, double* norm2, double* s_next, const DotWork& dw, hipStream_t st);
int basis_combine(double* out, const void* V, bool v32, int64_t ld, int k, const double* coef, int64_t n,
                  hipStream_t st);
int vec_dot(const double* a, const double* b, int64_t n, double* out, const DotWork& dw, hipStream_t st);
int vec_store(void* out, bool out32, const double* in, int64_t n, hipStream_t st);

int blas_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s);
int layout_embed(const Mesh* m, double* U, const double* x, const double* st, hipStream_t s);
int layout_level(const Mesh* m, double* st, const double* x, int lev, hipStream_t s);
int layout_guess(const Mesh* m, double* x, const double* st, hipStream_t s);
int energy_async(const Mesh* m, const double* state, double* d_partial, double* d_out, hipStream_t s);
// (||R_E||^2, ||R_H||^2) in W_h' of a residual-layout FP64 vector; d_partial holds 2 ne doubles
int dual_norms_async(const Mesh* m, double dt, const double* R, double* d_partial, double* d_out, hipStream_t s);
int ensure_state_off(Mesh* m);

// Options of one slab solve (validated copies of stdg_solve_opts).
struct SlabOpts {
  bool f32 = false;
  bool v32 = false;  // Krylov basis stored in FP32 (FP32 inner applies only)
  int restart = 10, max_iters = 500, max_refine = 100;
  double rtol = 1e-10, inner_rtol = 1e-4;
  double eta_tol = 0.0, eta_t_final = 0.0;  // inexact solve: stop once eta_it^2 of the slab <= eta_tol^2
  bool use_graph = false;                    // replay Arnoldi iterations as captured HIP graphs
};
int slab_opts_from(const stdg_solve_opts* o, SlabOpts* out);

// Device bytes a SlabSolver allocates for a mesh (admission control).
size_t slab_solver_bytes(int64_t n_unknowns, int64_t n_trial, int64_t ne, const SlabOpts& o);

// Restarted right-preconditioned GMRES for one slab as a resumable state
// machine: every step enqueues its device work on the solver's stream and
// records event(); once the event has completed, advance() does the host part
// (Givens rotations, convergence tests) and enqueues the next step.  The
// blocking stdg_slab_solve and the serving loop both drive it.
class SlabSolver {
 public:
  int init(Mesh* m, const SlabOpts& o, hipStream_t s);
  void release();
  // reuse for another solve: same allocation (precisions, restart), new
  // tolerances and stream
  bool compatible(const SlabOpts& o) const { return o.f32 == o_.f32 && o.v32 == o_.v32 && o.restart == o_.restart; }
  int rebind(const SlabOpts& o, hipStream_t s);
  // start a slab: state (FP64, device) at its start, load may be NULL
  int begin(double dt, const double* load, double* state, double* slab_U);
  hipEvent_t event() const { return ev_; }
  // call once event() has completed; *done = true when the slab is finished
  int advance(bool* done);

  // results of the finished slab
  int status = 0;  // STDG_OK or STDG_E_NOT_CONVERGED
  int iters = 0, refinements = 0;
  double rel_res = 0.0, energy_start = 0.0, energy_end = 0.0;
  double eta2 = 0.0;  // the slab's term of eta_it^2 at the final iterate (inexact solve only)

 private:
  enum Phase { kIdle, kWaitStart, kWaitIter, kWaitCycle, kWaitEnd };
  int launch_true_residual();
  int start_cycle();
  int launch_iteration();
  int launch_cycle_end();
  int launch_slab_end();

  Mesh* m_ = nullptr;
  SlabOpts o_;
  hipStream_t s_ = nullptr;
  hipEvent_t ev_ = nullptr;
  Phase phase_ = kIdle;
  int64_t n_ = 0;
  void* basis(int j) const { return (char*)V_ + (size_t)j * (size_t)ld_ * (o_.v32 ? 4 : 8); }
  int64_t ld_ = 0;  // basis leading dimension: n rounded up to a multiple of 64
  // device work vectors
  void* V_ = nullptr;  // restart + 1 unnormalised basis vectors (FP32 or FP64)
  double *w_ = nullptr, *x_ = nullptr, *r_ = nullptr, *U_ = nullptr, *d_ = nullptr, *pd_ = nullptr;
  float *v32_ = nullptr, *w32_ = nullptr;
  // captured Arnoldi iterations, one per basis index j (valid for graph_dt_)
  int enqueue_iteration(int j);
  void drop_graphs();
  hipGraphExec_t gexec_[kMaxBasis] = {};
  hipStream_t cap_ = nullptr;  // capture stream (the caller's may be the null stream, which cannot capture)
  bool seen_[kMaxBasis] = {};
  double graph_dt_ = 0.0;
  uint64_t graph_epoch_ = 0;  // mesh epoch the graphs were captured at
  DotWork dw_;
  double *hv_ = nullptr, *etmp_ = nullptr;  // device scalars (layout kH1.. in solver.cpp)
  double* hb_ = nullptr;                    // pinned host copy of the scalars
  double hs_[kMaxBasis + 1];                // basis scales s_j on the host
  // slab state
  double dt_ = 0.0;
  const double* load_ = nullptr;
  double* state_ = nullptr;
  double* slabU_ = nullptr;
  double beta0_ = 0.0, beta_ = 0.0, inner_target_ = 0.0;
  double eta_term() const;  // eta_it^2 term of the residual in the scalars
  int cycles_ = 0, j_ = 0;
  bool converged_ = false;
  double H_[kMaxBasis * kMaxBasis], cs_[kMaxBasis], sn_[kMaxBasis], g_[kMaxBasis + 1];
};

}  // namespace stdg
