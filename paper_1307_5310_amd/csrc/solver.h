// Slab-solver internals: device vector kernels and layout conversions.
#pragma once

#include "internal.h"

namespace stdg {

constexpr int kMaxBasis = 32;   // restart + 1 <= 32
constexpr int kDotBlocks = 1024;

int blas_multi_dot(const double* V, int64_t ld, int k, const void* w, bool w_f32, int64_t n, double* partial,
                   double* out, hipStream_t s);
int blas_update(double* w, const void* src, bool src_f32, const double* V, int64_t ld, int k, const double* h,
                int64_t n, hipStream_t s);
int blas_scale(double* out, const double* in, double alpha, int64_t n, hipStream_t s);
int blas_lincomb(void* out, bool out_f32, const double* V, int64_t ld, int k, const double* y, int64_t n,
                 hipStream_t s);
int blas_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s);
int blas_to_f32(float* out, const double* in, double alpha, int64_t n, hipStream_t s);
int layout_embed(const Mesh* m, double* U, const double* x, const double* st, hipStream_t s);
int layout_level(const Mesh* m, double* st, const double* x, int lev, hipStream_t s);
int layout_guess(const Mesh* m, double* x, const double* st, hipStream_t s);
int energy_async(const Mesh* m, const double* state, double* d_partial, double* d_out, hipStream_t s);
int ensure_state_off(Mesh* m);

// Options of one slab solve (validated copies of stdg_solve_opts).
struct SlabOpts {
  bool f32 = false;
  int restart = 10, max_iters = 500, max_refine = 100;
  double rtol = 1e-10, inner_rtol = 1e-4;
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
  // start a slab: state (FP64, device) at its start, load may be NULL
  int begin(double dt, const double* load, double* state, double* slab_U);
  hipEvent_t event() const { return ev_; }
  // call once event() has completed; *done = true when the slab is finished
  int advance(bool* done);

  // results of the finished slab
  int status = 0;  // STDG_OK or STDG_E_NOT_CONVERGED
  int iters = 0, refinements = 0;
  double rel_res = 0.0, energy_start = 0.0, energy_end = 0.0;

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
  // device work vectors
  double *V_ = nullptr, *w_ = nullptr, *x_ = nullptr, *r_ = nullptr, *U_ = nullptr, *d_ = nullptr, *pd_ = nullptr;
  float *v32_ = nullptr, *w32_ = nullptr;
  double *partial_ = nullptr, *hdev_ = nullptr, *etmp_ = nullptr;
  // pinned host scalars: [0, kMaxBasis) h1, [kMaxBasis, 2k) h2, then norm2, beta2, e0, e1, and y
  double* hb_ = nullptr;
  // slab state
  double dt_ = 0.0;
  const double* load_ = nullptr;
  double* state_ = nullptr;
  double* slabU_ = nullptr;
  double beta0_ = 0.0, beta_ = 0.0, inner_target_ = 0.0;
  int cycles_ = 0, j_ = 0;
  bool converged_ = false;
  double H_[kMaxBasis * kMaxBasis], cs_[kMaxBasis], sn_[kMaxBasis], g_[kMaxBasis + 1];
};

}  // namespace stdg
