// Slab-solver internals: device vector kernels, layout conversions, the fused
// Arnoldi kernels and the resumable GMRES state machine.
#pragma once

#include "internal.h"

namespace stdg {

// restart + 1 <= 16: the Arnoldi passes keep one FP64 accumulator per basis
// vector in registers, and past 16 the compiler moves them to scratch memory
constexpr int kMaxBasis = 16;
constexpr int kMaxDotBlocks = 1024;

// Scratch of the deterministic reductions: kMaxBasis * kMaxDotBlocks partials
// and a counter that must be zero before the first use (kernels leave it zero).
struct DotWork {
  double* partial = nullptr;
  unsigned* counter = nullptr;
};
// Device state of one GMRES restart cycle (krylov.hip): the host writes
// target, restart and max_iters before the cycle; the kernels keep the rest.
struct CycleCtl {
  double target;     // the cycle stops once the residual estimate |g_{j+1}| <= target
  int32_t restart;   // columns at most
  int32_t max_iters; // inner iterations allowed for the slab (counted in iters)
  int32_t active;    // 1 while the cycle runs: kernels of later iterations return at once otherwise
  int32_t k;         // columns done
  int32_t iters;     // inner iterations of the slab so far
  int32_t bad;       // a non-finite Hessenberg entry was met
  double nu, inv_nu;        // norm estimate of the pending vector, and 1 / nu for pass 2
  double hp[kMaxBasis];     // second-projection coefficients of the pending vector
  double h[kMaxBasis];      // Hessenberg entries of the first projection, current column
  double cz[kMaxBasis];     // (V_l . z) / nu, current column
  double Hraw[kMaxBasis * kMaxBasis];  // Hessenberg matrix as built, row-major [l * kMaxBasis + j]
  double R[kMaxBasis * kMaxBasis];     // the same after the Givens rotations (upper triangular)
  double cs[kMaxBasis], sn[kMaxBasis], g[kMaxBasis + 1];
  double y[kMaxBasis];      // combination coefficients at the cycle end
};
// Arnoldi passes (krylov.hip).  V: basis slots (leading dimension ldv) in
// FP32 (v32) or FP64; z: apply output in FP32 (z32) or FP64; w: pending
// vector, FP32 when v32 else FP64, with an optional FP32 copy w32 (the input
// of FP32 applies next to an FP64 basis).
int arnoldi_pass1(const void* V, bool v32, int64_t ldv, int j, const void* z, bool z32, const void* w, int64_t n,
                  CycleCtl* ctl, const DotWork& dw, hipStream_t st);
int arnoldi_pass2(void* V, bool v32, int64_t ldv, int j, const void* z, bool z32, void* w, float* w32, int64_t n,
                  CycleCtl* ctl, const DotWork& dw, hipStream_t st);
// V_0 = r / sqrt(*norm2) (and its FP32 copy v0_32 when not NULL); resets the cycle state
int cycle_start(const double* r, const double* norm2, void* v0, bool v32, float* v0_32, int64_t n, CycleCtl* ctl,
                hipStream_t st);
int cycle_least_squares(CycleCtl* ctl, hipStream_t st);
// out = sum_{l < k} coef_l V_l, with k read from kdev when not NULL
int basis_combine(double* out, const void* V, bool v32, int64_t ld, int k, const int* kdev, const double* coef,
                  int64_t n, hipStream_t st);
int vec_dot(const double* a, const double* b, int64_t n, double* out, const DotWork& dw, hipStream_t st);

// Batched cycle kernels: the restart cycles of up to kMaxBatch requests (the
// serving loop), one launch per step, each request on a segment of the grid
// with the block partition of its own unbatched launch (so that its
// reductions, and every result, are bitwise those of a solve alone).  All
// requests of a batch run the same iteration with the same precisions.
constexpr int kMaxBatch = 16;
struct CycleSeg {
  void* V = nullptr;             // basis (slot 0 is the start vector)
  int64_t ldv = 0;
  const void* z = nullptr;       // apply output
  void* w = nullptr;             // pending vector
  float* w32 = nullptr;          // FP32 copy of the apply input (FP32 applies, FP64 basis)
  const double* r = nullptr;     // cycle start: residual (FP64) and its squared norm
  const double* norm2 = nullptr;
  double* out = nullptr;         // cycle end: out = sum_l y_l V_l
  int64_t n = 0;
  CycleCtl* ctl = nullptr;
  DotWork dw;
};
int cycle_start_batch(const CycleSeg* segs, int count, bool v32, hipStream_t st);
int arnoldi_pass1_batch(const CycleSeg* segs, int count, bool v32, bool z32, int j, hipStream_t st);
int arnoldi_pass2_batch(const CycleSeg* segs, int count, bool v32, bool z32, int j, hipStream_t st);
int cycle_least_squares_batch(const CycleSeg* segs, int count, hipStream_t st);
// out = sum_{l < ctl->k} ctl->y[l] V_l for each request (k <= kmax)
int basis_combine_batch(const CycleSeg* segs, int count, bool v32, int kmax, hipStream_t st);
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
// (the tests between restart cycles) and enqueues the next step.  A restart
// cycle (up to `restart` Arnoldi iterations, the least-squares update of the
// iterate and its true FP64 residual) runs on the device without the host.
// The blocking stdg_slab_solve and the serving loop both drive it.
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

  // Deferred cycles (the serving loop): advance() does not enqueue a restart
  // cycle itself but leaves it pending (cycle_pending()); the caller then
  // launches it alone (launch_pending_cycle) or together with the pending
  // cycles of other solvers of the same batch_key() (launch_cycles_batched),
  // before it next polls event().
  void set_defer_cycles(bool d) { defer_ = d; }
  bool cycle_pending() const { return phase_ == kWantCycle; }
  // key of the batched cycles this solver can join (the kernel group's a and q
  // with the precisions), or -1: FP32 applies on a mesh of one affine kernel
  // group with a diagonal metric and no D_h
  int batch_key() const;
  int launch_pending_cycle();
  // one restart cycle of each of the count solvers (pending, same batch_key)
  // on stream bs, one launch per step for all; then each solver's true
  // residual on its own stream after event bev
  static int launch_cycles_batched(SlabSolver* const* s, int count, hipStream_t bs, hipEvent_t bev);
  int batched_cycles = 0;  // restart cycles run in a batch (of this solver's life)

  // results of the finished slab
  int status = 0;  // STDG_OK or STDG_E_NOT_CONVERGED
  int iters = 0, refinements = 0;
  double rel_res = 0.0, energy_start = 0.0, energy_end = 0.0;
  double eta2 = 0.0;  // the slab's term of eta_it^2 at the final iterate (inexact solve only)

 private:
  enum Phase { kIdle, kWaitStart, kWaitCycle, kWaitEnd, kWantCycle };
  int launch_true_residual();
  int launch_cycle();
  int prepare_cycle();  // the cycle count, inner target and control parameters (host)
  int run_cycle();      // the prepared cycle (graph or direct), then the true residual
  bool defer_ = false;
  int enqueue_cycle();  // the cycle's kernels, from the start vector to the updated iterate
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
  void* V_ = nullptr;   // restart + 1 basis vectors (FP32 or FP64)
  void* w_ = nullptr;   // the pending vector (FP32 with an FP32 basis, else FP64)
  void* z_ = nullptr;   // apply output (FP32 with FP32 applies, else FP64)
  float* w32_ = nullptr;  // FP32 copy of the apply input (FP32 applies, FP64 basis)
  double *x_ = nullptr, *r_ = nullptr, *U_ = nullptr, *d_ = nullptr, *pd_ = nullptr;
  CycleCtl* ctl_ = nullptr;
  // a whole restart cycle captured as one graph (valid for graph_dt_ and the
  // mesh epoch graph_epoch_), launched from the second cycle on
  void drop_graphs();
  hipGraphExec_t gexec_ = nullptr;
  hipStream_t cap_ = nullptr;  // capture stream (the caller's may be the null stream, which cannot capture)
  bool seen_ = false;
  double graph_dt_ = 0.0;
  uint64_t graph_epoch_ = 0;
  DotWork dw_;
  double *hv_ = nullptr, *etmp_ = nullptr;  // device scalars (layout kBeta.. in solver.cpp)
  double* hb_ = nullptr;                    // pinned host copy of the scalars
  CycleCtl* hctl_ = nullptr;                // pinned host copy of the cycle parameters
  // slab state
  double dt_ = 0.0;
  const double* load_ = nullptr;
  double* state_ = nullptr;
  double* slabU_ = nullptr;
  double beta0_ = 0.0, beta_ = 0.0;
  double eta_term() const;  // eta_it^2 term of the residual in the scalars
  int cycles_ = 0;
  bool converged_ = false;
};

}  // namespace stdg
