// One (precision, a, element kind) slice of the residual kernels: instantiates
// q = 1..6 and exposes a launcher.  Compiled once per (STDG_REAL, STDG_A,
// STDG_AFF, STDG_DISS) by the build; STDG_AFF = 1 for affine elements (constant
// metric), 0 for trilinear ones (mass by quadrature, no fused P^{-1});
// STDG_DISS = 1 adds the dissipative face terms (affine elements only).
#include "residual_kernel.h"

#ifndef STDG_A
#error "STDG_A must be defined"
#endif
#ifndef STDG_REAL
#error "STDG_REAL must be defined"
#endif
#ifndef STDG_AFF
#error "STDG_AFF must be defined"
#endif

#ifndef STDG_DISS
#define STDG_DISS 0
#endif
#if STDG_DISS && !STDG_AFF
#error "the dissipative kernels are built for affine elements only"
#endif

#define STDG_CAT2(a, b) a##b
#define STDG_CAT(a, b) STDG_CAT2(a, b)
#if STDG_DISS
#define STDG_KIND affine_diss_
#elif STDG_AFF
#define STDG_KIND affine_
#else
#define STDG_KIND trilinear_
#endif

namespace stdg {

template <int QQ, int MODE>
static constexpr size_t shmem_bytes() {
  return sizeof(STDG_REAL) * KCfg<STDG_A>::template lds_elems<STDG_REAL, QQ, (bool)STDG_AFF, MODE, (bool)STDG_DISS>();
}

template <int QQ, int MODE, int VAR>
static int launch_one(const KParams<STDG_REAL>& P, dim3 grid, dim3 block, hipStream_t stream) {
  hipLaunchKernelGGL((residual_kernel<STDG_REAL, STDG_A, QQ, MODE, (bool)STDG_AFF, (bool)STDG_DISS, VAR>), grid, block,
                     (shmem_bytes<QQ, MODE>()), stream, P);
  return STDG_OK;
}

// The launch variants (residual_kernel.h, element_body) exist for affine
// groups without D_h in the operator modes and for trilinear groups in the
// operator mode (the ones a slab solve repeats: trilinear elements take
// P^{-1} in a pre-pass); every other kernel runs variant 0.
template <int QQ, int MODE>
static int launch_var(const KParams<STDG_REAL>& P, dim3 grid, dim3 block, hipStream_t stream) {
#if STDG_AFF && !STDG_DISS
  if (MODE != 1) {
    if (P.variant == 1) return launch_one<QQ, MODE, 1>(P, grid, block, stream);
    if (P.variant == 2) return launch_one<QQ, MODE, 2>(P, grid, block, stream);
  }
#elif !STDG_AFF
  // trilinear groups, variant 1: one workgroup per element and test level
  // (built for 1 < q <= 4: past that the per-level selection of the element's
  // registers goes through scratch memory)
  if constexpr (MODE == 0 && QQ > 1 && QQ <= kMaxLevelSplitQ) {
    if (P.variant == 1) {
      if (grid.x > 0xffffffffu / QQ) return fail(STDG_E_ARG, "residual kernel: too many elements for the level split");
      return launch_one<QQ, MODE, 3>(P, dim3(grid.x * QQ), block, stream);
    }
  }
#endif
  return launch_one<QQ, MODE, 0>(P, grid, block, stream);
}

template <int QQ>
static int launch_q(const KParams<STDG_REAL>& P, dim3 grid, dim3 block, hipStream_t stream) {
  switch (P.mode) {
    case 0:
      return launch_var<QQ, 0>(P, grid, block, stream);
    case 1:
      return launch_var<QQ, 1>(P, grid, block, stream);
    default:
#if STDG_AFF
      return launch_var<QQ, 2>(P, grid, block, stream);
#else
      return fail(STDG_E_UNSUPPORTED, "trilinear elements take P^{-1} in a separate pass");
#endif
  }
}

int STDG_CAT(STDG_CAT(STDG_CAT(launch_, STDG_KIND), STDG_REAL), STDG_A)(int q, const KParams<STDG_REAL>& P, int64_t n,
                                                                       hipStream_t stream) {
  using Cf = KCfg<STDG_A>;
  const dim3 grid((unsigned)n), block(Cf::NT);
  int rc;
  switch (q) {
    case 1: rc = launch_q<1>(P, grid, block, stream); break;
    case 2: rc = launch_q<2>(P, grid, block, stream); break;
    case 3: rc = launch_q<3>(P, grid, block, stream); break;
    case 4: rc = launch_q<4>(P, grid, block, stream); break;
    case 5: rc = launch_q<5>(P, grid, block, stream); break;
    case 6: rc = launch_q<6>(P, grid, block, stream); break;
    default:
      return fail(STDG_E_ARG, "q out of range");
  }
  if (rc != STDG_OK) return rc;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "residual kernel launch");
  return STDG_OK;
}

#if STDG_AFF && !STDG_DISS
template <int QQ>
static int launch_batch_q(const BatchKParams<STDG_REAL>& B, uint32_t total, hipStream_t stream) {
  hipLaunchKernelGGL((residual_batch_kernel<STDG_REAL, STDG_A, QQ>), dim3(total), dim3(KCfg<STDG_A>::NT),
                     (shmem_bytes<QQ, 2>()), stream, B);
  return STDG_OK;
}

int STDG_CAT(STDG_CAT(launch_batch_, STDG_REAL), STDG_A)(int q, const BatchKParams<STDG_REAL>& B, uint32_t total,
                                                        hipStream_t stream) {
  int rc;
  switch (q) {
    case 1: rc = launch_batch_q<1>(B, total, stream); break;
    case 2: rc = launch_batch_q<2>(B, total, stream); break;
    case 3: rc = launch_batch_q<3>(B, total, stream); break;
    case 4: rc = launch_batch_q<4>(B, total, stream); break;
    case 5: rc = launch_batch_q<5>(B, total, stream); break;
    case 6: rc = launch_batch_q<6>(B, total, stream); break;
    default:
      return fail(STDG_E_ARG, "q out of range");
  }
  if (rc != STDG_OK) return rc;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "batched residual kernel launch");
  return STDG_OK;
}
#endif

}  // namespace stdg
