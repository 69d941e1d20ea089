// One (precision, a) slice of the residual kernels: instantiates q = 1..6 and
// exposes a launcher.  Compiled once per (STDG_REAL, STDG_A) by the build.
#include "residual_kernel.h"

#ifndef STDG_A
#error "STDG_A must be defined"
#endif
#ifndef STDG_REAL
#error "STDG_REAL must be defined"
#endif

#define STDG_CAT2(a, b) a##b
#define STDG_CAT(a, b) STDG_CAT2(a, b)

namespace stdg {

template <int QQ>
static constexpr size_t shmem_bytes() {
  return sizeof(STDG_REAL) * KCfg<STDG_A>::template lds_elems<STDG_REAL, QQ>();
}

int STDG_CAT(STDG_CAT(launch_affine_, STDG_REAL), STDG_A)(int q, const KParams<STDG_REAL>& P, int64_t n,
                                                         hipStream_t stream) {
  using Cf = KCfg<STDG_A>;
  const dim3 grid((unsigned)n), block(Cf::NT);
  switch (q) {
#define STDG_CASE(QQ)                                                                                    \
  case QQ:                                                                                             \
    hipLaunchKernelGGL((residual_affine_kernel<STDG_REAL, STDG_A, QQ>), grid, block, shmem_bytes<QQ>(), stream, \
                       P);                                                                             \
    break;
    STDG_CASE(1)
    STDG_CASE(2)
    STDG_CASE(3)
    STDG_CASE(4)
    STDG_CASE(5)
    STDG_CASE(6)
#undef STDG_CASE
    default:
      return fail(STDG_E_ARG, "q out of range");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "residual kernel launch");
  return STDG_OK;
}

}  // namespace stdg
