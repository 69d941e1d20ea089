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

template <int QQ>
static void launch_q(const KParams<STDG_REAL>& P, dim3 grid, dim3 block, hipStream_t stream) {
  switch (P.mode) {
    case 0:
      hipLaunchKernelGGL((residual_affine_kernel<STDG_REAL, STDG_A, QQ, 0>), grid, block, shmem_bytes<QQ>(), stream, P);
      break;
    case 1:
      hipLaunchKernelGGL((residual_affine_kernel<STDG_REAL, STDG_A, QQ, 1>), grid, block, shmem_bytes<QQ>(), stream, P);
      break;
    default:
      hipLaunchKernelGGL((residual_affine_kernel<STDG_REAL, STDG_A, QQ, 2>), grid, block, shmem_bytes<QQ>(), stream, P);
      break;
  }
}

int STDG_CAT(STDG_CAT(launch_affine_, STDG_REAL), STDG_A)(int q, const KParams<STDG_REAL>& P, int64_t n,
                                                         hipStream_t stream) {
  using Cf = KCfg<STDG_A>;
  const dim3 grid((unsigned)n), block(Cf::NT);
  switch (q) {
    case 1: launch_q<1>(P, grid, block, stream); break;
    case 2: launch_q<2>(P, grid, block, stream); break;
    case 3: launch_q<3>(P, grid, block, stream); break;
    case 4: launch_q<4>(P, grid, block, stream); break;
    case 5: launch_q<5>(P, grid, block, stream); break;
    case 6: launch_q<6>(P, grid, block, stream); break;
    default:
      return fail(STDG_E_ARG, "q out of range");
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "residual kernel launch");
  return STDG_OK;
}

}  // namespace stdg
