// Vector update of the slab solver and the layout conversions between
// unknowns, full trial vectors and states (the Arnoldi kernels are in
// krylov.hip).
#include "internal.h"
#include "solver.h"

namespace stdg {

namespace {

__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] += a * x[i];
}

// full trial U (per element [f][c][m=0..n q][s]) from unknowns x ([f][c][m=1..n q][s])
// and a state ([f][c][s]) for the l_0 block (n = sub-intervals, usually 1)
__global__ void embed_kernel(double* __restrict__ U, const double* __restrict__ x, const double* __restrict__ st,
                             const ElemInfo* __restrict__ info, const int64_t* __restrict__ soff) {
  const int64_t e = blockIdx.x;
  const ElemInfo I = info[e];
  const int a3 = I.a * I.a * I.a, q = I.q * I.nsub;
  const int per = (q + 1) * a3;
  for (int idx = threadIdx.x; idx < 6 * per; idx += blockDim.x) {
    const int fc = idx / per, rest = idx - fc * per;
    const int m = rest / a3, s = rest - m * a3;
    U[I.trial_off + idx] = m == 0 ? st[soff[e] + (int64_t)fc * a3 + s] : x[I.unk_off + ((int64_t)fc * q + m - 1) * a3 + s];
  }
}

// state := trial level `lev` of the unknowns (lev >= 1)
__global__ void level_kernel(double* __restrict__ st, const double* __restrict__ x, int lev,
                             const ElemInfo* __restrict__ info, const int64_t* __restrict__ soff) {
  const int64_t e = blockIdx.x;
  const ElemInfo I = info[e];
  const int a3 = I.a * I.a * I.a, q = I.q * I.nsub;
  for (int idx = threadIdx.x; idx < 6 * a3; idx += blockDim.x) {
    const int fc = idx / a3, s = idx - fc * a3;
    st[soff[e] + idx] = x[I.unk_off + ((int64_t)fc * q + lev - 1) * a3 + s];
  }
}

// unknowns initial guess, the constant continuation: the values at the slab
// end (level 1) and, with sub-intervals, at their interior ends (levels
// 1 + j q) = state, the interior functions 0
__global__ void guess_kernel(double* __restrict__ x, const double* __restrict__ st, const ElemInfo* __restrict__ info,
                             const int64_t* __restrict__ soff) {
  const int64_t e = blockIdx.x;
  const ElemInfo I = info[e];
  const int a3 = I.a * I.a * I.a, q = I.q;
  const int per = q * I.nsub * a3;
  for (int idx = threadIdx.x; idx < 6 * per; idx += blockDim.x) {
    const int fc = idx / per, rest = idx - fc * per;
    const int m = rest / a3, s = rest - m * a3;  // unknown m is trial level m + 1
    x[I.unk_off + idx] = m % q == 0 ? st[soff[e] + (int64_t)fc * a3 + s] : 0.0;
  }
}

// Streaming copy: 16-byte lanes, two chunks in flight per thread,
// non-temporal loads and stores (the data is touched once), grid-stride.
typedef unsigned int u4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) stream_copy_kernel(const u4* __restrict__ src, u4* __restrict__ dst,
                                                          int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + stride < n16; i += 2 * stride) {
    const u4 a = __builtin_nontemporal_load(src + i);
    const u4 b = __builtin_nontemporal_load(src + i + stride);
    __builtin_nontemporal_store(a, dst + i);
    __builtin_nontemporal_store(b, dst + i + stride);
  }
  if (i < n16) __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

int stream_copy(const void* src, void* dst, size_t bytes, hipStream_t s) {
  const int64_t n16 = (int64_t)(bytes / 16);
  if (n16 == 0) return STDG_OK;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    cus = 256;
  // 32 blocks of 256 threads per compute unit: every CU full, one wave of blocks
  int64_t g = (int64_t)cus * 32, need = (n16 + 255) / 256;
  if (g > need) g = need;
  hipLaunchKernelGGL(stream_copy_kernel, dim3((unsigned)g), dim3(256), 0, s, (const u4*)src, (u4*)dst, n16);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "stream copy");
}

int blas_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, a, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "axpy");
}

int layout_embed(const Mesh* m, double* U, const double* x, const double* st, hipStream_t s) {
  hipLaunchKernelGGL(embed_kernel, dim3((unsigned)m->ne), dim3(256), 0, s, U, x, st, m->d_info, m->d_state_off);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "embed");
}

int layout_level(const Mesh* m, double* st, const double* x, int lev, hipStream_t s) {
  hipLaunchKernelGGL(level_kernel, dim3((unsigned)m->ne), dim3(256), 0, s, st, x, lev, m->d_info, m->d_state_off);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "level");
}

int layout_guess(const Mesh* m, double* x, const double* st, hipStream_t s) {
  hipLaunchKernelGGL(guess_kernel, dim3((unsigned)m->ne), dim3(256), 0, s, x, st, m->d_info, m->d_state_off);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "guess");
}

}  // namespace stdg
