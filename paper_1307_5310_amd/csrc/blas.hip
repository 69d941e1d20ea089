// Vector kernels of the slab solver (FP64 Krylov vectors) and the layout
// conversions between unknowns, full trial vectors and states.  Reductions
// use a fixed grid and a fixed combination order, so results are bitwise
// reproducible run to run.
#include "internal.h"
#include "solver.h"

namespace stdg {

namespace {

constexpr int kRedThreads = 256;

template <typename TW>
__global__ void __launch_bounds__(kRedThreads)
multi_dot_kernel(const double* __restrict__ V, int64_t ld, int k, const TW* __restrict__ w, int64_t n,
                 double* __restrict__ partial) {
  // partial[b * kMaxBasis + j] = sum over this block's chunk of V_j . w, j < k
  __shared__ double red[kRedThreads];
  double acc[kMaxBasis];
#pragma unroll
  for (int j = 0; j < kMaxBasis; ++j) acc[j] = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    const double wi = (double)w[i];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j)
      if (j < k) acc[j] += V[j * ld + i] * wi;
  }
  for (int j = 0; j < k; ++j) {
    red[threadIdx.x] = acc[j];
    __syncthreads();
    for (int s = kRedThreads / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.x * kMaxBasis + j] = red[0];
    __syncthreads();
  }
}

__global__ void finish_dot_kernel(const double* __restrict__ partial, int nblk, int k, double* __restrict__ out) {
  // one thread per j, fixed order over blocks
  const int j = threadIdx.x;
  if (j >= k) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += partial[(int64_t)b * kMaxBasis + j];
  out[j] = s;
}

// w (FP64) = src (TW) - sum_j h[j] V_j ; h on the device
template <typename TW>
__global__ void update_kernel(double* __restrict__ w, const TW* __restrict__ src, const double* __restrict__ V,
                              int64_t ld, int k, const double* __restrict__ h, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double hh[kMaxBasis];
#pragma unroll
  for (int j = 0; j < kMaxBasis; ++j) hh[j] = j < k ? h[j] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double v = (double)src[i];
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j)
      if (j < k) v -= hh[j] * V[j * ld + i];
    w[i] = v;
  }
}

__global__ void scale_kernel(double* __restrict__ out, const double* __restrict__ in, double alpha, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = alpha * in[i];
}

template <typename TO>
__global__ void lincomb_kernel(TO* __restrict__ out, const double* __restrict__ V, int64_t ld, int k,
                               const double* __restrict__ y, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  double yy[kMaxBasis];
#pragma unroll
  for (int j = 0; j < kMaxBasis; ++j) yy[j] = j < k ? y[j] : 0.0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double v = 0.0;
#pragma unroll
    for (int j = 0; j < kMaxBasis; ++j)
      if (j < k) v += yy[j] * V[j * ld + i];
    out[i] = (TO)v;
  }
}

__global__ void axpy_kernel(double* __restrict__ y, const double* __restrict__ x, double a, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) y[i] += a * x[i];
}

template <typename TI, typename TO>
__global__ void convert_kernel(TO* __restrict__ out, const TI* __restrict__ in, double alpha, int64_t n) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    out[i] = (TO)(alpha * (double)in[i]);
}

// full trial U (per element [f][c][m=0..q][s]) from unknowns x ([f][c][m=1..q][s])
// and a state ([f][c][s]) for the l_0 block
__global__ void embed_kernel(double* __restrict__ U, const double* __restrict__ x, const double* __restrict__ st,
                             const ElemInfo* __restrict__ info, const int64_t* __restrict__ soff) {
  const int64_t e = blockIdx.x;
  const ElemInfo I = info[e];
  const int a3 = I.a * I.a * I.a, q = I.q;
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
  const int a3 = I.a * I.a * I.a, q = I.q;
  for (int idx = threadIdx.x; idx < 6 * a3; idx += blockDim.x) {
    const int fc = idx / a3, s = idx - fc * a3;
    st[soff[e] + idx] = x[I.unk_off + ((int64_t)fc * q + lev - 1) * a3 + s];
  }
}

// unknowns initial guess: level 1 = state (constant continuation), others 0
__global__ void guess_kernel(double* __restrict__ x, const double* __restrict__ st, const ElemInfo* __restrict__ info,
                             const int64_t* __restrict__ soff) {
  const int64_t e = blockIdx.x;
  const ElemInfo I = info[e];
  const int a3 = I.a * I.a * I.a, q = I.q;
  const int per = q * a3;
  for (int idx = threadIdx.x; idx < 6 * per; idx += blockDim.x) {
    const int fc = idx / per, rest = idx - fc * per;
    const int m = rest / a3, s = rest - m * a3;
    x[I.unk_off + idx] = m == 0 ? st[soff[e] + (int64_t)fc * a3 + s] : 0.0;
  }
}

int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  return (int)g;
}

}  // namespace

int blas_multi_dot(const double* V, int64_t ld, int k, const void* w, bool w_f32, int64_t n, double* partial,
                   double* out, hipStream_t s) {
  const int nblk = kDotBlocks;
  if (w_f32)
    hipLaunchKernelGGL(multi_dot_kernel<float>, dim3(nblk), dim3(kRedThreads), 0, s, V, ld, k, (const float*)w, n,
                       partial);
  else
    hipLaunchKernelGGL(multi_dot_kernel<double>, dim3(nblk), dim3(kRedThreads), 0, s, V, ld, k, (const double*)w, n,
                       partial);
  hipLaunchKernelGGL(finish_dot_kernel, dim3(1), dim3(kMaxBasis), 0, s, partial, nblk, k, out);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "multi_dot");
}

int blas_update(double* w, const void* src, bool src_f32, const double* V, int64_t ld, int k, const double* h,
                int64_t n, hipStream_t s) {
  if (src_f32)
    hipLaunchKernelGGL(update_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, w, (const float*)src, V, ld, k, h, n);
  else
    hipLaunchKernelGGL(update_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, w, (const double*)src, V, ld, k, h,
                       n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "update");
}

int blas_scale(double* out, const double* in, double alpha, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(scale_kernel, dim3(grid_for(n)), dim3(256), 0, s, out, in, alpha, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "scale");
}

int blas_lincomb(void* out, bool out_f32, const double* V, int64_t ld, int k, const double* y, int64_t n,
                 hipStream_t s) {
  if (out_f32)
    hipLaunchKernelGGL(lincomb_kernel<float>, dim3(grid_for(n)), dim3(256), 0, s, (float*)out, V, ld, k, y, n);
  else
    hipLaunchKernelGGL(lincomb_kernel<double>, dim3(grid_for(n)), dim3(256), 0, s, (double*)out, V, ld, k, y, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "lincomb");
}

int blas_axpy(double* y, const double* x, double a, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpy_kernel, dim3(grid_for(n)), dim3(256), 0, s, y, x, a, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "axpy");
}

int blas_to_f32(float* out, const double* in, double alpha, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL((convert_kernel<double, float>), dim3(grid_for(n)), dim3(256), 0, s, out, in, alpha, n);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "to_f32");
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
