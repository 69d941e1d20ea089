// Fused Arnoldi kernels of the slab GMRES (Section 5.4): classical
// Gram-Schmidt applied twice, in three passes over the basis per iteration.
//
// The basis is stored unnormalised, V_j = s_j Vt_j with Vt_j in FP64 or FP32
// and the scales s_j in FP64 on the device, so a new basis vector is written
// once (no separate normalisation pass).  All sums are FP64.  Reductions are
// deterministic: fixed-order reductions inside each block, per-block partials,
// and the last block to finish (detected with a device-scope counter) sums the
// partials in block order and resets the counter.
//
//   arnoldi_dot         d_j = Vt_j . w                       -> h_j = s_j d_j, c_j = s_j^2 d_j
//   arnoldi_update_dot  w' = w - sum_j c_j Vt_j,  d'_j = Vt_j . w'  -> h', c'  (w' may overwrite w)
//   arnoldi_update_norm Vt_{k} = w' - sum_j c'_j Vt_j (stored), ||Vt_k||^2, s_k = 1 / ||Vt_k||
//
// Each thread streams 4 consecutive entries per step with 16-byte loads;
// basis slots therefore have a leading dimension that is a multiple of 64.
#include "solver.h"

namespace stdg {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double load_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Block-reduce acc[0..k) into partial[j * kMaxDotBlocks + blockIdx.x]; the
// last block reduces the partials over blocks and calls fin(j, total) on
// thread 0 for each j.  Returns after every block has passed the counter.
template <int KM, typename Fin>
__device__ __forceinline__ void reduce_and_finish(const double (&acc)[KM], int k, double* __restrict__ partial,
                                                  unsigned* __restrict__ counter, Fin fin) {
  __shared__ double wsum[kWaves][KM];
  __shared__ double red[kThreads];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j >= k) break;
    const double v = wave_sum(acc[j]);
    if (lane == 0) wsum[wave][j] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) v += wsum[w][threadIdx.x];
    partial[(int64_t)threadIdx.x * kMaxDotBlocks + blockIdx.x] = v;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int nb = (int)gridDim.x;
  for (int j = 0; j < k; ++j) {
    double v = 0.0;
    for (int b = threadIdx.x; b < nb; b += kThreads) v += load_agent(partial + (int64_t)j * kMaxDotBlocks + b);
    red[threadIdx.x] = v;
    __syncthreads();
#pragma unroll
    for (int w = kThreads / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) fin(j, red[0]);
    __syncthreads();
  }
  if (threadIdx.x == 0) atomicExch(counter, 0u);
}

// W consecutive values (W = 4: 16-byte vector loads; the caller keeps the
// address aligned: basis slots have a leading dimension that is a multiple of
// 64 and i is a multiple of W) converted to FP64.
template <int W>
__device__ __forceinline__ void ld(const float* p, double (&v)[W]) {
  if constexpr (W == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    const f4 t = *reinterpret_cast<const f4*>(p);
    v[0] = t.x; v[1] = t.y; v[2] = t.z; v[3] = t.w;
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) v[e] = p[e];
  }
}
template <int W>
__device__ __forceinline__ void ld(const double* p, double (&v)[W]) {
  if constexpr (W == 4) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 a = *reinterpret_cast<const d2*>(p), b = *reinterpret_cast<const d2*>(p + 2);
    v[0] = a.x; v[1] = a.y; v[2] = b.x; v[3] = b.y;
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) v[e] = p[e];
  }
}
template <int W>
__device__ __forceinline__ void st(float* p, const double (&v)[W]) {
  if constexpr (W == 4) {
    typedef float f4 __attribute__((ext_vector_type(4)));
    f4 t;
    t.x = (float)v[0]; t.y = (float)v[1]; t.z = (float)v[2]; t.w = (float)v[3];
    *reinterpret_cast<f4*>(p) = t;
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) p[e] = (float)v[e];
  }
}
template <int W>
__device__ __forceinline__ void st(double* p, const double (&v)[W]) {
  if constexpr (W == 4) {
    typedef double d2 __attribute__((ext_vector_type(2)));
    d2 a, b;
    a.x = v[0]; a.y = v[1]; b.x = v[2]; b.y = v[3];
    *reinterpret_cast<d2*>(p) = a;
    *reinterpret_cast<d2*>(p + 2) = b;
  } else {
#pragma unroll
    for (int e = 0; e < W; ++e) p[e] = v[e];
  }
}

// Runs body<4>(i) over i = 0, 4, .. < n rounded down to 4 (grid-stride), then
// body<1>(i) over the remaining tail on the first block.
template <typename Body>
__device__ __forceinline__ void for_vec4(int64_t n, Body body) {
  const int64_t n4 = n >> 2, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n4; q += stride)
    body.template run<4>(q << 2);
  const int64_t tail = n - (n4 << 2);
  if (blockIdx.x == 0 && (int64_t)threadIdx.x < tail) body.template run<1>((n4 << 2) + threadIdx.x);
}

template <typename TV, typename TW, int KM>
struct DotBody {
  const TV* V;
  int64_t ldv;
  int k;
  const TW* w;
  double* acc;
  template <int W>
  __device__ __forceinline__ void run(int64_t i) {
    double wv[W];
    ld<W>(w + i, wv);
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if (j < k) {
        double vv[W];
        ld<W>(V + j * ldv + i, vv);
#pragma unroll
        for (int e = 0; e < W; ++e) acc[j] += vv[e] * wv[e];
      }
    }
  }
};

template <typename TV, typename TW, int KM>
__global__ void __launch_bounds__(kThreads)
dot_kernel(const TV* __restrict__ V, int64_t ldv, int k, const TW* __restrict__ w, int64_t n,
           const double* __restrict__ s, double* __restrict__ h, double* __restrict__ c, double* __restrict__ partial,
           unsigned* __restrict__ counter) {
  double acc[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) acc[j] = 0.0;
  for_vec4(n, DotBody<TV, TW, KM>{V, ldv, k, w, acc});
  reduce_and_finish<KM>(acc, k, partial, counter, [&](int j, double d) {
    const double sj = s ? s[j] : 1.0;
    h[j] = sj * d;
    if (c) c[j] = sj * sj * d;
  });
}

template <typename TV, typename TW, int KM>
struct UpdateDotBody {
  const TV* V;
  int64_t ldv;
  int k;
  const TW* w;
  const double* cc;
  double* wout;
  double* acc;
  template <int W>
  __device__ __forceinline__ void run(int64_t i) {
    double x[W];
    ld<W>(w + i, x);
    double vv[KM][W];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if (j < k) {
        ld<W>(V + j * ldv + i, vv[j]);
#pragma unroll
        for (int e = 0; e < W; ++e) x[e] -= cc[j] * vv[j][e];
      }
    }
    st<W>(wout + i, x);
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) {
#pragma unroll
        for (int e = 0; e < W; ++e) acc[j] += vv[j][e] * x[e];
      }
  }
};

template <typename TV, typename TW, int KM>
__global__ void __launch_bounds__(kThreads)
update_dot_kernel(const TV* __restrict__ V, int64_t ldv, int k, const TW* w, const double* __restrict__ cin,
                  double* wout, int64_t n, const double* __restrict__ s, double* __restrict__ h,
                  double* __restrict__ c, double* __restrict__ partial, unsigned* __restrict__ counter) {
  double cc[KM], acc[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    cc[j] = j < k ? cin[j] : 0.0;
    acc[j] = 0.0;
  }
  for_vec4(n, UpdateDotBody<TV, TW, KM>{V, ldv, k, w, cc, wout, acc});
  reduce_and_finish<KM>(acc, k, partial, counter, [&](int j, double d) {
    const double sj = s[j];
    h[j] = sj * d;
    c[j] = sj * sj * d;
  });
}

template <typename TV, int KM>
struct UpdateNormBody {
  const TV* V;
  int64_t ldv;
  int k;
  const double* w;
  const double* cc;
  TV* vout;
  double* acc;
  template <int W>
  __device__ __forceinline__ void run(int64_t i) {
    double x[W];
    ld<W>(w + i, x);
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if (j < k) {
        double vv[W];
        ld<W>(V + j * ldv + i, vv);
#pragma unroll
        for (int e = 0; e < W; ++e) x[e] -= cc[j] * vv[e];
      }
    }
    // the norm of the stored (rounded) vector, so s normalises what is kept
#pragma unroll
    for (int e = 0; e < W; ++e) x[e] = (double)(TV)x[e];
    st<W>(vout + i, x);
#pragma unroll
    for (int e = 0; e < W; ++e) acc[0] += x[e] * x[e];
  }
};

template <typename TV, int KM>
__global__ void __launch_bounds__(kThreads)
update_norm_kernel(const TV* __restrict__ V, int64_t ldv, int k, const double* __restrict__ w,
                   const double* __restrict__ cin, TV* __restrict__ vout, int64_t n, double* __restrict__ norm2,
                   double* __restrict__ s_next, double* __restrict__ partial, unsigned* __restrict__ counter) {
  double cc[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) cc[j] = j < k ? cin[j] : 0.0;
  double acc[1] = {0.0};
  for_vec4(n, UpdateNormBody<TV, KM>{V, ldv, k, w, cc, vout, acc});
  reduce_and_finish<1>(acc, 1, partial, counter, [&](int, double d) {
    *norm2 = d;
    *s_next = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
  });
}

template <typename TV, int KM>
struct CombineBody {
  const TV* V;
  int64_t ldv;
  int k;
  const double* cc;
  double* out;
  template <int W>
  __device__ __forceinline__ void run(int64_t i) {
    double x[W];
#pragma unroll
    for (int e = 0; e < W; ++e) x[e] = 0.0;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
      if (j < k) {
        double vv[W];
        ld<W>(V + j * ldv + i, vv);
#pragma unroll
        for (int e = 0; e < W; ++e) x[e] += cc[j] * vv[e];
      }
    }
    st<W>(out + i, x);
  }
};

template <typename TV, int KM>
__global__ void __launch_bounds__(kThreads)
combine_kernel(double* __restrict__ out, const TV* __restrict__ V, int64_t ldv, int k,
               const double* __restrict__ coef, int64_t n) {
  double cc[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) cc[j] = j < k ? coef[j] : 0.0;
  for_vec4(n, CombineBody<TV, KM>{V, ldv, k, cc, out});
}

template <typename TO>
struct CopyBody {
  const double* in;
  TO* out;
  template <int W>
  __device__ __forceinline__ void run(int64_t i) {
    double x[W];
    ld<W>(in + i, x);
    st<W>(out + i, x);
  }
};

template <typename TO>
__global__ void __launch_bounds__(kThreads) copy_kernel(TO* __restrict__ out, const double* __restrict__ in, int64_t n) {
  for_vec4(n, CopyBody<TO>{in, out});
}

int dot_blocks(int64_t n) {
  int64_t b = (n + 16 * kThreads - 1) / (16 * kThreads);
  if (b > kMaxDotBlocks) b = kMaxDotBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

int stream_blocks(int64_t n) {
  int64_t b = (n + 4 * kThreads - 1) / (4 * kThreads);
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

int check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, what);
}

// smallest compiled basis bound that holds k vectors
int km_for(int k) { return k <= 4 ? 4 : (k <= 8 ? 8 : (k <= 12 ? 12 : (k <= 16 ? 16 : 32))); }

}  // namespace

#define STDG_KM_SWITCH(KMV, CALL) \
  switch (KMV) {                       \
    case 4: CALL(4); break;            \
    case 8: CALL(8); break;            \
    case 12: CALL(12); break;          \
    case 16: CALL(16); break;          \
    default: CALL(32); break;          \
  }

int arnoldi_dot(const void* V, bool v32, int64_t ldv, int k, const void* w, bool w32, int64_t n, const double* s,
                double* h, double* c, const DotWork& dw, hipStream_t st) {
  if (k < 1 || k > kMaxBasis) return fail(STDG_E_ARG, "arnoldi_dot: basis size out of range");
  if (ldv % 64) return fail(STDG_E_ARG, "arnoldi_dot: leading dimension must be a multiple of 64");
  const dim3 g(dot_blocks(n)), b(kThreads);
#define STDG_LAUNCH(TV, TW, KM)                                                                                \
  hipLaunchKernelGGL((dot_kernel<TV, TW, KM>), g, b, 0, st, (const TV*)V, ldv, k, (const TW*)w, n, s, h, c, \
                     dw.partial, dw.counter)
#define STDG_FF(KM) STDG_LAUNCH(float, float, KM)
#define STDG_FD(KM) STDG_LAUNCH(float, double, KM)
#define STDG_DF(KM) STDG_LAUNCH(double, float, KM)
#define STDG_DD(KM) STDG_LAUNCH(double, double, KM)
  const int km = km_for(k);
  if (v32) {
    if (w32) { STDG_KM_SWITCH(km, STDG_FF) } else { STDG_KM_SWITCH(km, STDG_FD) }
  } else {
    if (w32) { STDG_KM_SWITCH(km, STDG_DF) } else { STDG_KM_SWITCH(km, STDG_DD) }
  }
#undef STDG_FF
#undef STDG_FD
#undef STDG_DF
#undef STDG_DD
#undef STDG_LAUNCH
  return check_launch("arnoldi_dot");
}

int arnoldi_update_dot(const void* V, bool v32, int64_t ldv, int k, const void* w, bool w32, const double* cin,
                       double* wout, int64_t n, const double* s, double* h, double* c, const DotWork& dw,
                       hipStream_t st) {
  if (k < 1 || k > kMaxBasis) return fail(STDG_E_ARG, "arnoldi_update_dot: basis size out of range");
  if (ldv % 64) return fail(STDG_E_ARG, "arnoldi_update_dot: leading dimension must be a multiple of 64");
  const dim3 g(dot_blocks(n)), b(kThreads);
#define STDG_LAUNCH(TV, TW, KM)                                                                                   \
  hipLaunchKernelGGL((update_dot_kernel<TV, TW, KM>), g, b, 0, st, (const TV*)V, ldv, k, (const TW*)w, cin, wout, \
                     n, s, h, c, dw.partial, dw.counter)
#define STDG_FF(KM) STDG_LAUNCH(float, float, KM)
#define STDG_FD(KM) STDG_LAUNCH(float, double, KM)
#define STDG_DF(KM) STDG_LAUNCH(double, float, KM)
#define STDG_DD(KM) STDG_LAUNCH(double, double, KM)
  const int km = km_for(k);
  if (v32) {
    if (w32) { STDG_KM_SWITCH(km, STDG_FF) } else { STDG_KM_SWITCH(km, STDG_FD) }
  } else {
    if (w32) { STDG_KM_SWITCH(km, STDG_DF) } else { STDG_KM_SWITCH(km, STDG_DD) }
  }
#undef STDG_FF
#undef STDG_FD
#undef STDG_DF
#undef STDG_DD
#undef STDG_LAUNCH
  return check_launch("arnoldi_update_dot");
}

int arnoldi_update_norm(const void* V, bool v32, int64_t ldv, int k, const double* w, const double* cin, void* vout,
                        int64_t n, double* norm2, double* s_next, const DotWork& dw, hipStream_t st) {
  if (k < 1 || k > kMaxBasis) return fail(STDG_E_ARG, "arnoldi_update_norm: basis size out of range");
  if (ldv % 64) return fail(STDG_E_ARG, "arnoldi_update_norm: leading dimension must be a multiple of 64");
  const dim3 g(dot_blocks(n)), b(kThreads);
#define STDG_LAUNCH(TV, KM)                                                                                    \
  hipLaunchKernelGGL((update_norm_kernel<TV, KM>), g, b, 0, st, (const TV*)V, ldv, k, w, cin, (TV*)vout, n, \
                     norm2, s_next, dw.partial, dw.counter)
#define STDG_F(KM) STDG_LAUNCH(float, KM)
#define STDG_D(KM) STDG_LAUNCH(double, KM)
  const int km = km_for(k);
  if (v32) { STDG_KM_SWITCH(km, STDG_F) } else { STDG_KM_SWITCH(km, STDG_D) }
#undef STDG_F
#undef STDG_D
#undef STDG_LAUNCH
  return check_launch("arnoldi_update_norm");
}

int vec_dot(const double* a, const double* b, int64_t n, double* out, const DotWork& dw, hipStream_t st) {
  const dim3 g(dot_blocks(n)), bl(kThreads);
  hipLaunchKernelGGL((dot_kernel<double, double, 1>), g, bl, 0, st, a, 0, 1, b, n, nullptr, out, nullptr, dw.partial,
                     dw.counter);
  return check_launch("vec_dot");
}

int basis_combine(double* out, const void* V, bool v32, int64_t ldv, int k, const double* coef, int64_t n,
                  hipStream_t st) {
  if (k < 1 || k > kMaxBasis) return fail(STDG_E_ARG, "basis_combine: basis size out of range");
  if (ldv % 64) return fail(STDG_E_ARG, "basis_combine: leading dimension must be a multiple of 64");
  const dim3 g(stream_blocks(n)), b(kThreads);
#define STDG_F(KM) hipLaunchKernelGGL((combine_kernel<float, KM>), g, b, 0, st, out, (const float*)V, ldv, k, coef, n)
#define STDG_D(KM) hipLaunchKernelGGL((combine_kernel<double, KM>), g, b, 0, st, out, (const double*)V, ldv, k, coef, n)
  const int km = km_for(k);
  if (v32) { STDG_KM_SWITCH(km, STDG_F) } else { STDG_KM_SWITCH(km, STDG_D) }
#undef STDG_F
#undef STDG_D
  return check_launch("basis_combine");
}

int vec_store(void* out, bool out32, const double* in, int64_t n, hipStream_t st) {
  const dim3 g(stream_blocks(n)), b(kThreads);
  if (out32)
    hipLaunchKernelGGL(copy_kernel<float>, g, b, 0, st, (float*)out, in, n);
  else
    hipLaunchKernelGGL(copy_kernel<double>, g, b, 0, st, (double*)out, in, n);
  return check_launch("vec_store");
}

#undef STDG_KM_SWITCH

}  // namespace stdg
