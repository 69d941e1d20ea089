// Arnoldi kernels of the slab GMRES (Section 5.4): classical Gram-Schmidt
// applied twice, with the second projection of each new basis vector
// delayed into the next iteration, so that an iteration makes two passes over
// the basis instead of three; the Hessenberg column, its Givens rotation and
// the stopping test run on the device, so that a whole restart cycle runs
// without the host.
//
// Iteration j (V_0 .. V_{j-1} formed and orthonormal; w the previous
// iteration's vector after one projection, whose second-projection
// coefficients hp = V^T w and norm estimate nu = sqrt(|w|^2 - |hp|^2) are
// known; for j = 0 nothing is pending and V_0 is the start vector):
//   z = B P^{-1} w (z = B P^{-1} V_0 for j = 0)                    [the apply]
//   pass 1: c_l = V_l . z (l < j), d = w . z; then, with the pending
//           V_j = (w - sum_l hp_l V_l) / nu, V_j . z = (d - hp . c) / nu, and
//           A V_j = (z - V H hp) / nu gives the Hessenberg entries
//           h_l = (V_l . z - (H hp)_l) / nu, l <= j
//   pass 2: V_j formed and stored; w' = (z - sum_{l<=j} (V_l . z) V_l) / nu
//           (the first projection of A V_j: the V H hp part lies in the
//           span), e_l = V_l . w', |w'|^2; column j of H = h + e, its
//           subdiagonal sqrt(|w'|^2 - |e|^2); Givens rotation, residual
//           estimate |g_{j+1}| and the stopping test; w', e carried on.
// At the cycle end the least-squares solution y = R^{-1} g combines the
// formed vectors V_0 .. V_{k-1}.  All sums are FP64; reductions are
// deterministic: fixed-order block reductions, per-block partials, and the
// last block to finish (detected with a device-scope counter) sums the
// partials in block order and resets the counter.  Each thread streams 4
// consecutive entries per step with 16-byte loads; basis slots therefore
// have a leading dimension that is a multiple of 64.
#include <cstring>

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

// Block-reduce acc[0..k) into partial[j * kMaxDotBlocks + blk]; the last
// block to arrive reduces the partials over blocks (every partial of every j
// loaded at once, each thread summing blocks tid, tid + kThreads, .. in
// order, then the same wave and block sums as the first stage) and calls
// fin(j, total) on thread j.  Returns true on every thread of the last block
// (after a barrier, so fin's LDS writes are visible), false elsewhere; the
// counter is left zero.
template <int KM, typename Fin>
__device__ __forceinline__ bool reduce_and_finish(const double (&acc)[KM], int k, double* __restrict__ partial,
                                                  unsigned* __restrict__ counter, Fin fin, uint32_t blk,
                                                  uint32_t nblk) {
  __shared__ double wsum[kWaves][KM];
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
    partial[(int64_t)threadIdx.x * kMaxDotBlocks + blk] = v;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(counter, 1u) == nblk - 1;
  __syncthreads();
  if (!last) return false;
  __threadfence();
  const int nb = (int)nblk;
  double s[KM];
#pragma unroll
  for (int j = 0; j < KM; ++j) s[j] = 0.0;
  for (int b = threadIdx.x; b < nb; b += kThreads) {
#pragma unroll
    for (int j = 0; j < KM; ++j)
      if (j < k) s[j] += load_agent(partial + (int64_t)j * kMaxDotBlocks + b);
  }
#pragma unroll
  for (int j = 0; j < KM; ++j) {
    if (j >= k) break;
    const double v = wave_sum(s[j]);
    if (lane == 0) wsum[wave][j] = v;
  }
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) v += wsum[w][threadIdx.x];
    fin((int)threadIdx.x, v);
  }
  __syncthreads();
  if (threadIdx.x == 0) atomicExch(counter, 0u);
  return true;
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
// Blocks blk of nblk (a kernel's own grid, or one request's segment of a
// batched grid).
template <typename Body>
__device__ __forceinline__ void for_vec4(int64_t n, Body body, uint32_t blk, uint32_t nblk) {
  const int64_t n4 = n >> 2, stride = (int64_t)nblk * kThreads;
  for (int64_t q = (int64_t)blk * kThreads + threadIdx.x; q < n4; q += stride)
    body.template run<4>(q << 2);
  const int64_t tail = n - (n4 << 2);
  if (blk == 0 && (int64_t)threadIdx.x < tail) body.template run<1>((n4 << 2) + threadIdx.x);
}
template <typename Body>
__device__ __forceinline__ void for_vec4(int64_t n, Body body) {
  for_vec4(n, body, blockIdx.x, gridDim.x);
}


// Block-reduce acc[0..k) into per-block partials; in the last block to
// finish, thread 0 gets the totals 0..k) as an LDS array (indexed at run time
// without private scratch memory); NULL everywhere else.  Resets the counter.
template <int KM>
__device__ __forceinline__ const double* reduce_totals(const double (&acc)[KM], int k, double* __restrict__ partial,
                                                       unsigned* __restrict__ counter, uint32_t blk, uint32_t nblk) {
  __shared__ double stot[KM];
  const bool last = reduce_and_finish<KM>(acc, k, partial, counter, [&](int j, double d) { stot[j] = d; }, blk, nblk);
  return last ? stot : nullptr;
}

// coefficients c[0..k) (zero past k) into an LDS array: read by every thread
// at each use instead of held in scalar registers, whose file is too small
// for KM doubles
template <int KM>
__device__ __forceinline__ const double* coef_lds(const double* __restrict__ c, int k) {
  __shared__ double sc[KM];
  if ((int)threadIdx.x < KM) sc[threadIdx.x] = (int)threadIdx.x < k ? c[threadIdx.x] : 0.0;
  __syncthreads();
  return sc;
}

template <typename TV>
__device__ __forceinline__ double round_to(double v) { return (double)(TV)v; }

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
  }, blockIdx.x, gridDim.x);
}


template <typename TV, typename TZ, typename TW, int KM>
struct Pass1Body {
  const TV* V;
  int64_t ldv;
  int j;
  const TZ* z;
  const TW* w;
  double* acc;
  template <int W>
  __device__ __forceinline__ void run(int64_t i) {
    double zv[W];
    ld<W>(z + i, zv);
#pragma unroll
    for (int l = 0; l < KM; ++l) {
      if (l < j) {
        double vv[W];
        ld<W>(V + l * ldv + i, vv);
#pragma unroll
        for (int e = 0; e < W; ++e) acc[l] += vv[e] * zv[e];
      }
    }
    double wv[W];
    if (j > 0) ld<W>(w + i, wv); else ld<W>(V + i, wv);
#pragma unroll
    for (int e = 0; e < W; ++e) acc[j] += wv[e] * zv[e];
  }
};

// pass 1: c = V^T z (and d = w . z), then the Hessenberg entries h of
// column j and the update coefficients of pass 2
template <typename TV, typename TZ, typename TW, int KM>
__device__ __forceinline__ void pass1_run(const TV* __restrict__ V, int64_t ldv, int j, const TZ* __restrict__ z,
                                          const TW* __restrict__ w, int64_t n, CycleCtl* __restrict__ ctl,
                                          double* __restrict__ partial, unsigned* __restrict__ counter, uint32_t blk,
                                          uint32_t nblk) {
  if (!ctl->active) return;
  double acc[KM];
#pragma unroll
  for (int l = 0; l < KM; ++l) acc[l] = 0.0;
  for_vec4(n, Pass1Body<TV, TZ, TW, KM>{V, ldv, j, z, w, acc}, blk, nblk);
  // the last block (all its threads): the Hessenberg entries of column j,
  // lanes l <= j in parallel from the control block staged in LDS
  const double* tot = reduce_totals<KM>(acc, j + 1, partial, counter, blk, nblk);
  if (!tot) return;
  const int t = threadIdx.x;
  if (j == 0) {
    if (t == 0) {
      ctl->h[0] = tot[0];
      ctl->cz[0] = tot[0];
      ctl->inv_nu = 1.0;
    }
    return;
  }
  __shared__ double shp[kMaxBasis], sc[kMaxBasis];
  __shared__ double sinv;
  if (t < j) shp[t] = ctl->hp[t];
  if (t == 0) sinv = 1.0 / ctl->nu;
  __syncthreads();
  const double inv = sinv;
  if (t == 0) {
    double v = tot[j];
    for (int l = 0; l < j; ++l) v -= shp[l] * tot[l];
    sc[j] = v * inv;
  } else if (t <= j) {
    sc[t - 1] = tot[t - 1];
  }
  __syncthreads();
  if (t <= j) {
    double g = 0.0;  // (H hp)_l over the columns 0 .. j-1
    for (int i = (t > 0 ? t - 1 : 0); i < j; ++i) g += ctl->Hraw[t * kMaxBasis + i] * shp[i];
    ctl->h[t] = (sc[t] - g) * inv;
    ctl->cz[t] = sc[t] * inv;
  }
  if (t == 0) ctl->inv_nu = inv;
}

template <typename TV, typename TZ, typename TW, int KM>
__global__ void __launch_bounds__(kThreads)
pass1_kernel(const TV* __restrict__ V, int64_t ldv, int j, const TZ* __restrict__ z, const TW* __restrict__ w,
             int64_t n, CycleCtl* __restrict__ ctl, double* __restrict__ partial, unsigned* __restrict__ counter) {
  pass1_run<TV, TZ, TW, KM>(V, ldv, j, z, w, n, ctl, partial, counter, blockIdx.x, gridDim.x);
}

template <typename TV, typename TZ, typename TW, int KM>
struct Pass2Body {
  TV* V;
  int64_t ldv;
  int j;
  const TZ* z;
  TW* w;
  float* w32;
  const double* hp;  // second-projection coefficients of the pending vector
  const double* cz;  // (V_l . z) / nu
  double inv;
  double* acc;
  template <int W>
  __device__ __forceinline__ void run(int64_t i) {
    // first sweep over the basis: the pending vector's second projection
    // and the first projection of z, one read of each V_l
    double xj[W], xw[W];
    if (j > 0) ld<W>(w + i, xj);
    ld<W>(z + i, xw);
#pragma unroll
    for (int e = 0; e < W; ++e) xw[e] *= inv;
#pragma unroll
    for (int l = 0; l < KM; ++l) {
      if (l < j) {
        double vv[W];
        ld<W>(V + l * ldv + i, vv);
#pragma unroll
        for (int e = 0; e < W; ++e) {
          xj[e] -= hp[l] * vv[e];
          xw[e] -= cz[l] * vv[e];
        }
      }
    }
    double vj[W], wn[W];
    if (j > 0) {
#pragma unroll
      for (int e = 0; e < W; ++e) vj[e] = round_to<TV>(xj[e] * inv);
      st<W>(V + j * ldv + i, vj);
    } else {
      ld<W>(V + i, vj);
    }
#pragma unroll
    for (int e = 0; e < W; ++e) wn[e] = round_to<TW>(xw[e] - cz[j] * vj[e]);
    st<W>(w + i, wn);
    if (w32) st<W>(w32 + i, wn);
    // second sweep: the dots with w' (the V_l entries are read again, from
    // cache: keeping them in registers across both sweeps cost occupancy)
#pragma unroll
    for (int l = 0; l < KM; ++l) {
      if (l < j) {
        double vv[W];
        ld<W>(V + l * ldv + i, vv);
#pragma unroll
        for (int e = 0; e < W; ++e) acc[l] += vv[e] * wn[e];
      }
    }
#pragma unroll
    for (int e = 0; e < W; ++e) {
      acc[j] += vj[e] * wn[e];
      acc[j + 1] += wn[e] * wn[e];
    }
  }
};

// pass 2: V_j formed, w' = (z - V (V^T z)) / nu, e = V^T w', |w'|^2; then the
// Hessenberg column, its Givens rotation and the stopping test
template <typename TV, typename TZ, typename TW, int KM>
__device__ __forceinline__ void pass2_run(TV* __restrict__ V, int64_t ldv, int j, const TZ* __restrict__ z, TW* w,
                                          float* w32, int64_t n, CycleCtl* __restrict__ ctl,
                                          double* __restrict__ partial, unsigned* __restrict__ counter, uint32_t blk,
                                          uint32_t nblk) {
  if (!ctl->active) return;
  // hp and cz stay uniform (scalar registers, spilled to vector lanes
  // for large KM): held in LDS the compiler hoists them into vector
  // registers instead, which costs two occupancy steps
  double hp[KM], cz[KM], acc[KM];
#pragma unroll
  for (int l = 0; l < KM; ++l) {
    hp[l] = l < j ? ctl->hp[l] : 0.0;
    cz[l] = l <= j ? ctl->cz[l] : 0.0;
    acc[l] = 0.0;
  }
  const double inv = ctl->inv_nu;
  for_vec4(n, Pass2Body<TV, TZ, TW, KM>{V, ldv, j, z, w, w32, hp, cz, inv, acc}, blk, nblk);
  const double* tot = reduce_totals<KM>(acc, j + 2, partial, counter, blk, nblk);
  if (!tot) return;
  // the last block (all its threads): column j of H from both projections,
  // its subdiagonal from the norm of w' after its second projection
  // (Pythagoras: V is orthonormal), the Givens rotations and the stopping
  // test; the control block is staged in LDS by lanes in parallel and the
  // sequential recurrences run on thread 0 from LDS
  const int t = threadIdx.x;
  __shared__ double col[kMaxBasis + 1], scs[kMaxBasis], ssn[kMaxBasis];
  if (t <= j) {
    col[t] = ctl->h[t] + tot[t];
    ctl->hp[t] = tot[t];
  }
  if (t < j) {
    scs[t] = ctl->cs[t];
    ssn[t] = ctl->sn[t];
  }
  __syncthreads();
  if (t == 0) {
    const double s2 = tot[j + 1];
    double e2 = 0.0;
    for (int l = 0; l <= j; ++l) e2 += tot[l] * tot[l];
    const double r2 = s2 - e2;
    // breakdown: w' lies in the span of V to rounding (the Krylov space is invariant)
    const double nu = (r2 > 1e-28 * s2 && r2 > 0.0) ? sqrt(r2) : 0.0;
    col[j + 1] = nu;
    ctl->nu = nu;
  }
  __syncthreads();
  if (t <= j + 1) ctl->Hraw[t * kMaxBasis + j] = col[t];
  __syncthreads();  // the raw column is stored before thread 0 rotates it in place
  if (t == 0) {
    for (int i = 0; i < j; ++i) {
      const double a = scs[i] * col[i] + ssn[i] * col[i + 1];
      col[i + 1] = -ssn[i] * col[i] + scs[i] * col[i + 1];
      col[i] = a;
    }
    const double nu = col[j + 1];
    const double den = hypot(col[j], col[j + 1]);
    const double cs = den > 0.0 ? col[j] / den : 1.0, sn = den > 0.0 ? col[j + 1] / den : 0.0;
    ctl->cs[j] = cs;
    ctl->sn[j] = sn;
    col[j] = den;
    const double gj = ctl->g[j];
    const double g1 = -sn * gj;
    ctl->g[j + 1] = g1;
    ctl->g[j] = cs * gj;
    ctl->k = j + 1;
    const int iters = ctl->iters + 1;
    ctl->iters = iters;
    const bool finite = isfinite(nu) && isfinite(den) && isfinite(g1);
    if (!finite) ctl->bad = 1;
    if (!finite || fabs(g1) <= ctl->target || nu == 0.0 || den == 0.0 || j + 1 >= ctl->restart ||
        iters >= ctl->max_iters)
      ctl->active = 0;
  }
  __syncthreads();
  if (t <= j) ctl->R[t * kMaxBasis + j] = col[t];
}

template <typename TV, typename TZ, typename TW, int KM>
__global__ void __launch_bounds__(kThreads)
pass2_kernel(TV* __restrict__ V, int64_t ldv, int j, const TZ* __restrict__ z, TW* w, float* w32, int64_t n,
             CycleCtl* __restrict__ ctl, double* __restrict__ partial, unsigned* __restrict__ counter) {
  pass2_run<TV, TZ, TW, KM>(V, ldv, j, z, w, w32, n, ctl, partial, counter, blockIdx.x, gridDim.x);
}

// cycle start: V_0 = r / |r| from the residual r and its squared norm, the
// least-squares state reset (one thread of block 0)
template <typename TV>
__device__ __forceinline__ void cycle_start_run(const double* r, const double* __restrict__ norm2, TV* v0,
                                                float* __restrict__ v32, int64_t n, CycleCtl* __restrict__ ctl,
                                                uint32_t blk, uint32_t nblk) {
  // r and v0 may be the same memory (an FP64 basis holds the residual in slot 0): in place, entry by entry
  const double beta = sqrt(*norm2);
  const double inv = beta > 0.0 ? 1.0 / beta : 0.0;
  const int64_t stride = (int64_t)nblk * kThreads;
  for (int64_t i = (int64_t)blk * kThreads + threadIdx.x; i < n; i += stride) {
    const double v = round_to<TV>(r[i] * inv);
    v0[i] = (TV)v;
    if (v32) v32[i] = (float)v;
  }
  if (blk == 0 && threadIdx.x == 0) {
    ctl->active = beta > 0.0 ? 1 : 0;
    ctl->k = 0;
    ctl->bad = 0;
    ctl->nu = 1.0;
    ctl->g[0] = beta;
    for (int l = 1; l <= kMaxBasis; ++l) ctl->g[l] = 0.0;
  }
}

template <typename TV>
__global__ void __launch_bounds__(kThreads)
cycle_start_kernel(const double* r, const double* __restrict__ norm2, TV* v0, float* __restrict__ v32, int64_t n,
                   CycleCtl* __restrict__ ctl) {
  cycle_start_run<TV>(r, norm2, v0, v32, n, ctl, blockIdx.x, gridDim.x);
}

// cycle end: y = R^{-1} g over the k columns done, coefficients -y (the
// Krylov system is solved for the negated residual)
__device__ __forceinline__ void least_squares_run(CycleCtl* __restrict__ ctl) {
  const int k = ctl->k;
  __shared__ double y[kMaxBasis];
  for (int i = k - 1; i >= 0; --i) {
    double t = ctl->g[i];
    for (int l = i + 1; l < k; ++l) t -= ctl->R[i * kMaxBasis + l] * y[l];
    y[i] = t / ctl->R[i * kMaxBasis + i];
  }
  for (int i = 0; i < kMaxBasis; ++i) ctl->y[i] = i < k ? -y[i] : 0.0;
}

__global__ void least_squares_kernel(CycleCtl* __restrict__ ctl) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  least_squares_run(ctl);
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
__device__ __forceinline__ void combine_run(double* __restrict__ out, const TV* __restrict__ V, int64_t ldv, int k,
                                            const int* __restrict__ kdev, const double* __restrict__ coef, int64_t n,
                                            uint32_t blk, uint32_t nblk) {
  if (kdev) k = *kdev;
  const double* cc = coef_lds<KM>(coef, k);
  for_vec4(n, CombineBody<TV, KM>{V, ldv, k, cc, out}, blk, nblk);
}

template <typename TV, int KM>
__global__ void __launch_bounds__(kThreads)
combine_kernel(double* __restrict__ out, const TV* __restrict__ V, int64_t ldv, int k, const int* __restrict__ kdev,
               const double* __restrict__ coef, int64_t n) {
  combine_run<TV, KM>(out, V, ldv, k, kdev, coef, n, blockIdx.x, gridDim.x);
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

// ---- batched cycle kernels: one request per segment of the grid -----------

struct SegK {
  void* V;
  int64_t ldv;
  const void* z;
  void* w;
  float* w32;
  const double* r;
  const double* norm2;
  double* out;
  int64_t n;
  CycleCtl* ctl;
  double* partial;
  unsigned* counter;
  uint32_t first, nblk;  // the segment's blocks in the grid
};
struct SegBatch {
  SegK s[kMaxBatch];
  int count, j, k;
};

// the segment that owns grid block b (uniform over the block)
__device__ __forceinline__ int seg_of(const SegBatch& B, uint32_t b) {
  int m = 0;
  for (int k = 1; k < B.count; ++k)
    if (b >= B.s[k].first) m = k;
  return m;
}

template <typename TV, typename TZ, typename TW, int KM>
__global__ void __launch_bounds__(kThreads) pass1_batch_kernel(SegBatch B) {
  const SegK& S = B.s[seg_of(B, blockIdx.x)];
  pass1_run<TV, TZ, TW, KM>((const TV*)S.V, S.ldv, B.j, (const TZ*)S.z, (const TW*)S.w, S.n, S.ctl, S.partial,
                            S.counter, blockIdx.x - S.first, S.nblk);
}

template <typename TV, typename TZ, typename TW, int KM>
__global__ void __launch_bounds__(kThreads) pass2_batch_kernel(SegBatch B) {
  const SegK& S = B.s[seg_of(B, blockIdx.x)];
  pass2_run<TV, TZ, TW, KM>((TV*)S.V, S.ldv, B.j, (const TZ*)S.z, (TW*)S.w, S.w32, S.n, S.ctl, S.partial, S.counter,
                            blockIdx.x - S.first, S.nblk);
}

template <typename TV>
__global__ void __launch_bounds__(kThreads) cycle_start_batch_kernel(SegBatch B) {
  const SegK& S = B.s[seg_of(B, blockIdx.x)];
  cycle_start_run<TV>(S.r, S.norm2, (TV*)S.V, S.w32, S.n, S.ctl, blockIdx.x - S.first, S.nblk);
}

__global__ void least_squares_batch_kernel(SegBatch B) {
  if (threadIdx.x != 0 || (int)blockIdx.x >= B.count) return;
  least_squares_run(B.s[blockIdx.x].ctl);
}

template <typename TV, int KM>
__global__ void __launch_bounds__(kThreads) combine_batch_kernel(SegBatch B) {
  const SegK& S = B.s[seg_of(B, blockIdx.x)];
  combine_run<TV, KM>(S.out, (const TV*)S.V, S.ldv, B.k, &S.ctl->k, S.ctl->y, S.n, blockIdx.x - S.first, S.nblk);
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
int km_for(int k) {
  if (k <= 12) return k <= 2 ? 2 : (k <= 4 ? 4 : (k <= 6 ? 6 : (k <= 8 ? 8 : (k <= 10 ? 10 : 12))));
  return 16;
}

// blocks for a grid-stride reduction kernel: as many as the device holds at
// once (no partial second wave of blocks), at most kMaxDotBlocks partials
template <typename K>
int resident_blocks(K kernel, int64_t n) {
  static int per_cu = 0, cus = 0;  // per instantiation; one device type per process
  if (per_cu == 0) {
    int nb = 0, dev = 0, c = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, kThreads, 0) != hipSuccess || nb < 1) nb = 1;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
      c = 256;
    cus = c;
    per_cu = nb;
  }
  int64_t b = (int64_t)per_cu * cus;
  const int64_t need = (n + 4 * kThreads - 1) / (4 * kThreads);
  if (b > need) b = need;
  if (b > kMaxDotBlocks) b = kMaxDotBlocks;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

#define STDG_KM_SWITCH(KMV, CALL) \
  switch (KMV) {                       \
    case 2: CALL(2); break;            \
    case 4: CALL(4); break;            \
    case 6: CALL(6); break;            \
    case 8: CALL(8); break;            \
    case 10: CALL(10); break;          \
    case 12: CALL(12); break;          \
    default: CALL(16); break;          \
  }

// precision combinations of (basis, apply output, pending vector)
#define STDG_PRECS(CALL, KM)                                   \
  if (v32) { CALL(float, float, float, KM); }                  \
  else if (z32) { CALL(double, float, double, KM); }           \
  else { CALL(double, double, double, KM); }

int arnoldi_pass1(const void* V, bool v32, int64_t ldv, int j, const void* z, bool z32, const void* w, int64_t n,
                  CycleCtl* ctl, const DotWork& dw, hipStream_t st) {
  if (j < 0 || j + 1 > kMaxBasis) return fail(STDG_E_ARG, "arnoldi_pass1: basis index out of range");
  if (ldv % 64) return fail(STDG_E_ARG, "arnoldi_pass1: leading dimension must be a multiple of 64");
  if (v32 && !z32) return fail(STDG_E_ARG, "arnoldi_pass1: an FP32 basis needs FP32 applies");
  const dim3 b(kThreads);
#define STDG_L(TV, TZ, TW, KM)                                                                                 \
  hipLaunchKernelGGL((pass1_kernel<TV, TZ, TW, KM>), dim3(resident_blocks(pass1_kernel<TV, TZ, TW, KM>, n)), b, \
                     0, st, (const TV*)V, ldv, j, (const TZ*)z, (const TW*)w, n, ctl, dw.partial, dw.counter)
#define STDG_K(KM) STDG_PRECS(STDG_L, KM)
  STDG_KM_SWITCH(km_for(j + 1), STDG_K)
#undef STDG_K
#undef STDG_L
  return check_launch("arnoldi_pass1");
}

int arnoldi_pass2(void* V, bool v32, int64_t ldv, int j, const void* z, bool z32, void* w, float* w32, int64_t n,
                  CycleCtl* ctl, const DotWork& dw, hipStream_t st) {
  if (j < 0 || j + 2 > kMaxBasis) return fail(STDG_E_ARG, "arnoldi_pass2: basis index out of range");
  if (ldv % 64) return fail(STDG_E_ARG, "arnoldi_pass2: leading dimension must be a multiple of 64");
  if (v32 && !z32) return fail(STDG_E_ARG, "arnoldi_pass2: an FP32 basis needs FP32 applies");
  const dim3 b(kThreads);
#define STDG_L(TV, TZ, TW, KM)                                                                                     \
  hipLaunchKernelGGL((pass2_kernel<TV, TZ, TW, KM>), dim3(resident_blocks(pass2_kernel<TV, TZ, TW, KM>, n)), b,  \
                     0, st, (TV*)V, ldv, j, (const TZ*)z, (TW*)w, w32, n, ctl, dw.partial, dw.counter)
#define STDG_K(KM) STDG_PRECS(STDG_L, KM)
  STDG_KM_SWITCH(km_for(j + 2), STDG_K)
#undef STDG_K
#undef STDG_L
  return check_launch("arnoldi_pass2");
}

// Segment table of a batch: blocks(n) blocks per request, in order.
template <typename F>
int make_batch(const CycleSeg* segs, int count, F blocks, SegBatch* B, uint32_t* total) {
  if (count < 1 || count > kMaxBatch) return fail(STDG_E_ARG, "batched cycle kernel: 1 to kMaxBatch requests");
  std::memset(B, 0, sizeof(*B));
  uint64_t first = 0;
  for (int i = 0; i < count; ++i) {
    const CycleSeg& c = segs[i];
    SegK& k = B->s[i];
    k.V = c.V;
    k.ldv = c.ldv;
    k.z = c.z;
    k.w = c.w;
    k.w32 = c.w32;
    k.r = c.r;
    k.norm2 = c.norm2;
    k.out = c.out;
    k.n = c.n;
    k.ctl = c.ctl;
    k.partial = c.dw.partial;
    k.counter = c.dw.counter;
    k.first = (uint32_t)first;
    k.nblk = (uint32_t)blocks(c.n);
    first += k.nblk;
  }
  if (first > 0x7fffffffu) return fail(STDG_E_ARG, "batched cycle kernel: grid too large");
  B->count = count;
  *total = (uint32_t)first;
  return STDG_OK;
}

int arnoldi_pass1_batch(const CycleSeg* segs, int count, bool v32, bool z32, int j, hipStream_t st) {
  if (j < 0 || j + 1 > kMaxBasis) return fail(STDG_E_ARG, "arnoldi_pass1_batch: basis index out of range");
  if (v32 && !z32) return fail(STDG_E_ARG, "arnoldi_pass1_batch: an FP32 basis needs FP32 applies");
  SegBatch B;
  uint32_t total = 0;
  int rc;
  // each request's blocks as in its own launch (resident_blocks of the plain kernel)
#define STDG_L(TV, TZ, TW, KM)                                                                                   \
  if ((rc = make_batch(segs, count, [](int64_t n) { return resident_blocks(pass1_kernel<TV, TZ, TW, KM>, n); }, \
                       &B, &total)) != STDG_OK)                                                                  \
    return rc;                                                                                                   \
  B.j = j;                                                                                                       \
  hipLaunchKernelGGL((pass1_batch_kernel<TV, TZ, TW, KM>), dim3(total), dim3(kThreads), 0, st, B)
#define STDG_K(KM) STDG_PRECS(STDG_L, KM)
  STDG_KM_SWITCH(km_for(j + 1), STDG_K)
#undef STDG_K
#undef STDG_L
  return check_launch("arnoldi_pass1_batch");
}

int arnoldi_pass2_batch(const CycleSeg* segs, int count, bool v32, bool z32, int j, hipStream_t st) {
  if (j < 0 || j + 2 > kMaxBasis) return fail(STDG_E_ARG, "arnoldi_pass2_batch: basis index out of range");
  if (v32 && !z32) return fail(STDG_E_ARG, "arnoldi_pass2_batch: an FP32 basis needs FP32 applies");
  SegBatch B;
  uint32_t total = 0;
  int rc;
#define STDG_L(TV, TZ, TW, KM)                                                                                   \
  if ((rc = make_batch(segs, count, [](int64_t n) { return resident_blocks(pass2_kernel<TV, TZ, TW, KM>, n); }, \
                       &B, &total)) != STDG_OK)                                                                  \
    return rc;                                                                                                   \
  B.j = j;                                                                                                       \
  hipLaunchKernelGGL((pass2_batch_kernel<TV, TZ, TW, KM>), dim3(total), dim3(kThreads), 0, st, B)
#define STDG_K(KM) STDG_PRECS(STDG_L, KM)
  STDG_KM_SWITCH(km_for(j + 2), STDG_K)
#undef STDG_K
#undef STDG_L
  return check_launch("arnoldi_pass2_batch");
}

#undef STDG_PRECS

int cycle_start_batch(const CycleSeg* segs, int count, bool v32, hipStream_t st) {
  SegBatch B;
  uint32_t total = 0;
  int rc = make_batch(segs, count, [](int64_t n) { return stream_blocks(n); }, &B, &total);
  if (rc != STDG_OK) return rc;
  if (v32)
    hipLaunchKernelGGL(cycle_start_batch_kernel<float>, dim3(total), dim3(kThreads), 0, st, B);
  else
    hipLaunchKernelGGL(cycle_start_batch_kernel<double>, dim3(total), dim3(kThreads), 0, st, B);
  return check_launch("cycle_start_batch");
}

int cycle_least_squares_batch(const CycleSeg* segs, int count, hipStream_t st) {
  SegBatch B;
  uint32_t total = 0;
  int rc = make_batch(segs, count, [](int64_t) { return 1; }, &B, &total);
  if (rc != STDG_OK) return rc;
  hipLaunchKernelGGL(least_squares_batch_kernel, dim3(count), dim3(64), 0, st, B);
  return check_launch("cycle_least_squares_batch");
}

int basis_combine_batch(const CycleSeg* segs, int count, bool v32, int kmax, hipStream_t st) {
  if (kmax < 1 || kmax > kMaxBasis) return fail(STDG_E_ARG, "basis_combine_batch: basis size out of range");
  SegBatch B;
  uint32_t total = 0;
  int rc = make_batch(segs, count, [](int64_t n) { return stream_blocks(n); }, &B, &total);
  if (rc != STDG_OK) return rc;
  B.k = kmax;
#define STDG_F(KM) hipLaunchKernelGGL((combine_batch_kernel<float, KM>), dim3(total), dim3(kThreads), 0, st, B)
#define STDG_D(KM) hipLaunchKernelGGL((combine_batch_kernel<double, KM>), dim3(total), dim3(kThreads), 0, st, B)
  const int km = km_for(kmax);
  if (v32) { STDG_KM_SWITCH(km, STDG_F) } else { STDG_KM_SWITCH(km, STDG_D) }
#undef STDG_F
#undef STDG_D
  return check_launch("basis_combine_batch");
}

int cycle_start(const double* r, const double* norm2, void* v0, bool v32, float* v0_32, int64_t n, CycleCtl* ctl,
                hipStream_t st) {
  const dim3 g(stream_blocks(n)), b(kThreads);
  if (v32)
    hipLaunchKernelGGL(cycle_start_kernel<float>, g, b, 0, st, r, norm2, (float*)v0, v0_32, n, ctl);
  else
    hipLaunchKernelGGL(cycle_start_kernel<double>, g, b, 0, st, r, norm2, (double*)v0, v0_32, n, ctl);
  return check_launch("cycle_start");
}

int cycle_least_squares(CycleCtl* ctl, hipStream_t st) {
  hipLaunchKernelGGL(least_squares_kernel, dim3(1), dim3(64), 0, st, ctl);
  return check_launch("cycle_least_squares");
}

int vec_dot(const double* a, const double* b, int64_t n, double* out, const DotWork& dw, hipStream_t st) {
  const dim3 g(dot_blocks(n)), bl(kThreads);
  hipLaunchKernelGGL((dot_kernel<double, double, 1>), g, bl, 0, st, a, 0, 1, b, n, nullptr, out, nullptr, dw.partial,
                     dw.counter);
  return check_launch("vec_dot");
}

int basis_combine(double* out, const void* V, bool v32, int64_t ldv, int k, const int* kdev, const double* coef,
                  int64_t n, hipStream_t st) {
  if (k < 1 || k > kMaxBasis) return fail(STDG_E_ARG, "basis_combine: basis size out of range");
  if (ldv % 64) return fail(STDG_E_ARG, "basis_combine: leading dimension must be a multiple of 64");
  const dim3 g(stream_blocks(n)), b(kThreads);
#define STDG_F(KM) \
  hipLaunchKernelGGL((combine_kernel<float, KM>), g, b, 0, st, out, (const float*)V, ldv, k, kdev, coef, n)
#define STDG_D(KM) \
  hipLaunchKernelGGL((combine_kernel<double, KM>), g, b, 0, st, out, (const double*)V, ldv, k, kdev, coef, n)
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
