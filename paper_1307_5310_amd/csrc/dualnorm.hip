// Dual norms of the residual on trilinear elements (Section 5.3, the norm of
// W_h' behind eq. a_posteriori:iteration): per element and test level the
// Riesz representor of R_i in L2(I_n; L2(K)) solves (dt M_K) z = R_i with M_K
// the element's unit-coefficient mass, and ||R||^2 = sum R_i . z.  On
// trilinear elements M_K is not the centre metric times the identity, so each
// solve is a conjugate-gradient iteration on the sum-factorised quadrature
// mass of the residual (the (p + 2)-point Gauss rule of the residual's own mass
// term), preconditioned by the block mass with the metric at the element
// centre, run to 1e-14 of the right-hand side.  One workgroup per element,
// FP64; both fields at once (the unit mass is the same block for E and H).
#include "residual_kernel.h"

namespace stdg {

namespace {

// (a, b) summed over the workgroup, returned to every thread
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, 64);
    b += __shfl_xor(b, off, 64);
  }
  constexpr int NW = NT / 64;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();  // red may still be read from the previous call
  if (lane == 0) {
    red[2 * wave] = a;
    red[2 * wave + 1] = b;
  }
  __syncthreads();
  a = 0.0;
  b = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    a += red[2 * w];
    b += red[2 * w + 1];
  }
}

template <int A>
__global__ void __launch_bounds__(KCfg<A>::NT)
dual_norm_trilinear_kernel(const ElemInfo* __restrict__ info, const ElemMetric* __restrict__ metric,
                           const double* __restrict__ verts, const QTables<double>* __restrict__ qt,
                           const int32_t* __restrict__ list, const double* __restrict__ R, double* __restrict__ partial) {
  using C = KCfg<A>;
  constexpr int A3 = C::A3, NT = C::NT;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  double* sm = reinterpret_cast<double*>(smem_raw);
  double* qB = sm + C::MASS;
  double* Gl = qB + C::QTAB_PAD;
  double* red = Gl + 6 * C::G3;
  const int tid = threadIdx.x;
  const int e = list[blockIdx.x];
  const ElemInfo I = info[e];
  const int q = I.q;
  const bool pos_lane = tid < A3;
  const uint32_t s = pos_lane ? (uint32_t)tid : 0u;
  for (int k = tid; k < C::QTAB; k += NT) qB[k] = qt->B[k];
  trilinear_metric<double, A>(verts + 24 * (int64_t)e, qt, tid, Gl);
  __syncthreads();
  // centre-metric preconditioner: G_c^{-1} = eps (eps G_c)^{-1} (the same for both fields)
  double Gi[6];
  {
    const double* mm = metric[e].m;
#pragma unroll
    for (int k = 0; k < 6; ++k) Gi[k] = metric[e].eps * mm[12 + k];
  }
  auto precond = [&](const double (&r)[6], double (&z)[6]) {
#pragma unroll
    for (int f = 0; f < 2; ++f)
#pragma unroll
      for (int c = 0; c < 3; ++c)
        z[3 * f + c] = symget(Gi, c, 0) * r[3 * f + 0] + symget(Gi, c, 1) * r[3 * f + 1] + symget(Gi, c, 2) * r[3 * f + 2];
  };
  double tot[2] = {0.0, 0.0};
  for (int i = 0; i < q; ++i) {
    double b[6], x[6], r[6], z[6], p[6], Ap[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      b[c] = pos_lane ? R[I.unk_off + ((int64_t)c * q + i) * A3 + s] : 0.0;
      x[c] = 0.0;
      r[c] = b[c];
    }
    precond(r, z);
#pragma unroll
    for (int c = 0; c < 6; ++c) p[c] = pos_lane ? z[c] : 0.0;
    double rz = 0.0, bb = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      rz += pos_lane ? r[c] * z[c] : 0.0;
      bb += b[c] * b[c];
    }
    block_sum2<NT>(rz, bb, red);
    for (int it = 0; it < 80 && bb > 0.0; ++it) {
      trilinear_mass<double, A>(sm, sm + C::MASS_A, qB, Gl, 1.0, 1.0, p, Ap, tid, pos_lane, s);
      double pAp = 0.0, dummy = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) pAp += pos_lane ? p[c] * Ap[c] : 0.0;
      block_sum2<NT>(pAp, dummy, red);
      const double alpha = pAp > 0.0 ? rz / pAp : 0.0;
      double rr = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        x[c] += alpha * p[c];
        r[c] -= alpha * Ap[c];
        rr += pos_lane ? r[c] * r[c] : 0.0;
      }
      precond(r, z);
      double rz_new = 0.0;
#pragma unroll
      for (int c = 0; c < 6; ++c) rz_new += pos_lane ? r[c] * z[c] : 0.0;
      block_sum2<NT>(rz_new, rr, red);
      if (rr <= 1e-28 * bb) break;  // uniform: every thread has the same sums
      const double beta = rz > 0.0 ? rz_new / rz : 0.0;
      rz = rz_new;
#pragma unroll
      for (int c = 0; c < 6; ++c) p[c] = pos_lane ? z[c] + beta * p[c] : 0.0;
    }
    double eE = 0.0, eH = 0.0;
    if (pos_lane) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        eE += b[c] * x[c];
        eH += b[3 + c] * x[3 + c];
      }
    }
    block_sum2<NT>(eE, eH, red);
    tot[0] += eE;
    tot[1] += eH;
  }
  if (tid == 0) {
    partial[2 * e] = tot[0];
    partial[2 * e + 1] = tot[1];
  }
}

template <int A>
int launch_one(const Mesh* m, const Group& g, const double* R, double* partial, hipStream_t s) {
  using C = KCfg<A>;
  const size_t lds = sizeof(double) * (C::MASS + C::QTAB_PAD + 6 * C::G3 + 2 * (C::NT / 64));
  hipLaunchKernelGGL(dual_norm_trilinear_kernel<A>, dim3((unsigned)g.count), dim3(C::NT), lds, s, m->d_info,
                     m->d_metric, m->d_verts, (const QTables<double>*)m->d_qt64 + A, g.d_list, R, partial);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "dual norm (trilinear) launch");
}

}  // namespace

int launch_dual_norm_trilinear(const Mesh* m, const double* R, double* partial, hipStream_t s) {
  for (const Group& g : m->groups) {
    if (g.affine || g.count == 0) continue;
    int rc;
    switch (g.a) {
      case 2: rc = launch_one<2>(m, g, R, partial, s); break;
      case 3: rc = launch_one<3>(m, g, R, partial, s); break;
      case 4: rc = launch_one<4>(m, g, R, partial, s); break;
      case 5: rc = launch_one<5>(m, g, R, partial, s); break;
      case 6: rc = launch_one<6>(m, g, R, partial, s); break;
      case 7: rc = launch_one<7>(m, g, R, partial, s); break;
      case 8: rc = launch_one<8>(m, g, R, partial, s); break;
      case 9: rc = launch_one<9>(m, g, R, partial, s); break;
      default: return fail(STDG_E_ARG, "dual norm: degree out of range");
    }
    if (rc != STDG_OK) return rc;
  }
  return STDG_OK;
}

}  // namespace stdg
