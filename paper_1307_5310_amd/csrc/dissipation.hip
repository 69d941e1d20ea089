// Dissipative stabilisation D_h (the remark closing Section 4) on trilinear
// elements.  On an affine element the face metric is constant and the
// residual kernels fold D_h into their face pass; on a trilinear element
// the metric varies over a face, so this kernel adds the D_h terms to the
// residual after the element's residual kernel has written it (same stream).
//
// For element K, test level i, face (alpha, side) and field F in {E, H}:
//   R_F[c](phi_s) += dt alpha_F sum_k w_k K_cd(x_k) J_d(x_k) phi_s(x_k)
// over the n x n Gauss points x_k of the face (n = max(a, a') + 2), where
//   J_d = T_self(sum_m N[i][m] U_m)_d - T_nb(sum_m N[i][m] U'_m)_d
// is the tangential jump of the time-contracted covariant components (the
// neighbour's components carried into K's frame by the signed permutation of
// the face map; T_self alone on PEC faces, where only E is stabilised;
// nothing on interior faces for i >= min(q, q'), where the projected test
// function vanishes), and K = |t_u x t_v| G^{-1} is the face metric of the
// tangent vectors t_u, t_v of the trilinear map at x_k, which turns the
// physical (n x v) . (n x u) dS into sum K_cd v_c u_d du dv.
//
// One workgroup per element: the contracted level in LDS, then face by face
// the two traces (face modes by the L_l(side) sums, point values by two 1D
// sum-factorised sweeps), the weighted jump at the points and its projection
// back onto the face modes; finally every position adds the lifts of the
// four faces tangential to each component, L_{s_alpha}(side) times the face
// mode, to its outputs.
#include "internal.h"

namespace stdg {

namespace {

constexpr int kDThreads = 256;
constexpr int kA2 = kMaxA * kMaxA;

template <typename T>
struct DParams {
  const ElemInfo* info;
  const double* verts;          // [ne][8][3]
  const int32_t* list;
  const T* x;
  T* y;
  const T* diss;                // per element: alpha_E[6], alpha_H[6], ...
  const FaceRule<T>* fr;        // indexed by n
  const FaceRule<double>* fr64; // point coordinates for the geometry
  const int* skip;
  T dt;
  int resid;                    // 1: x is the full trial vector (levels m = 0..q)
  Tables<T> tab;
};

// d F / d xhat_d at xhat = (x0, x1, x2) of the trilinear map with corners
// X[c] (corner c = b0 + 2 b1 + 4 b2 sits at xhat = (b0, b1, b2))
__device__ inline void tangent(const double* X, double x0, double x1, double x2, int d, double t[3]) {
  t[0] = t[1] = t[2] = 0.0;
  for (int c = 0; c < 8; ++c) {
    const double f0 = d == 0 ? ((c & 1) ? 1.0 : -1.0) : ((c & 1) ? x0 : 1.0 - x0);
    const double f1 = d == 1 ? ((c & 2) ? 1.0 : -1.0) : ((c & 2) ? x1 : 1.0 - x1);
    const double f2 = d == 2 ? ((c & 4) ? 1.0 : -1.0) : ((c & 4) ? x2 : 1.0 - x2);
    const double f = f0 * f1 * f2;
    t[0] += f * X[3 * c + 0];
    t[1] += f * X[3 * c + 1];
    t[2] += f * X[3 * c + 2];
  }
}

// stride of reference axis d in the position index s = s0 + a (s1 + a s2)
__device__ inline int axis_stride(int d, int a) { return d == 0 ? 1 : (d == 1 ? a : a * a); }

template <typename T>
__global__ void __launch_bounds__(kDThreads) diss_trilinear_kernel(DParams<T> P) {
  if (P.skip && *P.skip == 0) return;
  extern __shared__ __align__(16) unsigned char dsm_raw[];
  T* sm = reinterpret_cast<T*>(dsm_raw);
  __shared__ double vx[24];
  const int tid = threadIdx.x;
  const int e = P.list[blockIdx.x];
  const ElemInfo* Ie = P.info + e;  // (read in place: a private copy indexed by face would go to scratch)
  const int a = Ie->a, q = Ie->q, a2 = a * a, a3 = a2 * a;
  const int m0 = P.resid ? 0 : 1, nl = P.resid ? q + 1 : q;
  const T* xe = P.x + (P.resid ? Ie->trial_off : Ie->unk_off);
  T* ye = P.y + Ie->unk_off;
  if (tid < 24) vx[tid] = P.verts[(int64_t)24 * e + tid];
  T* Xs = sm;                              // [6 components][a^3] contracted level
  T* proj = Xs + 6 * a3;                   // [6 faces][2 fields x 2 slots][a^2]
  T* two = proj + 24 * a2;                 // [4][kMaxFaceQ * kMaxA] sweep buffers
  T* twn = two + 4 * kMaxFaceQ * kMaxA;
  // the face modes are dead once the first sweep has read them: the point
  // values take their place (keeps a = 9 in FP64 within 64 KB)
  T* co = twn + 4 * kMaxFaceQ * kMaxA;     // [4][kA2] own face modes
  T* cn = co + 4 * kA2;                    // [4][kA2] neighbour face modes
  T* Vo = co;                              // [4][kMaxFaceQ^2] own values, then weighted jumps
  T* Vn = Vo + 4 * kMaxFaceQ * kMaxFaceQ;  // [4][kMaxFaceQ^2] neighbour values
  const T* al = P.diss + (int64_t)Mesh::kDissWords * e;

  for (int i = 0; i < q; ++i) {
    __syncthreads();  // the previous level's lifts have read Xs and proj
    for (int t = tid; t < 6 * a3; t += kDThreads) {
      const int fc = t / a3, s = t - fc * a3;
      T v = T(0);
      for (int m = m0; m <= q; ++m) v += P.tab.N[i][m] * xe[((int64_t)fc * nl + (m - m0)) * a3 + s];
      Xs[t] = v;
    }
    for (int t = tid; t < 24 * a2; t += kDThreads) proj[t] = T(0);
    __syncthreads();

    for (int g = 0; g < 6; ++g) {
      const int k = Ie->nb[g];
      int ak = a, qk = q;
      int64_t koff = 0;
      int orient = 0;
      if (k >= 0) {
        const ElemInfo* Ik = P.info + k;
        ak = Ik->a;
        qk = Ik->q;
        koff = P.resid ? Ik->trial_off : Ik->unk_off;
        orient = Ie->orient[g];
        if (i >= (q < qk ? q : qk)) continue;  // uniform over the workgroup
      }
      const int nf = (k >= 0 && ak > a ? ak : a) + 2;
      const FaceRule<T>& R = P.fr[nf];
      const int alpha = g >> 1, side = g & 1;
      const int ua = alpha == 0 ? 1 : 0, va = alpha == 2 ? 1 : 2;  // tangential axes, increasing
      // own face modes co[2 F + slot][ju + a jv], slot 0 along ua, 1 along va
      for (int t = tid; t < 4 * a2; t += kDThreads) {
        const int ft = t / a2, jj = t - ft * a2, ju = jj % a, jv = jj / a;
        const int comp = 3 * (ft >> 1) + ((ft & 1) ? va : ua);
        const T* src = Xs + comp * a3 + ju * axis_stride(ua, a) + jv * axis_stride(va, a);
        const int ns = axis_stride(alpha, a);
        T v = T(0);
        for (int l = 0; l < a; ++l) v += (side ? P.tab.tr1[l] : P.tab.tr0[l]) * src[l * ns];
        co[ft * kA2 + jj] = v;
      }
      // neighbour face modes on its own face f' (its axes u' < v'), contracted in time
      const int fo = orient & 7, alo = fo >> 1, sdo = fo & 1;
      const int uo = alo == 0 ? 1 : 0, vo = alo == 2 ? 1 : 2;
      if (k >= 0) {
        const int ak2 = ak * ak, ak3 = ak2 * ak, nlk = P.resid ? qk + 1 : qk;
        const T* xk = P.x + koff;
        for (int t = tid; t < 4 * ak2; t += kDThreads) {
          const int ft = t / ak2, jj = t - ft * ak2, ju = jj % ak, jv = jj / ak;
          const int comp = 3 * (ft >> 1) + ((ft & 1) ? vo : uo);
          const int base = ju * axis_stride(uo, ak) + jv * axis_stride(vo, ak), ns = axis_stride(alo, ak);
          T v = T(0);
          for (int l = 0; l < ak; ++l) {
            const int64_t pos = base + l * ns;
            T tl = T(0);
            for (int m = m0; m <= qk; ++m) tl += P.tab.N[i][m] * xk[((int64_t)comp * nlk + (m - m0)) * ak3 + pos];
            v += (sdo ? P.tab.tr1[l] : P.tab.tr0[l]) * tl;
          }
          cn[ft * kA2 + jj] = v;
        }
      }
      __syncthreads();
      // point values, first sweep: tw[ft][ku + nf jv] = sum_ju c[ju + a jv] L_ju(x_ku)
      for (int t = tid; t < 4 * nf * a; t += kDThreads) {
        const int ft = t / (nf * a), r = t - ft * nf * a, ku = r % nf, jv = r / nf;
        T v = T(0);
        for (int ju = 0; ju < a; ++ju) v += co[ft * kA2 + ju + a * jv] * R.L[ku * kMaxA + ju];
        two[ft * kMaxFaceQ * kMaxA + ku + nf * jv] = v;
      }
      if (k >= 0) {
        for (int t = tid; t < 4 * nf * ak; t += kDThreads) {
          const int ft = t / (nf * ak), r = t - ft * nf * ak, ku = r % nf, jv = r / nf;
          T v = T(0);
          for (int ju = 0; ju < ak; ++ju) v += cn[ft * kA2 + ju + ak * jv] * R.L[ku * kMaxA + ju];
          twn[ft * kMaxFaceQ * kMaxA + ku + nf * jv] = v;
        }
      }
      __syncthreads();
      // second sweep: V[ft][ku + nf kv] = sum_jv tw[ft][ku + nf jv] L_jv(x_kv)
      for (int t = tid; t < 4 * nf * nf; t += kDThreads) {
        const int ft = t / (nf * nf), r = t - ft * nf * nf, ku = r % nf, kv = r / nf;
        T v = T(0);
        for (int jv = 0; jv < a; ++jv) v += two[ft * kMaxFaceQ * kMaxA + ku + nf * jv] * R.L[kv * kMaxA + jv];
        Vo[ft * kMaxFaceQ * kMaxFaceQ + r] = v;
        if (k >= 0) {
          T w = T(0);
          for (int jv = 0; jv < ak; ++jv) w += twn[ft * kMaxFaceQ * kMaxA + ku + nf * jv] * R.L[kv * kMaxA + jv];
          Vn[ft * kMaxFaceQ * kMaxFaceQ + r] = w;
        }
      }
      __syncthreads();
      // weighted jumps at the points, in place of the own values
      const bool swap = (orient & kOrientSwap) != 0;
      const bool flu = (orient & kOrientFlipU) != 0, flv = (orient & kOrientFlipV) != 0;
      for (int r = tid; r < nf * nf; r += kDThreads) {
        const int ku = r % nf, kv = r / nf;
        const double xu = P.fr64[nf].x[ku], xv = P.fr64[nf].x[kv], xs = (double)side;
        // reference point: the normal axis at the side, u and v along the increasing tangential axes
        const double x0 = alpha == 0 ? xs : xu;
        const double x1 = alpha == 1 ? xs : (alpha == 0 ? xu : xv);
        const double x2 = alpha == 2 ? xs : xv;
        double tu[3], tv[3];
        tangent(vx, x0, x1, x2, ua, tu);
        tangent(vx, x0, x1, x2, va, tv);
        const double uu = tu[0] * tu[0] + tu[1] * tu[1] + tu[2] * tu[2];
        const double vv = tv[0] * tv[0] + tv[1] * tv[1] + tv[2] * tv[2];
        const double uv = tu[0] * tv[0] + tu[1] * tv[1] + tu[2] * tv[2];
        const double cx = tu[1] * tv[2] - tu[2] * tv[1], cy = tu[2] * tv[0] - tu[0] * tv[2],
                     cz = tu[0] * tv[1] - tu[1] * tv[0];
        const double inv_area = 1.0 / sqrt(cx * cx + cy * cy + cz * cz);
        const T Kuu = (T)(vv * inv_area), Kvv = (T)(uu * inv_area), Kuv = (T)(-uv * inv_area);
        // the neighbour point matched with (ku, kv) and its slots along our u and v
        const int wu = flu ? nf - 1 - ku : ku, wv = flv ? nf - 1 - kv : kv;
        const int rn = swap ? (wv + nf * wu) : (wu + nf * wv);
        const int su_slot = swap ? 1 : 0, sv_slot = swap ? 0 : 1;
        const T su = flu ? T(-1) : T(1), sv = flv ? T(-1) : T(1);
        const T wgt = R.w[ku] * R.w[kv];
        for (int f = 0; f < 2; ++f) {
          T ju = Vo[(2 * f) * kMaxFaceQ * kMaxFaceQ + r];
          T jv = Vo[(2 * f + 1) * kMaxFaceQ * kMaxFaceQ + r];
          if (k >= 0) {
            ju -= su * Vn[(2 * f + su_slot) * kMaxFaceQ * kMaxFaceQ + rn];
            jv -= sv * Vn[(2 * f + sv_slot) * kMaxFaceQ * kMaxFaceQ + rn];
          }
          const T c = al[6 * f + g] * wgt;  // alpha_H is 0 on PEC faces
          Vo[(2 * f) * kMaxFaceQ * kMaxFaceQ + r] = c * (Kuu * ju + Kuv * jv);
          Vo[(2 * f + 1) * kMaxFaceQ * kMaxFaceQ + r] = c * (Kuv * ju + Kvv * jv);
        }
      }
      __syncthreads();
      // projection onto the face modes: tw[ft][ju + a kv] = sum_ku P[ku + nf kv] L_ju(x_ku)
      for (int t = tid; t < 4 * a * nf; t += kDThreads) {
        const int ft = t / (a * nf), r = t - ft * a * nf, ju = r % a, kv = r / a;
        T v = T(0);
        for (int ku = 0; ku < nf; ++ku) v += Vo[ft * kMaxFaceQ * kMaxFaceQ + ku + nf * kv] * R.L[ku * kMaxA + ju];
        two[ft * kMaxFaceQ * kMaxA + ju + a * kv] = v;
      }
      __syncthreads();
      for (int t = tid; t < 4 * a2; t += kDThreads) {
        const int ft = t / a2, jj = t - ft * a2, ju = jj % a, jv = jj / a;
        T v = T(0);
        for (int kv = 0; kv < nf; ++kv) v += two[ft * kMaxFaceQ * kMaxA + ju + a * kv] * R.L[kv * kMaxA + jv];
        proj[(g * 4 + ft) * a2 + jj] = v;
      }
      __syncthreads();  // the sweep buffers are reused by the next face
    }

    // lifts: component c of field F at position s takes the four faces whose
    // normal is not c, L_{s_alpha}(side) times the face mode (s_u, s_v)
    for (int t = tid; t < 6 * a3; t += kDThreads) {
      const int fc = t / a3, s = t - fc * a3;
      const int f = fc / 3, c = fc - 3 * f;
      const int s0 = s % a, s1 = (s / a) % a, s2 = s / a2;
      T v = T(0);
      for (int alpha = 0; alpha < 3; ++alpha) {
        if (alpha == c) continue;
        const int ua = alpha == 0 ? 1 : 0;
        const int slot = c == ua ? 0 : 1;
        // face mode (s_u, s_v) over the increasing tangential axes, level s_alpha
        const int jj = alpha == 0 ? s1 + a * s2 : (alpha == 1 ? s0 + a * s2 : s0 + a * s1);
        const int l = alpha == 0 ? s0 : (alpha == 1 ? s1 : s2);
        v += P.tab.tr0[l] * proj[((2 * alpha) * 4 + 2 * f + slot) * a2 + jj] +
             P.tab.tr1[l] * proj[((2 * alpha + 1) * 4 + 2 * f + slot) * a2 + jj];
      }
      T* yp = ye + ((int64_t)fc * q + i) * a3 + s;
      *yp += P.dt * v;
    }
  }
}

constexpr int kDUnion = 8 * kMaxFaceQ * kMaxFaceQ > 8 * kA2 ? 8 * kMaxFaceQ * kMaxFaceQ : 8 * kA2;

template <typename T>
size_t diss_shmem(int a) {
  return sizeof(T) * (size_t)(6 * a * a * a + 24 * a * a + 8 * kMaxFaceQ * kMaxA + kDUnion);
}
static_assert(sizeof(double) * (6 * kMaxA * kMaxA * kMaxA + 24 * kMaxA * kMaxA + 8 * kMaxFaceQ * kMaxA + kDUnion) +
                      sizeof(double) * 24 <= 65536,
              "D_h kernel LDS must stay within 64 KB");

}  // namespace

template <typename T>
int launch_diss_trilinear(const Mesh* m, const Group& g, double dt, int mode, const T* x, T* y, hipStream_t s,
                          const int* skip) {
  if (g.count == 0) return STDG_OK;
  if (!m->d_fr64 || !m->d_fr32) return fail(STDG_E_ARG, "D_h on trilinear elements: face rules missing");
  DParams<T> P;
  P.info = m->d_info;
  P.verts = m->d_verts;
  P.list = g.d_list;
  P.x = x;
  P.y = y;
  if constexpr (sizeof(T) == 8) {
    P.diss = m->d_diss;
    P.fr = (const FaceRule<T>*)m->d_fr64;
  } else {
    P.diss = m->d_diss32;
    P.fr = (const FaceRule<T>*)m->d_fr32;
  }
  P.fr64 = (const FaceRule<double>*)m->d_fr64;
  P.skip = skip;
  P.dt = (T)dt;
  P.resid = mode == STDG_RESIDUAL ? 1 : 0;
  if constexpr (sizeof(T) == 8) fill_tables_f64(&P.tab); else fill_tables_f32(&P.tab);
  const size_t shmem = diss_shmem<T>(g.a);
  hipLaunchKernelGGL(diss_trilinear_kernel<T>, dim3((unsigned)g.count), dim3(kDThreads), shmem, s, P);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "D_h kernel (trilinear elements)");
}

template int launch_diss_trilinear<float>(const Mesh*, const Group&, double, int, const float*, float*, hipStream_t,
                                          const int*);
template int launch_diss_trilinear<double>(const Mesh*, const Group&, double, int, const double*, double*,
                                           hipStream_t, const int*);

}  // namespace stdg
