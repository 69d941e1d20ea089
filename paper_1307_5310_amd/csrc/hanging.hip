// 2:1 hanging faces (Section 5.2 sums the flux terms of a face over the
// neighbours that share parts of it): a coarse face covered by the faces of
// four smaller elements.  The residual kernels take such a face as interior
// with the own half of the centred flux only (1/2 T_self); this kernel adds
// the neighbours' half after them, for every element with a hanging face:
//   R_E[c] += dt eps(c,d,alpha) sigma L_{s_alpha}(side) 1/2 T_nb(H_d)
//   R_H[c] -= dt eps(c,d,alpha) sigma L_{s_alpha}(side) 1/2 T_nb(E_d)
// (d = 3 - c - alpha, sigma = 2 side - 1; the same lift as the residual
// kernels), where T_nb is the neighbours' time-contracted tangential trace
// projected onto this element's face modes, in this element's covariant
// frame, for the test levels i < min(q, q') the coupling keeps.
//
// The projection factors into 1D half-interval integrals
//   S[h][k][m] = int_0^1 L_k(x) L_m((x + h) / 2) dx   (fine mode k, coarse mode m):
// a fine face sees the coarse trace on its half h (own mode k against the
// coarse mode m: S[h][k][m]); a coarse face integrates each fine trace over
// its quarter (own mode m against the fine mode k: S[h][k][m] / 2 per
// direction).  A reversed coordinate multiplies the fine-side mode by
// (-1)^k; covariant components scale by the face map (1/2 from the fine face
// to the coarse one, 2 the other way), so with the quarter's area both sides
// carry the factor 1/2.
#include "internal.h"

namespace stdg {

namespace {

constexpr int kHThreads = 256;

template <typename T>
struct HParams {
  const ElemInfo* info;
  const ElemMetric* metric;
  const HangRec* hang;
  const T* x;
  T* y;
  const T* hs;      // S[h][k][m], 2 kMaxA kMaxA entries
  const int* skip;
  T dt;
  int resid;        // x is the full trial vector (levels m = 0..q)
  int pre;          // P^{-1} fused: the neighbours' values scaled by their inverse metric
  Tables<T> tab;
};

template <typename T>
__device__ inline T legendre_at_side(int l, int side) {
  const T rho = (T)sqrt((double)(2 * l + 1));
  return (side == 0 && (l & 1)) ? -rho : rho;
}

template <typename T>
__global__ void __launch_bounds__(kHThreads) hanging_kernel(HParams<T> P) {
  if (P.skip && *P.skip == 0) return;
  __shared__ T proj[6 * 4 * kMaxA * kMaxA];  // [face][2 fields x 2 slots][own mode]
  const HangRec* R = P.hang + blockIdx.x;
  const int e = R->elem;
  const ElemInfo* Ie = P.info + e;
  const int a = Ie->a, q = Ie->q, a2 = a * a, a3 = a2 * a;
  const int m0 = P.resid ? 0 : 1;
  T* ye = P.y + Ie->unk_off;
  const int tid = threadIdx.x;
  for (int i = 0; i < q; ++i) {
    __syncthreads();  // the previous level's lifts have read proj
    for (int t = tid; t < 24 * a2; t += kHThreads) proj[t] = T(0);
    __syncthreads();
    for (int g = 0; g < 6; ++g) {
      const HangFace& H = R->f[g];
      if (H.kind == 0) continue;  // uniform
      const int alpha = g >> 1;
      const int ua = alpha == 0 ? 1 : 0, va = alpha == 2 ? 1 : 2;
      for (int t = tid; t < 4 * a2; t += kHThreads) {
        const int ft = t / a2, jj = t - ft * a2, fu = jj % a, fv = jj / a;
        const int tf = ft >> 1;             // field of the trace (0 = E, 1 = H)
        const bool slot_u = (ft & 1) == 0;  // own component along u (else along v)
        T acc = T(0);
        const int nn = H.kind == 1 ? 4 : 1;
        for (int j = 0; j < nn; ++j) {
          const int k = H.nb[j];
          const int code = H.code[j];
          const int fo = code & 7, alo = fo >> 1, sdo = fo & 1;
          const int uo = alo == 0 ? 1 : 0, vo = alo == 2 ? 1 : 2;
          const bool swap = (code & 8) != 0, flu = (code & 16) != 0, flv = (code & 32) != 0;
          const int mu_ax = swap ? vo : uo, mv_ax = swap ? uo : vo;  // the neighbour's axes matched with our u, v
          const int cn = slot_u ? mu_ax : mv_ax;
          const ElemInfo* Ik = P.info + k;
          const int ak = Ik->a, qk = Ik->q, ak3 = ak * ak * ak;
          if (i >= qk) continue;  // S_h: no coupling on test levels i >= min(q, q')
          const int nlk = P.resid ? qk + 1 : qk;
          const int str_u = mu_ax == 0 ? 1 : (mu_ax == 1 ? ak : ak * ak);
          const int str_v = mv_ax == 0 ? 1 : (mv_ax == 1 ? ak : ak * ak);
          const int str_n = alo == 0 ? 1 : (alo == 1 ? ak : ak * ak);
          const T sgn = (slot_u ? flu : flv) ? T(-0.5) : T(0.5);
          const T scale = (P.pre ? (T)P.metric[k].m[12 + 6 * tf + cn] : T(1)) * sgn;
          const int hu = H.kind == 2 ? ((code >> 6) & 1) : (j & 1);
          const int hv = H.kind == 2 ? ((code >> 7) & 1) : (j >> 1);
          const T* xk = P.x + (P.resid ? Ik->trial_off : Ik->unk_off) + (int64_t)(3 * tf + cn) * nlk * ak3;
          T sum = T(0);
          for (int m = 0; m < ak; ++m) {
            // weight of the neighbour's mode m along the axis matched with our u
            T wu = H.kind == 2 ? P.hs[(hu * kMaxA + fu) * kMaxA + m] : P.hs[(hu * kMaxA + m) * kMaxA + fu];
            if (flu && ((H.kind == 2 ? fu : m) & 1)) wu = -wu;
            for (int n = 0; n < ak; ++n) {
              T wv = H.kind == 2 ? P.hs[(hv * kMaxA + fv) * kMaxA + n] : P.hs[(hv * kMaxA + n) * kMaxA + fv];
              if (flv && ((H.kind == 2 ? fv : n) & 1)) wv = -wv;
              const T w = wu * wv;
              if (w == T(0)) continue;
              // time contraction of the neighbour's trace at face mode (m, n)
              T tr = T(0);
              for (int mp = m0; mp <= qk; ++mp) {
                const T nim = P.tab.N[i][mp];
                if (nim == T(0)) continue;
                const T* xp = xk + (int64_t)(mp - m0) * ak3 + m * str_u + n * str_v;
                T t = T(0);
                for (int l = 0; l < ak; ++l) t += legendre_at_side<T>(l, sdo) * xp[l * str_n];
                tr += nim * t;
              }
              sum += w * tr;
            }
          }
          acc += scale * sum;
        }
        proj[(g * 4 + ft) * a2 + jj] = acc;
      }
    }
    __syncthreads();
    // lifts: component c of field F takes the faces whose normal is not c
    for (int t = tid; t < 6 * a3; t += kHThreads) {
      const int fc = t / a3, s = t - fc * a3;
      const int f = fc / 3, c = fc - 3 * f;
      const int s0 = s % a, s1 = (s / a) % a, s2 = s / a2;
      T v = T(0);
      for (int alpha = 0; alpha < 3; ++alpha) {
        if (alpha == c) continue;
        const int d = 3 - c - alpha;
        const int ua = alpha == 0 ? 1 : 0;
        const int slot = d == ua ? 0 : 1;
        const T epsv = alpha == (c + 2) % 3 ? T(1) : T(-1);  // eps(c, d, alpha)
        const int jj = alpha == 0 ? s1 + a * s2 : (alpha == 1 ? s0 + a * s2 : s0 + a * s1);
        const int l = alpha == 0 ? s0 : (alpha == 1 ? s1 : s2);
        // E rows lift the H traces, H rows the E traces (with the opposite sign)
        const int ft = (f == 0 ? 2 : 0) + slot;
        for (int side = 0; side < 2; ++side) {
          const int g = 2 * alpha + side;
          if (R->f[g].kind == 0) continue;
          const T sl = side ? legendre_at_side<T>(l, 1) : -legendre_at_side<T>(l, 0);  // sigma L_l(side)
          v += (f == 0 ? epsv : -epsv) * sl * T(0.5) * proj[(g * 4 + ft) * a2 + jj];
        }
      }
      if (v != T(0)) ye[((int64_t)fc * q + i) * a3 + s] += P.dt * v;
    }
  }
}

}  // namespace

template <typename T>
int launch_hanging(const Mesh* m, double dt, int mode, const T* x, T* y, hipStream_t s, const int* skip) {
  if (m->hang.empty()) return STDG_OK;
  if (!m->d_hang) return fail(STDG_E_ARG, "hanging faces: device records missing");
  HParams<T> P;
  P.info = m->d_info;
  P.metric = m->d_metric;
  P.hang = m->d_hang;
  P.x = x;
  P.y = y;
  P.hs = (const T*)(sizeof(T) == 8 ? m->d_hs64 : m->d_hs32);
  P.skip = skip;
  P.dt = (T)dt;
  P.resid = mode == STDG_RESIDUAL ? 1 : 0;
  P.pre = mode == STDG_OPERATOR_PRECOND ? 1 : 0;
  if constexpr (sizeof(T) == 8) fill_tables_f64(&P.tab); else fill_tables_f32(&P.tab);
  hipLaunchKernelGGL(hanging_kernel<T>, dim3((unsigned)m->hang.size()), dim3(kHThreads), 0, s, P);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "hanging-face kernel");
}

template int launch_hanging<float>(const Mesh*, double, int, const float*, float*, hipStream_t, const int*);
template int launch_hanging<double>(const Mesh*, double, int, const double*, double*, hipStream_t, const int*);

}  // namespace stdg
