// The matrix-free space-time residual of one slab (Section 5, eq. residual;
// evaluation strategy of Section 5.2), one workgroup per element.
//
// Per element K with a = p + 1, test levels i = 0..q-1 and trial levels m:
//   R_E[c,i,s] = sum_d Meps[c][d] (x^E_{i+1} - delta_{i0} x^E_0)[d,s]
//              + dt * ( curl term from H~_i + lift of the centred H flux )
//   R_H[c,i,s] = the same with Mmu, the curl of E~_i and the E flux
// where E~_i = sum_m N[i][m] x_m is the time-contracted trial field
// (N[i][m] = int L_i l_m, at most 3 nonzeros per row), the mass factor
// int L_i l_m' is the shift delta_{m,i+1} - delta_{i0} delta_{m0}, and for
// covariant maps curl and flux are geometry-free in reference coordinates.
//
// Curl (from (curl E, w) and -(H, curl v), eq. bilinearform:C), with
// Dh[n][j] = int L_n L_j' = 2 sqrt(2n+1) sqrt(2j+1) for n < j, j - n odd:
//   R_H[c] += sum_n Dh[s_c1][n] E_c2(s_c1 -> n) - sum_n Dh[s_c2][n] E_c1(s_c2 -> n)
//   R_E[c] += sum_n Dh[n][s_c1] H_c2(s_c1 -> n) - sum_n Dh[n][s_c2] H_c1(s_c2 -> n)
// (c1, c2) = (c+1, c+2) mod 3; "s_m -> n" replaces the index along axis m.
//
// Faces (centred fluxes, S_h of eq. bilinearform:S with one temporal element):
// on face (alpha, side) with outward normal sigma e_alpha, sigma = 2 side - 1,
// the tangential traces T = sum_l L_l(side) x(.., l_alpha = l, ..) give
//   F = 1/2 T_self(H) + 1/2 T_nb(H),  G = -1/2 T_self(E) + 1/2 T_nb(E)  (interior)
//   F = T_self(H),                    G = -T_self(E)                    (PEC boundary)
// with the neighbour term present only for test levels i < min(q_K, q_K')
// (S_h restricts the coupling to the common temporal test space), and lifts
//   R_E[c] += sigma eps(c,d,alpha) L_{s_alpha}(side) F_d
//   R_H[c] -= sigma eps(c,d,alpha) L_{s_alpha}(side) G_d,  d = 3 - c - alpha.
// Faces with different p couple only the tangential modes < min(a, a').
//
// Thread layout: NT lanes per element; lane owns positions s = tid + NT r
// (all 6 components, all levels, in registers) and face items
// (face, tangential component, tangential mode) it = tid + NT k.  The
// neighbour traces are reduced straight from global memory (the neighbour
// blocks are read through L2, which the locality-ordered work list and the
// XCD-aware block mapping keep warm); per test level the contracted field and
// the face fluxes are staged in LDS.
#pragma once

#include "internal.h"

namespace stdg {

template <int A>
struct KCfg {
  static constexpr int A2 = A * A, A3 = A * A * A;
  static constexpr int NT = A <= 5 ? 64 : (A <= 7 ? 128 : (A == 8 ? 256 : 512));
  static constexpr int R = (A3 + NT - 1) / NT;
  static constexpr int NI = 24 * A2;
  static constexpr int IPL = (NI + NT - 1) / NT;
  static constexpr int LDS_ELEMS = 6 * A3 + 24 * A2 + 3 * kMaxA;
};

template <typename T>
struct KParams {
  const ElemInfo* info;
  const ElemMetric* metric;
  const int32_t* list;
  const T* x;
  const T* load;
  T* y;
  T dt;
  int mode;  // 0 operator, 1 residual, 2 operator with P^{-1} (diagonal metrics)
  Tables<T> tab;
};

__host__ __device__ constexpr bool nnzN(int i, int m) {
  return (i == 0 && m <= 2) || (i == 1 && (m == 0 || m == 1 || m == 3)) || (i >= 2 && (m == i || m == i + 2));
}

template <typename T>
__device__ __forceinline__ T symget(const T* M, int c, int d) {
  return c == d ? M[c] : ((c + d == 1) ? M[3] : ((c + d == 2) ? M[4] : M[5]));
}

template <typename T, int A, int Q>
__global__ void __launch_bounds__(KCfg<A>::NT) residual_affine_kernel(KParams<T> P) {
  using C = KCfg<A>;
  constexpr int A2 = C::A2, A3 = C::A3, NT = C::NT, R = C::R, NI = C::NI, IPL = C::IPL;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* Et = reinterpret_cast<T*>(smem_raw);  // [6][A3] contracted level
  T* Fl = Et + 6 * A3;                     // [6 faces][4][A2] fluxes
  T* s_rho = Fl + 24 * A2;                 // sqrt(2j+1)
  T* s_t0 = s_rho + kMaxA;                 // L_j(0)
  T* s_t1 = s_t0 + kMaxA;                  // L_j(1)

  const int tid = threadIdx.x;
  // XCD-aware block order: consecutive work-list entries run on the same XCD
  const uint32_t nblk = gridDim.x, b = blockIdx.x;
  const uint32_t xcd = b & 7u, idx = b >> 3;
  const uint32_t qq = nblk >> 3, rr = nblk & 7u;
  const uint32_t logical = xcd * qq + (xcd < rr ? xcd : rr) + idx;
  const int e = P.list[logical];
  const ElemInfo* Ip = P.info + e;
  const int mode = P.mode;
  const bool resid = mode == 1, pre = mode == 2;
  const int m0 = resid ? 0 : 1;
  const int64_t xoff = resid ? Ip->trial_off : Ip->unk_off;
  const int64_t yoff = Ip->unk_off;
  const int nlev = resid ? Q + 1 : Q;

#pragma unroll
  for (int j = 0; j < kMaxA; ++j)
    if (tid == j) {
      s_rho[j] = P.tab.tr1[j];
      s_t0[j] = P.tab.tr0[j];
      s_t1[j] = P.tab.tr1[j];
    }

  // own block into registers
  const T* xe = P.x + xoff;
  T xr[6][Q + 1][R];
#pragma unroll
  for (int fc = 0; fc < 6; ++fc)
#pragma unroll
    for (int m = 0; m <= Q; ++m)
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int s = tid + NT * r;
        T v = T(0);
        if ((R * NT == A3 || s < A3) && m >= m0) v = xe[(int64_t)(fc * nlev + m - m0) * A3 + s];
        xr[fc][m][r] = v;
      }

  // metric of K (uniform loads)
  T Me[6], Mh[6], Ie[6], Ih[6];
  {
    const double* mm = P.metric[e].m;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      Me[k] = (T)mm[k];
      Mh[k] = (T)mm[6 + k];
      Ie[k] = (T)mm[12 + k];
      Ih[k] = (T)mm[18 + k];
    }
  }
  __syncthreads();

  // neighbour table, uniform per block (scalar loads): id, degrees, offset, P^{-1} diagonal
  int nb_id[6], nb_a[6], nb_q[6];
  int64_t nb_off[6];
  T nb_sc[6][6];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    nb_id[f] = Ip->nb[f];
    nb_a[f] = A;
    nb_q[f] = Q;
    nb_off[f] = 0;
#pragma unroll
    for (int k = 0; k < 6; ++k) nb_sc[f][k] = T(1);
    if (nb_id[f] >= 0) {
      const ElemInfo* Np = P.info + nb_id[f];
      nb_a[f] = Np->a;
      nb_q[f] = Np->q;
      nb_off[f] = resid ? Np->trial_off : Np->unk_off;
      if (pre) {
        const double* mm = P.metric[nb_id[f]].m;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          nb_sc[f][k] = (T)mm[12 + k];
          nb_sc[f][3 + k] = (T)mm[18 + k];
        }
      }
    }
  }

  // neighbour traces, contracted in time: acc[k][i]
  T acc[IPL][Q];
  int nbk[IPL];
#pragma unroll
  for (int k = 0; k < IPL; ++k) {
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[k][i] = T(0);
    nbk[k] = -1;
    const int it = tid + NT * k;
    if (NI % NT != 0 && it >= NI) continue;
    const int phi = it / (4 * A2);
    const int rem = it - phi * (4 * A2);
    const int tc = rem / A2;
    const int t = rem - tc * A2;
    const int alpha = phi >> 1, side = phi & 1;
    const int f = tc >> 1;
    const int c = (alpha + 1 + (tc & 1)) % 3;
    // select this item's face from the uniform table
    int nbe = -1, na = A, nq = Q;
    int64_t noff = 0;
    T scale = T(1);
#pragma unroll
    for (int g = 0; g < 6; ++g)
      if (phi == g) {
        nbe = nb_id[g];
        na = nb_a[g];
        nq = nb_q[g];
        noff = nb_off[g];
#pragma unroll
        for (int kk = 0; kk < 6; ++kk)
          if (3 * f + c == kk) scale = nb_sc[g][kk];
      }
    nbk[k] = nbe;
    if (nbe < 0) continue;
    const int u = t % A, v = t / A;
    if (u >= na || v >= na) continue;
    const int na2 = na * na, na3 = na2 * na;
    int tb, ns;
    if (alpha == 0) { tb = na * u + na2 * v; ns = 1; }
    else if (alpha == 1) { tb = u + na2 * v; ns = na; }
    else { tb = u + na * v; ns = na2; }
    const int nnlev = resid ? nq + 1 : nq;
    const T* xb = P.x + noff + (int64_t)(3 * f + c) * nnlev * na3 + tb;
    const T* tau = side ? s_t0 : s_t1;  // neighbour's face sits at 1 - side
    if (na == A && nq == Q) {
      // same degrees (the common case): compile-time trip counts, so every load
      // of the item is in flight before the reductions start
      T vals[Q + 1][A];
#pragma unroll
      for (int mp = 0; mp <= Q; ++mp)
#pragma unroll
        for (int l = 0; l < A; ++l)
          vals[mp][l] = (mp >= m0) ? xb[(int64_t)(mp - m0) * A3 + l * ns] : T(0);
#pragma unroll
      for (int mp = 0; mp <= Q; ++mp) {
        T tr = T(0);
#pragma unroll
        for (int l = 0; l < A; ++l) tr += tau[l] * vals[mp][l];
        tr *= scale;
#pragma unroll
        for (int i = 0; i < Q; ++i)
          if (nnzN(i, mp)) acc[k][i] += P.tab.N[i][mp] * tr;
      }
      continue;
    }
#pragma unroll
    for (int mp = 0; mp <= kMaxQ; ++mp) {
      if (mp < m0 || mp > nq) continue;
      const T* xl = xb + (int64_t)(mp - m0) * na3;
      T tr = T(0);
      for (int l = 0; l < na; ++l) tr += tau[l] * xl[l * ns];
      tr *= scale;
#pragma unroll
      for (int i = 0; i < Q; ++i)
        if (nnzN(i, mp) && i < nq) acc[k][i] += P.tab.N[i][mp] * tr;
    }
  }

  const T dt = P.dt;
  const T* ld = (resid && P.load) ? P.load + yoff : nullptr;
  T* ye = P.y + yoff;

#pragma unroll
  for (int i = 0; i < Q; ++i) {
    // (a) contracted level E~_i, H~_i into LDS
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = tid + NT * r;
      if (!(R * NT == A3 || s < A3)) continue;
      T et[6];
#pragma unroll
      for (int fc = 0; fc < 6; ++fc) {
        T v = T(0);
#pragma unroll
        for (int m = 0; m <= Q; ++m)
          if (nnzN(i, m)) v += P.tab.N[i][m] * xr[fc][m][r];
        et[fc] = v;
      }
      if (pre) {
        T z[6];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          z[c] = symget(Ie, c, 0) * et[0] + symget(Ie, c, 1) * et[1] + symget(Ie, c, 2) * et[2];
          z[3 + c] = symget(Ih, c, 0) * et[3] + symget(Ih, c, 1) * et[4] + symget(Ih, c, 2) * et[5];
        }
#pragma unroll
        for (int fc = 0; fc < 6; ++fc) et[fc] = z[fc];
      }
#pragma unroll
      for (int fc = 0; fc < 6; ++fc) Et[fc * A3 + s] = et[fc];
    }
    __syncthreads();

    // (b) face fluxes into LDS
#pragma unroll
    for (int k = 0; k < IPL; ++k) {
      const int it = tid + NT * k;
      if (NI % NT != 0 && it >= NI) continue;
      const int phi = it / (4 * A2);
      const int rem = it - phi * (4 * A2);
      const int tc = rem / A2;
      const int t = rem - tc * A2;
      const int alpha = phi >> 1, side = phi & 1;
      const int f = tc >> 1;
      const int c = (alpha + 1 + (tc & 1)) % 3;
      int tb, ns;
      if (alpha == 0) { tb = A * t; ns = 1; }
      else if (alpha == 1) { tb = (t % A) + A2 * (t / A); ns = A; }
      else { tb = t; ns = A2; }
      const T* tau = side ? s_t1 : s_t0;
      const T* src = Et + (3 * f + c) * A3 + tb;
      T ts = T(0);
#pragma unroll
      for (int l = 0; l < A; ++l) ts += tau[l] * src[l * ns];
      T val;
      if (nbk[k] >= 0) val = (f == 0 ? T(-0.5) : T(0.5)) * ts + T(0.5) * acc[k][i];
      else val = (f == 0 ? T(-1) : T(1)) * ts;
      Fl[it] = val;
    }
    __syncthreads();

    // (c) outputs: mass + dt (curl + lift) - load
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int s = tid + NT * r;
      if (!(R * NT == A3 || s < A3)) continue;
      const int sj = s % A, sk = (s / A) % A, sl = s / A2;
      const int sidx[3] = {sj, sk, sl};
      const int tgt[3] = {sk + A * sl, sj + A * sl, sj + A * sk};  // tangential index per normal axis
      const T rho_s[3] = {s_rho[sj], s_rho[sk], s_rho[sl]};
      const T tr0s[3] = {s_t0[sj], s_t0[sk], s_t0[sl]};
      const T tr1s[3] = {s_t1[sj], s_t1[sk], s_t1[sl]};
#pragma unroll
      for (int f = 0; f < 2; ++f) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
          constexpr int stride[3] = {1, A, A2};
          T cu = T(0);
          if (f == 0) {
            // + sum_{n < s_c1} Dh[n][s_c1] H_c2(s_c1 -> n) - sum_{n < s_c2} Dh[n][s_c2] H_c1(s_c2 -> n)
            const T* H2 = Et + (3 + c2) * A3;
            const T* H1 = Et + (3 + c1) * A3;
            T p1 = T(0), p2 = T(0);
#pragma unroll
            for (int d = 1; d < A; d += 2) {
              const int n1 = sidx[c1] - d;
              if (n1 >= 0) p1 += s_rho[n1] * H2[s - d * stride[c1]];
              const int n2 = sidx[c2] - d;
              if (n2 >= 0) p2 += s_rho[n2] * H1[s - d * stride[c2]];
            }
            cu = T(2) * (rho_s[c1] * p1 - rho_s[c2] * p2);
          } else {
            // + sum_{n > s_c1} Dh[s_c1][n] E_c2(s_c1 -> n) - sum_{n > s_c2} Dh[s_c2][n] E_c1(s_c2 -> n)
            const T* E2 = Et + c2 * A3;
            const T* E1 = Et + c1 * A3;
            T p1 = T(0), p2 = T(0);
#pragma unroll
            for (int d = 1; d < A; d += 2) {
              const int n1 = sidx[c1] + d;
              if (n1 < A) p1 += s_rho[n1] * E2[s + d * stride[c1]];
              const int n2 = sidx[c2] + d;
              if (n2 < A) p2 += s_rho[n2] * E1[s + d * stride[c2]];
            }
            cu = T(2) * (rho_s[c1] * p1 - rho_s[c2] * p2);
          }
          // lifts from the four faces whose normal is not c
          T lift = T(0);
#pragma unroll
          for (int w = 0; w < 2; ++w) {
            const int alpha = w == 0 ? c1 : c2;
            const int dcomp = w == 0 ? c2 : c1;
            const T epsv = (alpha == c2) ? T(1) : T(-1);  // eps(c, d, alpha)
            const int tcd = (dcomp == (alpha + 1) % 3 ? 0 : 1) + (f == 0 ? 2 : 0);
            const int t = tgt[alpha];
            const T v0 = Fl[((2 * alpha + 0) * 4 + tcd) * A2 + t];
            const T v1 = Fl[((2 * alpha + 1) * 4 + tcd) * A2 + t];
            // sigma = -1 on side 0, +1 on side 1
            const T l = tr1s[alpha] * v1 - tr0s[alpha] * v0;
            lift += (f == 0 ? epsv : -epsv) * l;
          }
          // mass: the time-derivative factor is the shift delta_{m,i+1} - delta_{i0} delta_{m0}
          T mass;
          const int fo = 3 * f;
          if (pre) {
            mass = xr[fo + c][i + 1][r];
          } else {
            const T* Mm = f == 0 ? Me : Mh;
            T v0 = xr[fo + 0][i + 1][r], v1 = xr[fo + 1][i + 1][r], v2 = xr[fo + 2][i + 1][r];
            if (i == 0) {
              v0 -= xr[fo + 0][0][r];
              v1 -= xr[fo + 1][0][r];
              v2 -= xr[fo + 2][0][r];
            }
            mass = symget(Mm, c, 0) * v0 + symget(Mm, c, 1) * v1 + symget(Mm, c, 2) * v2;
          }
          T out = mass + dt * (cu + lift);
          const int64_t o = (int64_t)((fo + c) * Q + i) * A3 + s;
          if (ld) out -= ld[o];
          ye[o] = out;
        }
      }
    }
    __syncthreads();
  }
}

// P^{-1} applied blockwise (3x3 per spatial mode and level), for meshes whose
// metric is not diagonal: z = P^{-1} x on the unknowns layout.
template <typename T>
__global__ void precond_scale_kernel(const ElemInfo* info, const ElemMetric* metric, int64_t ne, const T* x, T* z) {
  const int64_t e = blockIdx.x;
  if (e >= ne) return;
  const ElemInfo I = info[e];
  const int a3 = I.a * I.a * I.a;
  const int per = I.q * a3;
  const double* mm = metric[e].m;
  for (int idx = threadIdx.x; idx < 2 * per; idx += blockDim.x) {
    const int f = idx / per, rest = idx - f * per;
    const double* Mi = mm + 12 + 6 * f;
    const T* xb = x + I.unk_off + (int64_t)3 * f * per + rest;
    T* zb = z + I.unk_off + (int64_t)3 * f * per + rest;
    const T v0 = xb[0], v1 = xb[per], v2 = xb[2 * per];
    zb[0] = (T)(Mi[0] * v0 + Mi[3] * v1 + Mi[4] * v2);
    zb[per] = (T)(Mi[3] * v0 + Mi[1] * v1 + Mi[5] * v2);
    zb[2 * per] = (T)(Mi[4] * v0 + Mi[5] * v1 + Mi[2] * v2);
  }
}

}  // namespace stdg
