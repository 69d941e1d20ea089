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
// Dh[n][j] = int L_n L_j' = 2 rho_n rho_j for n < j, j - n odd, rho_j = sqrt(2j+1):
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
// A neighbour met in another orientation (its face f' and a symmetry of the
// square between the face coordinates) is read on its own face, with its
// covariant tangential components and face modes carried into this
// element's frame by the signed permutation of the face map.
//
// Dissipative stabilisation D_h (the remark closing Section 4), affine
// elements only (DISS kernels): with the time-contracted tangential jumps
// J_c = T_self(U_c) - T_nb(U_c) (T_self alone on PEC faces; zero on interior
// faces for i >= min(q, q'), where the projected test function vanishes)
//   R_E[c] += alpha_E L_{s_alpha}(side) sum_d K_cd J_d(E),
//   R_H[c] += alpha_H L_{s_alpha}(side) sum_d K_cd J_d(H)   (interior faces only)
// over the four faces whose normal is not c; K = |t_a x t_b| g^{-1} is the
// constant metric of the face, so the physical (n x v) . (n x u) becomes
// sum K_cd v_c u_d for covariant reference components.
//
// Work layout: NT = a^3 rounded up to a multiple of 64 threads per element.
// Thread s owns spatial position s: all 6 components and all time levels in
// registers, so the time contraction, the mass term, the loads and the stores
// need no exchange.  For faces, thread (tc, t) < 4 a^2 owns tangential
// component tc and tangential mode t; the loops over faces are unrolled, so
// every neighbour parameter is a uniform scalar and every load is a uniform
// base plus a per-thread offset plus a compile-time immediate.  Neighbour
// blocks come through L2, kept warm by the locality-ordered work list and the
// XCD-aware block order.  Contracted levels are staged in LDS scaled by
// w(s) = rho_j rho_k rho_l, which turns the curl contractions and the own
// face traces into plain (alternating) sums with one factor per position or
// face mode; the curl sums use 0/1 masks instead of branches, and all their
// reads stay inside the staged level because the E-test reads H components
// below its position and the H-test reads E components above it.
#pragma once

#include "internal.h"

namespace stdg {

template <int A>
struct KCfg {
  static constexpr int A2 = A * A, A3 = A * A * A;
  static constexpr int NT = ((A3 + 63) / 64) * 64;  // one spatial position per thread
  static constexpr int NF = 4 * A2;                 // face items per face
  static constexpr int ND = A / 2;                  // odd offsets 1, 3, .. < A
  // staged level: E~', H~' then the fluxes (and with D_h the tangential jumps)
  static constexpr int lvl(bool diss) { return 6 * A3 + (diss ? 48 : 24) * A2; }
  static constexpr int LVL = lvl(false);
  template <typename T, int Q, bool AFF = true, bool DISS = false>
  static constexpr int LC() {
    // test levels staged per LDS pass: about 16 KB (24 KB with the D_h jumps,
    // which keeps p = 4, q = 3 in one FP32 pass); one for trilinear elements
    constexpr int c = AFF ? (DISS ? 24576 : 16384) / (lvl(DISS) * (int)sizeof(T)) : 1;
    return c < 1 ? 1 : (c > Q ? Q : c);
  }
  // FP32 neighbour blocks are staged through LDS a face at a time (4
  // tangential component blocks of the stored levels, double-buffered) when a
  // face of q + 1 levels fits in 24 KB; FP64 blocks and larger faces are
  // gathered straight from global memory (measured faster there)
  template <typename T, int Q>
  static constexpr bool stage() { return sizeof(T) == 4 && 4 * (Q + 1) * A3 * (int)sizeof(T) <= 24576; }
  static constexpr int levels(int Q, int MODE) { return MODE == 1 ? Q + 1 : Q; }  // stored trial levels
  // trilinear elements: Gauss rule of GQ = a + 1 points per direction for the
  // mass; PP quadrature points per thread
  static constexpr int GQ = A + 1, G2 = GQ * GQ, G3 = G2 * GQ;
  static constexpr int PP = (G3 + NT - 1) / NT;
  static constexpr int MASS_A = 6 * A * G2, MASS = MASS_A + 6 * G3;  // two sweep buffers, both fields
  static constexpr int QTAB = GQ * A;                                // sqrt(w_g) L_j(x_g)
  static constexpr int QTAB_PAD = (QTAB + 3) & ~3;
  template <typename T, int Q, bool AFF, int MODE, bool DISS = false>
  static constexpr int main_elems() {
    // staged contracted levels, or (aliased, used earlier) the staging
    // buffers, or (aliased) the mass sweep buffers
    constexpr int NL = levels(Q, MODE);
    constexpr int a = LC<T, Q, AFF, DISS>() * lvl(DISS), b = stage<T, Q>() ? 2 * 4 * NL * A3 : 0;
    constexpr int ab = a > b ? a : b;
    return AFF ? ab : (ab > MASS ? ab : MASS);
  }
  template <typename T, int Q, bool AFF, int MODE, bool DISS = false>
  static constexpr int lds_elems() {
    // trilinear elements add the quadrature table and the metric at the points
    return main_elems<T, Q, AFF, MODE, DISS>() + (AFF ? 0 : QTAB_PAD + 6 * G3);
  }
};

template <typename T>
struct KParams {
  const ElemInfo* info;
  const ElemMetric* metric;
  const int32_t* list;
  const T* x;
  const T* load;
  T* y;
  const double* verts;    // [ne][8][3] (trilinear elements)
  const QTables<T>* qt;   // mass rule of this group's a (trilinear elements)
  const T* diss;          // D_h coefficients per element (dissipative kernels)
  const int* skip;        // device flag: 0 = return at once (NULL: always run)
  T dt;
  int mode;     // kept for launch bookkeeping; the kernels take the mode as a template argument
  int variant;  // launch variant (launch bookkeeping; the kernels take it as a template argument)
  Tables<T> tab;
};

__host__ __device__ constexpr bool nnzN(int i, int m) {
  return (i == 0 && m <= 2) || (i == 1 && (m == 0 || m == 1 || m == 3)) || (i >= 2 && (m == i || m == i + 2));
}

template <typename T>
__device__ __forceinline__ T symget(const T* M, int c, int d) {
  return c == d ? M[c] : ((c + d == 1) ? M[3] : ((c + d == 2) ? M[4] : M[5]));
}

template <typename T>
__device__ __forceinline__ T dsqrt(T v) {
  return sqrt(v);
}
template <>
__device__ __forceinline__ float dsqrt<float>(float v) {
  return __fsqrt_rn(v);
}

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t byte_off);
template <>
__device__ __forceinline__ float buf_load<float>(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)byte_off, 0, 0));
}
template <>
__device__ __forceinline__ double buf_load<double>(__amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)byte_off, 0, 0));
}

// Output stores are non-temporal (cache policy nt): y is written once and not
// read again by the launch, so streaming it past L2 leaves L2 to the
// neighbour blocks of x (measured: 3-5% faster applies, same results).
constexpr int kStoreNT = 2;
template <typename T>
__device__ __forceinline__ void buf_store(T v, __amdgpu_buffer_rsrc_t r, uint32_t byte_off);
template <>
__device__ __forceinline__ void buf_store<float>(float v, __amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)byte_off, 0, kStoreNT);
}
template <>
__device__ __forceinline__ void buf_store<double>(double v, __amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)byte_off, 0, kStoreNT);
}

// 8 bytes (two FP32 values or one FP64 value) at a byte offset that is a
// multiple of 8, non-temporal like buf_store
__device__ __forceinline__ void buf_store8(const void* lds_src, __amdgpu_buffer_rsrc_t r, uint32_t byte_off) {
  typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(*reinterpret_cast<const u32x2*>(lds_src), r, (int)byte_off, 0, kStoreNT);
}

// stride along the normal and base offset of tangential mode (u, v) on a
// face normal to alpha, in a block of edge n (x-hat index fastest)
__host__ __device__ constexpr int face_stride(int alpha, int n) { return alpha == 0 ? 1 : (alpha == 1 ? n : n * n); }
__device__ __forceinline__ int face_base(int alpha, int u, int v, int n) {
  return alpha == 0 ? n * u + n * n * v : (alpha == 1 ? u + n * n * v : u + n * v);
}

// How the neighbour across face (alpha, side) is read for this element's
// tangential component c and face mode (fu, fv) (u, v: the two tangential
// axes in increasing order), from the face's orientation byte: the
// neighbour's face axis and side, its component along the axis matched with
// ours, its mode along its (u', v') axes, and the sign: minus where the
// matched axis runs reversed (covariant components follow the tangent
// vector) times (-1)^j for mode j along each reversed axis (L_j(1 - x) =
// (-1)^j L_j(x)).
struct FaceMap {
  int ax, so, cn, mu, mv;
  bool neg;
};
__device__ __forceinline__ FaceMap map_face(int alpha, int code, int c, int fu, int fv) {
  FaceMap m;
  m.ax = (code & 7) >> 1;
  m.so = code & 1;
  const bool swp = (code & kOrientSwap) != 0, flu = (code & kOrientFlipU) != 0, flv = (code & kOrientFlipV) != 0;
  const int tu = alpha == 0 ? 1 : 0;                          // our u axis (v is the other one)
  const int tuo = m.ax == 0 ? 1 : 0, tvo = m.ax == 2 ? 1 : 2;  // the neighbour's u', v' axes
  const bool on_u = c == tu;
  m.cn = on_u ? (swp ? tvo : tuo) : (swp ? tuo : tvo);
  m.mu = swp ? fv : fu;
  m.mv = swp ? fu : fv;
  m.neg = (on_u ? flu : flv) ^ ((((flu ? fu : 0) + (flv ? fv : 0)) & 1) != 0);
  return m;
}

// Metric G = |J| DF^{-1} DF^{-T} of a trilinear map at the quadrature points
// (index (m GQ + h) GQ + g, g along x-hat), into LDS as Gl[entry][point].  With DF columns d0, d1, d2 the rows of DF^{-1} are
// (d1 x d2, d2 x d0, d0 x d1) / det, so G_ij = r_i . r_j / det.
template <typename T, int A>
__device__ __forceinline__ void trilinear_metric(const double* X, const QTables<T>* qt, int tid, T* __restrict__ Gl) {
  using C = KCfg<A>;
  // x(xi) = sum_S c_S prod_{d in S} xi_d over subsets S of the axes (bit d),
  // c_S = sum_{V subset S} (-1)^{|S| - |V|} X_V  (vertex V = x-hat bit fastest)
  T cs[8][3];
#pragma unroll
  for (int S = 0; S < 8; ++S)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
#pragma unroll
      for (int V = 0; V < 8; ++V)
        if ((V & S) == V) v += ((__builtin_popcount(S ^ V) & 1) ? -1.0 : 1.0) * X[3 * V + c];
      cs[S][c] = (T)v;
    }
#pragma unroll
  for (int k = 0; k < C::PP; ++k) {
    const int pt = tid + k * C::NT;
    if (pt >= C::G3) break;
    const T x1 = qt->x[pt % C::GQ], x2 = qt->x[(pt / C::GQ) % C::GQ], x3 = qt->x[pt / C::G2];
    T d[3][3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      d[0][c] = cs[1][c] + cs[3][c] * x2 + cs[5][c] * x3 + cs[7][c] * (x2 * x3);
      d[1][c] = cs[2][c] + cs[3][c] * x1 + cs[6][c] * x3 + cs[7][c] * (x1 * x3);
      d[2][c] = cs[4][c] + cs[5][c] * x1 + cs[6][c] * x2 + cs[7][c] * (x1 * x2);
    }
    T r[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const int i1 = (i + 1) % 3, i2 = (i + 2) % 3;
      r[i][0] = d[i1][1] * d[i2][2] - d[i1][2] * d[i2][1];
      r[i][1] = d[i1][2] * d[i2][0] - d[i1][0] * d[i2][2];
      r[i][2] = d[i1][0] * d[i2][1] - d[i1][1] * d[i2][0];
    }
    const T idet = T(1) / (d[0][0] * r[0][0] + d[0][1] * r[0][1] + d[0][2] * r[0][2]);
    const int ii[6] = {0, 1, 2, 0, 0, 1}, jj[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int k6 = 0; k6 < 6; ++k6)
      Gl[k6 * C::G3 + pt] = (r[ii[k6]][0] * r[jj[k6]][0] + r[ii[k6]][1] * r[jj[k6]][1] + r[ii[k6]][2] * r[jj[k6]][2]) * idet;
  }
}

// Mass of a trilinear element applied to both fields (6 components: E with
// eps, H with mu) of one level, by sum factorisation over the GQ^3 Gauss rule:
//   r_fc(s) = kappa_f sum_g phi_s(x_g) w_g (G(x_g) u_f(x_g))_c,
//   u_f(x_g) = sum_t phi_t(x_g) u_f,t.
// Bt = sqrt(w_g) L_j(x_g) in LDS (the weight split over both sweeps).  Sweeps
// alternate between bufA (6 A GQ^2) and bufB (6 GQ^3); the caller must
// synchronise before reusing the buffers for anything but another call.
template <typename T, int A>
__device__ __forceinline__ void trilinear_mass(T* __restrict__ bufA, T* __restrict__ bufB, const T* __restrict__ Bt,
                                               const T* __restrict__ Gl, T keps, T kmu, const T (&u)[6], T (&r)[6],
                                               int tid, bool pos_lane, uint32_t s) {
  using C = KCfg<A>;
  constexpr int A2 = C::A2, A3 = C::A3, GQ = C::GQ, G2 = C::G2, G3 = C::G3, NT = C::NT;
  constexpr int NC = 6;
  if (pos_lane) {
#pragma unroll
    for (int c = 0; c < NC; ++c) bufA[c * A3 + s] = u[c];
  }
  __syncthreads();
  // x-hat: [c][l][k][j] -> [c][l][k][g]
  for (int o = tid; o < NC * A2 * GQ; o += NT) {
    const int g = o % GQ, row = o / GQ;
    const T* src = bufA + row * A;
    const T* b = Bt + g * A;
    T acc = T(0);
#pragma unroll
    for (int j = 0; j < A; ++j) acc += b[j] * src[j];
    bufB[o] = acc;
  }
  __syncthreads();
  // y-hat: [c][l][k][g] -> [c][l][h][g]
  for (int o = tid; o < NC * A * G2; o += NT) {
    const int g = o % GQ, h = (o / GQ) % GQ, row = o / G2;
    const T* src = bufB + row * (A * GQ) + g;
    const T* b = Bt + h * A;
    T acc = T(0);
#pragma unroll
    for (int k = 0; k < A; ++k) acc += b[k] * src[k * GQ];
    bufA[o] = acc;
  }
  __syncthreads();
  // z-hat to the points, and the pointwise kappa G, for both fields
#pragma unroll
  for (int kk = 0; kk < C::PP; ++kk) {
    const int pt = tid + kk * NT;
    if (pt < G3) {
      const int m = pt / G2, hg = pt - m * G2;
      const T* b = Bt + m * A;
      T G[6];
#pragma unroll
      for (int k6 = 0; k6 < 6; ++k6) G[k6] = Gl[k6 * G3 + pt];
#pragma unroll
      for (int f = 0; f < 2; ++f) {
        T v[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          T acc = T(0);
#pragma unroll
          for (int l = 0; l < A; ++l) acc += b[l] * bufA[((3 * f + c) * A + l) * G2 + hg];
          v[c] = acc;
        }
        const T kap = f == 0 ? keps : kmu;
        bufB[(3 * f + 0) * G3 + pt] = kap * (G[0] * v[0] + G[3] * v[1] + G[4] * v[2]);
        bufB[(3 * f + 1) * G3 + pt] = kap * (G[3] * v[0] + G[1] * v[1] + G[5] * v[2]);
        bufB[(3 * f + 2) * G3 + pt] = kap * (G[4] * v[0] + G[5] * v[1] + G[2] * v[2]);
      }
    }
  }
  __syncthreads();
  // back along z-hat: [c][m][h][g] -> [c][l][h][g]
  for (int o = tid; o < NC * A * G2; o += NT) {
    const int hg = o % G2, l = (o / G2) % A, c = o / (A * G2);
    const T* src = bufB + c * G3 + hg;
    T acc = T(0);
#pragma unroll
    for (int m = 0; m < GQ; ++m) acc += Bt[m * A + l] * src[m * G2];
    bufA[o] = acc;
  }
  __syncthreads();
  // back along y-hat: [c][l][h][g] -> [c][l][k][g]
  for (int o = tid; o < NC * A2 * GQ; o += NT) {
    const int g = o % GQ, k = (o / GQ) % A, row = o / (A * GQ);
    const T* src = bufA + row * G2 + g;
    T acc = T(0);
#pragma unroll
    for (int h = 0; h < GQ; ++h) acc += Bt[h * A + k] * src[h * GQ];
    bufB[o] = acc;
  }
  __syncthreads();
  // back along x-hat, at this thread's position s = (j, k, l)
  {
    const int j = (int)(s % A), kl = (int)(s / A);
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      const T* src = bufB + (c * A2 + kl) * GQ;
      T acc = T(0);
#pragma unroll
      for (int g = 0; g < GQ; ++g) acc += Bt[g * A + j] * src[g];
      r[c] = acc;
    }
  }
}

// Element e's own block: all components and stored trial levels at this
// thread's position (levels not stored in this mode are zero).
template <typename T, int A, int Q, int MODE>
__device__ __forceinline__ void load_own(const KParams<T>& P, int e, int tid, T (&xr)[6][Q + 1]) {
  constexpr int A3 = KCfg<A>::A3;
  constexpr bool resid = MODE == 1;
  constexpr int m0 = resid ? 0 : 1;
  constexpr int NL = Q + 1 - m0;
  constexpr int BLK = 6 * NL * A3 * (int)sizeof(T);
  const ElemInfo* Ip = P.info + e;
  const T* xe = P.x + (resid ? Ip->trial_off : Ip->unk_off);
  const __amdgpu_buffer_rsrc_t rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)xe, (short)0, BLK, 0x00020000);
  const uint32_t so = (uint32_t)tid * (uint32_t)sizeof(T);
#pragma unroll
  for (int fc = 0; fc < 6; ++fc)
#pragma unroll
    for (int m = 0; m <= Q; ++m)
      xr[fc][m] = m >= m0 ? buf_load<T>(rsrc, so + (uint32_t)(((fc * NL + m - m0) * A3) * (int)sizeof(T))) : T(0);
}

// The residual of element e from its own block xr (already loaded) and its
// face neighbours.  VAR selects the launch shape (tuned per kernel group):
//   0  outputs staged through LDS and stored as contiguous 8-byte lanes,
//      neighbour faces loaded 3 at a time;
//   1  outputs stored per position (no LDS stage), faces 3 at a time;
//   2  outputs staged, neighbour faces loaded one at a time (fewer registers);
//   3  (trilinear elements) one workgroup per element and test level: only
//      level only_level's outputs (and its quadrature mass) are computed.
template <typename T, int A, int Q, int MODE, bool AFF, bool DISS, int VAR>
__device__ __forceinline__ void element_body(const KParams<T>& P, const int e, const T (&xr)[6][Q + 1],
                                             T* __restrict__ sm, const int tid, const int only_level) {
  using C = KCfg<A>;
  constexpr int A2 = C::A2, A3 = C::A3, NF = C::NF, ND = C::ND, LVL = C::lvl(DISS);
  constexpr int LC = C::template LC<T, Q, AFF, DISS>();
  static_assert(AFF || !DISS, "the dissipative terms need the constant face metric of affine elements");
  constexpr bool resid = MODE == 1, pre = MODE == 2;  // operator / residual / operator with P^{-1}
  constexpr bool kSelectCurl = sizeof(T) == 4 && A >= 7;
  static_assert(AFF || !pre, "trilinear elements take P^{-1} in a separate pass");
  constexpr int m0 = resid ? 0 : 1;                   // first trial level stored in x
  constexpr int NL = Q + 1 - m0;                      // trial levels stored per component
  constexpr int BLK = 6 * NL * A3 * (int)sizeof(T);   // bytes of one element block of x
  constexpr int WORDS = (int)sizeof(T) / 4;
  const ElemInfo* Ip = P.info + e;
  const T* xe = P.x + (resid ? Ip->trial_off : Ip->unk_off);
  T* ye = P.y + Ip->unk_off;

  // neighbour table, uniform per block
  int nb_id[6], nb_a[6], nb_q[6];
  const T* nb_x[6];
  bool fast = true;
#pragma unroll
  for (int g = 0; g < 6; ++g) {
    nb_id[g] = Ip->nb[g];
    nb_a[g] = A;
    nb_q[g] = Q;
    nb_x[g] = xe;
    if (nb_id[g] >= 0) {
      const ElemInfo* Np = P.info + nb_id[g];
      nb_a[g] = Np->a;
      nb_q[g] = Np->q;
      nb_x[g] = P.x + (resid ? Np->trial_off : Np->unk_off);
      fast = fast && nb_a[g] == A && nb_q[g] == Q;
    }
  }

  const bool pos_lane = tid < A3;
  const uint32_t s = pos_lane ? (uint32_t)tid : 0u;
  const bool face_lane = tid < NF;
  // face item of this thread; threads past the items compute offsets beyond
  // the block, which the buffer range check turns into zero loads
  const int tc = tid / A2;                 // tangential component slot 0..3
  const int t = tid - tc * A2;
  const int fu = t % A, fv = t / A;        // tangential mode (u, v)
  const int tf = tc >> 1;                  // field of that component

  // ---- neighbour traces, contracted in time: acc[face][i] --------------------
  T acc[6][Q];
#pragma unroll
  for (int g = 0; g < 6; ++g)
#pragma unroll
    for (int i = 0; i < Q; ++i) acc[g][i] = T(0);

  // The two uniform-degree paths come in two forms: elements whose
  // neighbours all meet them in canonical orientation (compile-time face
  // axes, strides and components), and, for affine kernels, elements with a
  // permuted face, whose neighbours are read on their own face f' through
  // the face map.  Trilinear kernels send permuted elements down the general
  // path.  (Written out rather than as one generic lambda: the lambda form
  // cost the trilinear kernels up to 57 VGPRs and an occupancy step.)
  const bool permuted = (Ip->flags & kPermuted) != 0;
  const bool hanging = (Ip->flags & kHanging) != 0;  // 2:1 hanging faces take the general path
  if ((!AFF && permuted) || hanging) fast = false;
  const bool fast_perm = AFF && fast && permuted;
  if (fast && !fast_perm && C::template stage<T, Q>()) {
    // Neighbour blocks are read with unit-stride (coalesced) loads - thread
    // tid takes entries tid, tid + NT, ... of each tangential component block -
    // for a batch of GB faces at once, then passed face by face through a
    // double-buffered LDS staging area where the face lanes reduce them.
    constexpr int CH = NL * A3;                     // entries per component block
    constexpr int KC = (CH + C::NT - 1) / C::NT;    // loads per thread per block
    constexpr int GBC0 = 96 / (4 * KC * WORDS);
    constexpr int GBC = VAR == 2 ? 1 : (GBC0 < 1 ? 1 : (GBC0 > 3 ? 3 : GBC0));  // at most 3 faces in flight: fewer VGPRs, more waves
    int nstaged = 0;  // staged faces so far (uniform): buffers strictly alternate
#pragma unroll
    for (int g0 = 0; g0 < 6; g0 += GBC) {
      T nbv[GBC][4][KC];
#pragma unroll
      for (int gg = 0; gg < GBC; ++gg) {
        const int g = g0 + gg;
        if (g >= 6) break;
        if (nb_id[g] < 0) continue;
        // the neighbour's tangential blocks on its own face axis
        const int ax = g >> 1;
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc((void*)nb_x[g], (short)0, BLK, 0x00020000);
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int fc = 3 * (q4 >> 1) + (ax + 1 + (q4 & 1)) % 3;
#pragma unroll
          for (int k = 0; k < KC; ++k)
            nbv[gg][q4][k] = buf_load<T>(rsrc, (uint32_t)((fc * CH + k * C::NT) * (int)sizeof(T)) +
                                                   (uint32_t)tid * (uint32_t)sizeof(T));
        }
      }
#pragma unroll
      for (int gg = 0; gg < GBC; ++gg) {
        const int g = g0 + gg;
        if (g >= 6) break;
        if (nb_id[g] < 0) continue;
        const int alpha = g >> 1, side = g & 1;
        T* stg = sm + (nstaged & 1) * (4 * CH);
        ++nstaged;
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
          for (int k = 0; k < KC; ++k) {
            const int p = tid + k * C::NT;
            if (CH % C::NT == 0 || p < CH) stg[q4 * CH + p] = nbv[gg][q4][k];
          }
        __syncthreads();
        if (!face_lane) continue;
        const int c = (alpha + 1 + (tc & 1)) % 3;
        const T scale = pre ? (T)P.metric[nb_id[g]].m[12 + 6 * tf + c] : T(1);
        const int ns = face_stride(alpha, A);
        const T* src = stg + tc * CH + face_base(alpha, fu, fv, A);
        // the neighbour's face sits at 1 - side: weights L_l(1 - side)
#pragma unroll
        for (int ml = 0; ml < NL; ++ml) {
          const int mp = ml + m0;
          T tr = T(0);
#pragma unroll
          for (int l = 0; l < A; ++l) tr += (side ? P.tab.tr0[l] : P.tab.tr1[l]) * src[ml * A3 + l * ns];
          tr *= scale;
#pragma unroll
          for (int i = 0; i < Q; ++i)
            if (nnzN(i, mp)) acc[g][i] += P.tab.N[i][mp] * tr;
        }
      }
    }
    __syncthreads();  // staging area is reused for the contracted levels
  } else if (fast_perm && C::template stage<T, Q>()) {
    // Neighbour blocks are read with unit-stride (coalesced) loads - thread
    // tid takes entries tid, tid + NT, ... of each tangential component block -
    // for a batch of GB faces at once, then passed face by face through a
    // double-buffered LDS staging area where the face lanes reduce them.
    constexpr int CH = NL * A3;                     // entries per component block
    constexpr int KC = (CH + C::NT - 1) / C::NT;    // loads per thread per block
    constexpr int GBC0 = 96 / (4 * KC * WORDS);
    constexpr int GBC = VAR == 2 ? 1 : (GBC0 < 1 ? 1 : (GBC0 > 3 ? 3 : GBC0));  // at most 3 faces in flight: fewer VGPRs, more waves
    int nstaged = 0;  // staged faces so far (uniform): buffers strictly alternate
#pragma unroll
    for (int g0 = 0; g0 < 6; g0 += GBC) {
      T nbv[GBC][4][KC];
#pragma unroll
      for (int gg = 0; gg < GBC; ++gg) {
        const int g = g0 + gg;
        if (g >= 6) break;
        if (nb_id[g] < 0) continue;
        // the neighbour's tangential blocks on its own face axis
        const int ax = (Ip->orient[g] & 7) >> 1;
        const __amdgpu_buffer_rsrc_t rsrc =
            __builtin_amdgcn_make_buffer_rsrc((void*)nb_x[g], (short)0, BLK, 0x00020000);
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4) {
          const int fc = 3 * (q4 >> 1) + (ax + 1 + (q4 & 1)) % 3;
#pragma unroll
          for (int k = 0; k < KC; ++k)
            nbv[gg][q4][k] = buf_load<T>(rsrc, (uint32_t)((fc * CH + k * C::NT) * (int)sizeof(T)) +
                                                   (uint32_t)tid * (uint32_t)sizeof(T));
        }
      }
#pragma unroll
      for (int gg = 0; gg < GBC; ++gg) {
        const int g = g0 + gg;
        if (g >= 6) break;
        if (nb_id[g] < 0) continue;
        const int alpha = g >> 1, side = g & 1;
        T* stg = sm + (nstaged & 1) * (4 * CH);
        ++nstaged;
#pragma unroll
        for (int q4 = 0; q4 < 4; ++q4)
#pragma unroll
          for (int k = 0; k < KC; ++k) {
            const int p = tid + k * C::NT;
            if (CH % C::NT == 0 || p < CH) stg[q4 * CH + p] = nbv[gg][q4][k];
          }
        __syncthreads();
        if (!face_lane) continue;
        // the neighbour's face f' at the mapped mode, matched component and sign
        const FaceMap fm = map_face(alpha, Ip->orient[g], (alpha + 1 + (tc & 1)) % 3, fu, fv);
        const int slot = 2 * tf + (fm.cn == (fm.ax + 1) % 3 ? 0 : 1);
        const T scale = (pre ? (T)P.metric[nb_id[g]].m[12 + 6 * tf + fm.cn] : T(1)) * (fm.neg ? T(-1) : T(1));
        const int ns = face_stride(fm.ax, A);
        const T* src = stg + slot * CH + face_base(fm.ax, fm.mu, fm.mv, A);
#pragma unroll
        for (int ml = 0; ml < NL; ++ml) {
          const int mp = ml + m0;
          T tr = T(0);
#pragma unroll
          for (int l = 0; l < A; ++l) tr += (fm.so ? P.tab.tr1[l] : P.tab.tr0[l]) * src[ml * A3 + l * ns];
          tr *= scale;
#pragma unroll
          for (int i = 0; i < Q; ++i)
            if (nnzN(i, mp)) acc[g][i] += P.tab.N[i][mp] * tr;
        }
      }
    }
    __syncthreads();  // staging area is reused for the contracted levels
  } else if (fast && !fast_perm) {
    // faces too large to stage: gather each face item straight from global
    // memory (one buffer descriptor per face, compile-time immediates)
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      if (nb_id[g] < 0) continue;
      const int alpha = g >> 1, side = g & 1;
      const int c = (alpha + 1 + (tc & 1)) % 3;
      // canonical: the neighbour's face (alpha, 1 - side), same component and mode
      FaceMap fm{alpha, 1 - side, c, fu, fv, false};
      const int ns = face_stride(fm.ax, A);
      const __amdgpu_buffer_rsrc_t rsrc =
          __builtin_amdgcn_make_buffer_rsrc((void*)nb_x[g], (short)0, BLK, 0x00020000);
      const uint32_t lo = (uint32_t)(((3 * tf + fm.cn) * NL * A3 + face_base(fm.ax, fm.mu, fm.mv, A)) * (int)sizeof(T));
      T vals[NL][A];
#pragma unroll
      for (int ml = 0; ml < NL; ++ml)
#pragma unroll
        for (int l = 0; l < A; ++l) vals[ml][l] = buf_load<T>(rsrc, lo + (uint32_t)((ml * A3 + l * ns) * (int)sizeof(T)));
      if (!face_lane) continue;
      const T scale = (pre ? (T)P.metric[nb_id[g]].m[12 + 6 * tf + fm.cn] : T(1)) * (fm.neg ? T(-1) : T(1));
#pragma unroll
      for (int ml = 0; ml < NL; ++ml) {
        const int mp = ml + m0;
        T tr = T(0);
#pragma unroll
        for (int l = 0; l < A; ++l) tr += (fm.so ? P.tab.tr1[l] : P.tab.tr0[l]) * vals[ml][l];
        tr *= scale;
#pragma unroll
        for (int i = 0; i < Q; ++i)
          if (nnzN(i, mp)) acc[g][i] += P.tab.N[i][mp] * tr;
      }
    }
  } else if (fast_perm) {
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      if (nb_id[g] < 0) continue;
      const int alpha = g >> 1, side = g & 1;
      const int c = (alpha + 1 + (tc & 1)) % 3;
      // canonical: the neighbour's face (alpha, 1 - side), same component and mode
      FaceMap fm{alpha, 1 - side, c, fu, fv, false};
      fm = map_face(alpha, Ip->orient[g], c, fu, fv);
      const int ns = face_stride(fm.ax, A);
      const __amdgpu_buffer_rsrc_t rsrc =
          __builtin_amdgcn_make_buffer_rsrc((void*)nb_x[g], (short)0, BLK, 0x00020000);
      const uint32_t lo = (uint32_t)(((3 * tf + fm.cn) * NL * A3 + face_base(fm.ax, fm.mu, fm.mv, A)) * (int)sizeof(T));
      T vals[NL][A];
#pragma unroll
      for (int ml = 0; ml < NL; ++ml)
#pragma unroll
        for (int l = 0; l < A; ++l) vals[ml][l] = buf_load<T>(rsrc, lo + (uint32_t)((ml * A3 + l * ns) * (int)sizeof(T)));
      if (!face_lane) continue;
      const T scale = (pre ? (T)P.metric[nb_id[g]].m[12 + 6 * tf + fm.cn] : T(1)) * (fm.neg ? T(-1) : T(1));
#pragma unroll
      for (int ml = 0; ml < NL; ++ml) {
        const int mp = ml + m0;
        T tr = T(0);
#pragma unroll
        for (int l = 0; l < A; ++l) tr += (fm.so ? P.tab.tr1[l] : P.tab.tr0[l]) * vals[ml][l];
        tr *= scale;
#pragma unroll
        for (int i = 0; i < Q; ++i)
          if (nnzN(i, mp)) acc[g][i] += P.tab.N[i][mp] * tr;
      }
    }
  } else if (face_lane) {
    // different degrees or orientations around this element: p-truncated
    // coupling, S_h drops the neighbour term on test levels i >= min(q, q'),
    // and a neighbour met in another orientation is read on its own face f'
    // through the face map (strides are run-time here anyway: na varies)
#pragma unroll
    for (int g = 0; g < 6; ++g) {
      const int alpha = g >> 1;
      if (nb_id[g] < 0) continue;
      // 2:1 hanging faces: the neighbours' part of the flux is added by the
      // hanging-face kernel after this one (the own part is taken here)
      if (Ip->flags & (kHangFaceBase << g)) continue;
      const int c = (alpha + 1 + (tc & 1)) % 3;
      const FaceMap fm = map_face(alpha, Ip->orient[g], c, fu, fv);
      const T scale = (pre ? (T)P.metric[nb_id[g]].m[12 + 6 * tf + fm.cn] : T(1)) * (fm.neg ? T(-1) : T(1));
      const int na = nb_a[g], nq = nb_q[g];
      if (fu >= na || fv >= na) continue;
      const int na3 = na * na * na;
      const int ns = face_stride(fm.ax, na);
      const int nnlev = resid ? nq + 1 : nq;
      const T* xb = nb_x[g] + (int64_t)(3 * tf + fm.cn) * nnlev * na3 + face_base(fm.ax, fm.mu, fm.mv, na);
#pragma unroll
      for (int mp = 0; mp <= kMaxQ; ++mp) {
        if (mp < m0 || mp > nq) continue;
        const T* xl = xb + (int64_t)(mp - m0) * na3;
        T tr = T(0);
        // trace on the neighbour's face at its side: L_l(side')
        for (int l = 0; l < na; ++l) {
          const T rho = dsqrt<T>(T(2 * l + 1));
          tr += ((fm.so == 0 && (l & 1)) ? -rho : rho) * xl[l * ns];
        }
        tr *= scale;
#pragma unroll
        for (int i = 0; i < Q; ++i)
          if (nnzN(i, mp) && i < nq) acc[g][i] += P.tab.N[i][mp] * tr;
      }
    }
  }

  // ---- metric (uniform), per-position and per-face-mode constants ------------
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
  int sidx[3];
  sidx[0] = (int)(s % A);
  sidx[1] = (int)((s / A) % A);
  sidx[2] = (int)(s / A2);
  T rsm[3], sg[3], cf[3], mE[3][ND > 0 ? ND : 1], mH[3][ND > 0 ? ND : 1];
  T w = T(1);
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    rsm[m] = dsqrt<T>(T(2 * sidx[m] + 1));
    sg[m] = (sidx[m] & 1) ? T(-1) : T(1);
    w *= rsm[m];
#pragma unroll
    for (int dd = 0; dd < ND; ++dd) {
      mE[m][dd] = sidx[m] >= 2 * dd + 1 ? T(1) : T(0);
      mH[m][dd] = sidx[m] + 2 * dd + 1 < A ? T(1) : T(0);
    }
  }
  const T winv = T(1) / w;

  // trilinear elements: quadrature table and the metric at the points, in LDS
  T* qB = sm + C::template main_elems<T, Q, AFF, MODE, DISS>();
  T* Gl = qB + C::QTAB_PAD;
  T keps = T(0), kmu = T(0);
  if constexpr (!AFF) {
    for (int k = tid; k < C::QTAB; k += C::NT) qB[k] = P.qt->B[k];
    trilinear_metric<T, A>(P.verts + 24 * (int64_t)e, P.qt, tid, Gl);
    keps = (T)P.metric[e].eps;
    kmu = (T)P.metric[e].mu;
  }
  // Dh[n][s_m] X(s_m -> n) = 2 rho_{s_m}^2 / w(s) * (w X)(s_m -> n)
#pragma unroll
  for (int m = 0; m < 3; ++m) cf[m] = T(2 * (2 * sidx[m] + 1)) * winv;
  // sum_l L_l(side) X_l = (1 / (rho_u rho_v)) sum_l (+-1)^l (w X)_l
  const T iuv = T(1) / (dsqrt<T>(T(2 * fu + 1)) * dsqrt<T>(T(2 * fv + 1)));
  const int tgt[3] = {sidx[1] + A * sidx[2], sidx[0] + A * sidx[2], sidx[0] + A * sidx[1]};
  constexpr int stride[3] = {1, A, A2};

  // D_h coefficients (uniform, loaded once; read at their use they would be
  // reloaded after every output store): alpha_E, alpha_H per face, face metric
  // per axis
  T dc[DISS ? Mesh::kDissWords : 1];
  if constexpr (DISS) {
    const T* src = P.diss + (int64_t)Mesh::kDissWords * e;
#pragma unroll
    for (int k = 0; k < 21; ++k) dc[k] = src[k];
  }

  const T dt = P.dt;
  const bool has_load = resid && P.load != nullptr;
  const __amdgpu_buffer_rsrc_t yrs =
      __builtin_amdgcn_make_buffer_rsrc((void*)ye, (short)0, 6 * Q * A3 * (int)sizeof(T), 0x00020000);
  const __amdgpu_buffer_rsrc_t lrs = __builtin_amdgcn_make_buffer_rsrc(
      (void*)(has_load ? P.load + Ip->unk_off : ye), (short)0, 6 * Q * A3 * (int)sizeof(T), 0x00020000);
  const uint32_t so = (uint32_t)tid * (uint32_t)sizeof(T);
  // outputs staged through LDS when every level is in one pass (the element's
  // outputs are then one contiguous run, 8-byte aligned: 6 q a^3 is even)
  constexpr bool kStageOut = VAR != 1 && LC == Q && 6 * Q * A3 <= C::template main_elems<T, Q, AFF, MODE, DISS>();
  T yo[kStageOut ? Q : 1][6];

#pragma unroll
  for (int i0 = 0; i0 < Q; i0 += LC) {
    if (VAR == 3 && i0 != only_level) continue;  // uniform: this workgroup's test level only (LC = 1)
    // trilinear elements: the mass terms of these levels, by quadrature
    T mres[AFF ? 1 : LC][6];
    if constexpr (!AFF) {
#pragma unroll
      for (int ii = 0; ii < LC; ++ii) {
        const int i = i0 + ii;
        if (i >= Q) break;
        T u[6], r[6];
#pragma unroll
        for (int c = 0; c < 6; ++c) u[c] = xr[c][i + 1] - ((resid && i == 0) ? xr[c][0] : T(0));
        trilinear_mass<T, A>(sm, sm + C::MASS_A, qB, Gl, keps, kmu, u, r, tid, pos_lane, s);
#pragma unroll
        for (int c = 0; c < 6; ++c) mres[ii][c] = r[c];
      }
      __syncthreads();  // the sweep buffers alias the staged levels
    }
    // (a) contracted levels, scaled by w(s), into LDS
    if (pos_lane) {
#pragma unroll
      for (int ii = 0; ii < LC; ++ii) {
        const int i = i0 + ii;
        if (i >= Q) break;
#pragma unroll
        for (int f = 0; f < 2; ++f) {
          T et[3];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            T v = T(0);
#pragma unroll
            for (int m = 0; m <= Q; ++m)
              if (nnzN(i, m) && m >= m0) v += P.tab.N[i][m] * xr[3 * f + c][m];
            et[c] = v;
          }
          if (pre) {
            const T* Mi = f == 0 ? Ie : Ih;
            T z[3];
#pragma unroll
            for (int c = 0; c < 3; ++c)
              z[c] = symget(Mi, c, 0) * et[0] + symget(Mi, c, 1) * et[1] + symget(Mi, c, 2) * et[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) et[c] = z[c];
          }
#pragma unroll
          for (int c = 0; c < 3; ++c) sm[ii * LVL + (3 * f + c) * A3 + s] = w * et[c];
        }
      }
    }
    __syncthreads();

    // (b) face fluxes: own traces of both faces of an axis from one pass, plus
    //     the neighbour traces
    if (face_lane) {
#pragma unroll
      for (int alpha = 0; alpha < 3; ++alpha) {
        const int c = (alpha + 1 + (tc & 1)) % 3;
        const int ns = face_stride(alpha, A);
        const int base = (3 * tf + c) * A3 + face_base(alpha, fu, fv, A);
#pragma unroll
        for (int ii = 0; ii < LC; ++ii) {
          const int i = i0 + ii;
          if (i >= Q) break;
          const T* src = sm + ii * LVL + base;
          T s1 = T(0), s0 = T(0);
#pragma unroll
          for (int l = 0; l < A; ++l) {
            const T v = src[l * ns];
            s1 += v;
            s0 += (l & 1) ? -v : v;
          }
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int g = 2 * alpha + side;
            const bool has = nb_id[g] >= 0;
            const T ws = has ? T(0.5) : T(1);
            T val = (tf == 0 ? -ws : ws) * iuv * (side ? s1 : s0);  // G = -w T(E), F = w T(H)
            if (has) val += T(0.5) * acc[g][i];
            sm[ii * LVL + 6 * A3 + (g * 4 + tc) * A2 + t] = val;
            if constexpr (DISS) {
              // tangential jump own - neighbour of this component; on interior
              // faces rows i >= min(q, q') vanish (D_h tests with the function
              // projected onto the common temporal test space)
              const T own = iuv * (side ? s1 : s0);
              const T jmp = !has ? own : (i < nb_q[g] ? own - acc[g][i] : T(0));
              sm[ii * LVL + 6 * A3 + 24 * A2 + (g * 4 + tc) * A2 + t] = jmp;
            }
          }
        }
      }
    }
    __syncthreads();

    // (c) outputs: mass + dt (curl + lift) - load
    if (pos_lane) {
#pragma unroll
      for (int ii = 0; ii < LC; ++ii) {
        const int i = i0 + ii;
        if (i >= Q) break;
        const T* Et = sm + ii * LVL;
        const T* Fl = Et + 6 * A3;
#pragma unroll
        for (int f = 0; f < 2; ++f) {
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
            // curl: the other field's components c2 (along axis c1) and c1 (along axis c2)
            const T* X2 = Et + ((f == 0 ? 3 : 0) + c2) * A3 + s;
            const T* X1 = Et + ((f == 0 ? 3 : 0) + c1) * A3 + s;
            T p1 = T(0), p2 = T(0);
#pragma unroll
            for (int dd = 0; dd < ND; ++dd) {
              const int d = 2 * dd + 1;
              if constexpr (kSelectCurl) {
                // selects instead of 0/1 factors: fewer live registers (measured
                // faster for FP32 with p >= 6, slower elsewhere)
                if (f == 0) {
                  p1 += sidx[c1] >= d ? X2[-d * stride[c1]] : T(0);
                  p2 += sidx[c2] >= d ? X1[-d * stride[c2]] : T(0);
                } else {
                  p1 += sidx[c1] + d < A ? X2[d * stride[c1]] : T(0);
                  p2 += sidx[c2] + d < A ? X1[d * stride[c2]] : T(0);
                }
              } else if (f == 0) {
                p1 += mE[c1][dd] * X2[-d * stride[c1]];
                p2 += mE[c2][dd] * X1[-d * stride[c2]];
              } else {
                p1 += mH[c1][dd] * X2[d * stride[c1]];
                p2 += mH[c2][dd] * X1[d * stride[c2]];
              }
            }
            const T cu = cf[c1] * p1 - cf[c2] * p2;
            // lifts from the four faces whose normal is not c
            T lift = T(0);
#pragma unroll
            for (int wv = 0; wv < 2; ++wv) {
              const int alpha = wv == 0 ? c1 : c2;
              const int dcomp = wv == 0 ? c2 : c1;
              const T epsv = (alpha == c2) ? T(1) : T(-1);  // eps(c, d, alpha)
              const int tcd = (dcomp == (alpha + 1) % 3 ? 0 : 1) + (f == 0 ? 2 : 0);
              const T v0 = Fl[((2 * alpha + 0) * 4 + tcd) * A2 + tgt[alpha]];
              const T v1 = Fl[((2 * alpha + 1) * 4 + tcd) * A2 + tgt[alpha]];
              // sigma L_{s_alpha}(side): +rho on side 1, -(-1)^{s_alpha} rho on side 0
              const T lv = rsm[alpha] * (v1 - sg[alpha] * v0);
              lift += (f == 0 ? epsv : -epsv) * lv;
            }
            // mass: the time-derivative factor is the shift delta_{m,i+1} - delta_{i0} delta_{m0}
            T mass;
            if constexpr (!AFF) {
              mass = mres[ii][3 * f + c];
            } else if (pre) {
              mass = xr[3 * f + c][i + 1];
            } else {
              const T* Mm = f == 0 ? Me : Mh;
              T v0 = xr[3 * f + 0][i + 1], v1 = xr[3 * f + 1][i + 1], v2 = xr[3 * f + 2][i + 1];
              if (resid && i == 0) {
                v0 -= xr[3 * f + 0][0];
                v1 -= xr[3 * f + 1][0];
                v2 -= xr[3 * f + 2][0];
              }
              mass = symget(Mm, c, 0) * v0 + symget(Mm, c, 1) * v1 + symget(Mm, c, 2) * v2;
            }
            // D_h: sum over the four faces whose normal is not c of
            // alpha_f L_{s_alpha}(side) (K jump)_c, jumps of field f itself
            T dl = T(0);
            if constexpr (DISS) {
              const T* Dl = Fl + 24 * A2;
              const T* al = dc + 6 * f;
#pragma unroll
              for (int wv = 0; wv < 2; ++wv) {
                const int alpha = wv == 0 ? c1 : c2;
                const int ka = c == (alpha + 1) % 3 ? 0 : 1;  // slot of component c on faces normal to alpha
                const int sd = 2 * f + ka, sx = 2 * f + 1 - ka;
                const T kd = dc[12 + 3 * alpha + ka], ko = dc[12 + 3 * alpha + 2];
                const T* d0 = Dl + (2 * alpha) * 4 * A2 + tgt[alpha];
                const T* d1 = Dl + (2 * alpha + 1) * 4 * A2 + tgt[alpha];
                const T j0 = kd * d0[sd * A2] + ko * d0[sx * A2];
                const T j1 = kd * d1[sd * A2] + ko * d1[sx * A2];
                // L_l(1) = rho_l, L_l(0) = (-1)^l rho_l
                dl += rsm[alpha] * (al[2 * alpha + 1] * j1 + sg[alpha] * al[2 * alpha] * j0);
              }
            }
            T out = mass + dt * (cu + lift + dl);
            const uint32_t o = so + (uint32_t)((((3 * f + c) * Q + i) * A3) * (int)sizeof(T));
            if (has_load) out -= buf_load<T>(lrs, o);
            if constexpr (kStageOut)
              yo[ii][3 * f + c] = out;
            else
              buf_store<T>(out, yrs, o);
          }
        }
      }
    }
    if (VAR != 3 && i0 + LC < Q) __syncthreads();
  }
  if constexpr (kStageOut) {
    // The element's outputs (contiguous: all levels in one pass) go through
    // LDS and leave as contiguous 8-byte stores, so each store instruction
    // covers whole cache lines: per-position stores of the a^3-value runs
    // left partial lines at every run boundary, which the streaming stores
    // sent to memory as partial writes.  The staged levels are dead here.
    __syncthreads();
    if (pos_lane) {
#pragma unroll
      for (int ii = 0; ii < Q; ++ii)
#pragma unroll
        for (int fc = 0; fc < 6; ++fc) sm[(fc * Q + ii) * A3 + s] = yo[ii][fc];
    }
    __syncthreads();
    constexpr int N8 = 6 * Q * A3 * (int)sizeof(T) / 8;  // 8-byte units of the element's outputs
#pragma unroll
    for (int k = 0; k < (N8 + C::NT - 1) / C::NT; ++k) {
      const int u = tid + k * C::NT;
      if (N8 % C::NT == 0 || u < N8) buf_store8(reinterpret_cast<const char*>(sm) + 8 * u, yrs, (uint32_t)(8 * u));
    }
  }
}

template <typename T, int A, int Q, bool AFF, bool DISS>
constexpr bool C_LC1() { return KCfg<A>::template LC<T, Q, AFF, DISS>() == 1; }

// One workgroup per element (per element and test level in variant 3).
// Consecutive work-list entries run on one XCD
// (blocks are dispatched to the 8 XCDs round-robin), so neighbour blocks are
// found in that XCD's L2.
template <typename T, int A, int Q, int MODE, bool AFF, bool DISS = false, int VAR = 0>
__global__ void __launch_bounds__(KCfg<A>::NT) residual_kernel(KParams<T> P) {
  if (P.skip && *P.skip == 0) return;  // uniform: a finished restart cycle
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  const uint32_t nblk = gridDim.x, b = blockIdx.x;
  const uint32_t xcd = b & 7u, idx = b >> 3;
  const uint32_t qq = nblk >> 3, rr = nblk & 7u;
  const uint32_t logical = xcd * qq + (xcd < rr ? xcd : rr) + idx;
  static_assert(VAR != 3 || (!AFF && C_LC1<T, A, Q, AFF, DISS>()), "level split: trilinear elements, one level per pass");
  // variant 3: blocks (element, level), the levels of an element consecutive (same XCD)
  const int e = P.list[VAR == 3 ? logical / Q : logical];
  const int lev = VAR == 3 ? (int)(logical % Q) : -1;
  T xr[6][Q + 1];
  load_own<T, A, Q, MODE>(P, e, tid, xr);
  element_body<T, A, Q, MODE, AFF, DISS, VAR>(P, e, xr, sm, tid, lev);
}

// Batched preconditioned operator applies (mode 2) over the meshes of several
// requests that share one affine (a, q) kernel group with a diagonal metric
// and no D_h: the serving loop's restart cycles in lockstep.  Each request
// takes a segment of the grid (its work list in order); the block-to-segment
// lookup follows the same XCD-aware order as the plain kernel, and the
// element body is the plain kernel's, so every output is bitwise the same.
constexpr int kMaxApplyBatch = 16;
template <typename T>
struct BatchMember {
  const ElemInfo* info;
  const ElemMetric* metric;
  const int32_t* list;
  const T* x;
  T* y;
  const int* skip;  // device flag: 0 = this request's cycle has ended
  T dt;
  uint32_t first;   // the request's first logical block
};
template <typename T>
struct BatchKParams {
  BatchMember<T> m[kMaxApplyBatch];
  int count;
  Tables<T> tab;
};

template <typename T, int A, int Q>
__global__ void __launch_bounds__(KCfg<A>::NT) residual_batch_kernel(BatchKParams<T> B) {
  extern __shared__ __align__(16) unsigned char smem_raw[];
  T* sm = reinterpret_cast<T*>(smem_raw);
  const int tid = threadIdx.x;
  const uint32_t nblk = gridDim.x, b = blockIdx.x;
  const uint32_t xcd = b & 7u, idx = b >> 3;
  const uint32_t qq = nblk >> 3, rr = nblk & 7u;
  const uint32_t logical = xcd * qq + (xcd < rr ? xcd : rr) + idx;
  int mi = 0;
  for (int k = 1; k < B.count; ++k)
    if (logical >= B.m[k].first) mi = k;
  const BatchMember<T>& M = B.m[mi];
  if (M.skip && *M.skip == 0) return;  // uniform: that request's restart cycle has ended
  KParams<T> P;
  P.info = M.info;
  P.metric = M.metric;
  P.list = M.list;
  P.x = M.x;
  P.load = nullptr;
  P.y = M.y;
  P.verts = nullptr;
  P.qt = nullptr;
  P.diss = nullptr;
  P.skip = M.skip;
  P.dt = M.dt;
  P.mode = 2;
  P.variant = 0;
  P.tab = B.tab;
  const int e = P.list[logical - M.first];
  T xr[6][Q + 1];
  load_own<T, A, Q, 2>(P, e, tid, xr);
  element_body<T, A, Q, 2, true, false, 0>(P, e, xr, sm, tid, -1);
}

// P^{-1} applied blockwise (3x3 per spatial mode and level), for meshes whose
// metric is not diagonal: z = P^{-1} x on the unknowns layout.
template <typename T>
__global__ void precond_scale_kernel(const ElemInfo* info, const ElemMetric* metric, int64_t ne, const T* x, T* z,
                                     const int* skip) {
  if (skip && *skip == 0) return;
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
