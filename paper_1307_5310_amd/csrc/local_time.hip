// Rows of the elements with local time steps (Section 2.2: a macro-element's
// slab interval bisected into n equal sub-intervals; eq. spaces:local:patch)
// and of their face neighbours: one workgroup per such element, every test
// level I = j q + i in turn.  The same terms as the residual kernels, with the
// time factors read from tables instead of the one-interval shift and N:
//   mass   R_F[c,I,s] += sum_d M_F[c][d] sum_M D[I][M] x_F[d,M,s]
//   curl   with the contracted fields F~_I = sum_M N[I][M] x_F[., M]:
//          R_H[c] += dt (sum_n Dh[s_c1][n] E~_c2(s_c1 -> n) - sum_n Dh[s_c2][n] E~_c1(s_c2 -> n))
//          R_E[c] += dt (sum_n Dh[n][s_c1] H~_c2(s_c1 -> n) - sum_n Dh[n][s_c2] H~_c1(s_c2 -> n))
//          ((c1, c2) = (c + 1, c + 2) mod 3)
//   faces  F = 1/2 T_self(H~) + 1/2 T_nb(H), G = -1/2 T_self(E~) + 1/2 T_nb(E)
//          (interior), F = T_self(H~), G = -T_self(E~) (PEC), lifted as
//          R_E[c] += dt sigma eps(c,d,alpha) L_{s_alpha}(side) F_d,
//          R_H[c] -= dt sigma eps(c,d,alpha) L_{s_alpha}(side) G_d,  d = 3 - c - alpha
// where T_nb contracts the neighbour's trial levels with the coupling table
// C[I][M'] = int (pi L_I) phi'_M' of S_h (Section 4.1, eq. bilinearform:S: the
// test function projected onto the common temporal test space), in this
// element's covariant frame through the face orientation, modes < min(a, a').
// D[I][M] = int L_I d_s phi_M and N[I][M] = int L_I phi_M are the element's own
// tables over the unit slab coordinate s.  Elements with one sub-interval
// whose neighbour has several run here too (their coupling changes).
// One workgroup per (element, sub-interval), one thread per spatial
// position, instantiated per a = p + 1: the q test levels of one
// sub-interval.  Its table rows are staged in LDS, each thread keeps the
// sub-interval's q + 1 own trial levels of its position (all six components)
// in registers, and when they fit (dynamic LDS, 64 KB) the neighbours' traces
// contracted for all q levels are staged once (each neighbour level read once
// per workgroup); otherwise every level gathers them from global memory.
#include <algorithm>

#include "internal.h"

namespace stdg {

namespace {

template <typename T>
struct LParams {
  const ElemInfo* info;
  const ElemMetric* metric;
  const LTRec* rec;
  const T* bank;    // time tables (LTRec offsets)
  const T* x;
  const T* load;    // residual mode: subtracted (may be NULL)
  T* y;
  const int32_t* work;  // per workgroup: record index * kMaxSub + sub-interval
  const T* diss;        // D_h coefficients per element (Mesh::kDissWords each), NULL = off
  const int* skip;
  T dt;
  int resid;        // x is the full trial vector (levels 0..), else the unknowns (levels 1..)
  int staged;       // the own levels and the neighbours' traces of a sub-interval fit in LDS
  Tables<T> tab;    // Dh and the face traces
};

__device__ inline int axis_stride(int axis, int a) { return axis == 0 ? 1 : (axis == 1 ? a : a * a); }

template <int A>
struct LCfg {
  static constexpr int NT = ((A * A * A + 63) / 64) * 64;  // one spatial position per thread
};

// FP32, p <= 4, q <= 4 without D_h: five waves per SIMD (at most 102 VGPRs;
// they fit without scratch, and the kernel waits on memory most of its time).
// DIS: with D_h; not instantiated for p >= 5 with q >= 5 (registers spill;
// stdg_mesh_set_dissipation refuses such rows)
template <typename T, int A, int QM, bool DIS>
__global__ void __launch_bounds__(LCfg<A>::NT)
    __attribute__((amdgpu_waves_per_eu(!DIS && sizeof(T) == 4 && A <= 5 && QM <= 5 ? 5 : 1)))
    local_time_kernel(LParams<T> P) {
  if (P.skip && *P.skip == 0) return;
  extern __shared__ __align__(16) unsigned char lds_raw[];
  constexpr int TW = kMaxLocalLevels + 1;  // row width of the staged tables
  constexpr int a = A, a2 = A * A, a3 = A * A * A;  // this launch's rows all have a = p + 1 = A
  constexpr int NT = LCfg<A>::NT, nf = 24 * a2;     // face items: [face][F_u, F_v, G_u, G_v][face mode]
  // QM >= q + 1: trial levels of one sub-interval, at most (3, 5 or 7: the
  // register arrays are sized by it)
  const int32_t wk = P.work[blockIdx.x];
  const LTRec* R = P.rec + wk / kMaxSub;  // read through the pointer (no private copy)
  const int jsub = wk % kMaxSub;
  const int e = R->elem;
  const ElemInfo* Ie = P.info + e;
  const int q = Ie->q, ns = Ie->nsub;
  const int nt = q * ns;        // test levels
  const int ncol = nt + 1;      // trial levels (columns of the own tables)
  const int m0 = P.resid ? 0 : 1;
  const int nst = ncol - m0;    // stored trial levels
  // LDS: L_l(0), L_l(1), Dh; the table rows [D, N, C_0..C_5][i][M] of this
  // sub-interval's q test levels; the contracted own fields of one level; the
  // face values; staged: the neighbours' traces contracted for all q levels
  constexpr bool dis = DIS;  // D_h (P.diss set): 6 more table rows, the jumps, own projected traces
  const int nrow = dis ? 14 : 8;
  T* tr = (T*)lds_raw;
  T* dh = tr + 2 * kMaxA;
  T* tb = dh + kMaxA * kMaxA;
  T* xn = tb + nrow * q * TW;
  T* fl = xn + 6 * a3;
  T* jm = fl + nf;                    // D_h jumps, laid out as fl
  T* nbt = jm + (dis ? nf : 0);
  T* opt = nbt + q * nf;              // D_h, staged: own traces against the projected test functions
  // staged: per face and neighbour level, whether any of the q coupling rows
  // uses it (in the face-value area, free until the level loop)
  unsigned char* used = (unsigned char*)fl;
  const bool staged = P.staged != 0;
  const T* xe = P.x + (P.resid ? Ie->trial_off : Ie->unk_off);
  T* ye = P.y + Ie->unk_off;
  const T* le = (P.resid && P.load) ? P.load + Ie->unk_off : nullptr;
  const double* Me = P.metric[e].m;
  const int tid = threadIdx.x;
  for (int t = tid; t < 2 * kMaxA + kMaxA * kMaxA; t += NT) {
    const int u = t - 2 * kMaxA;
    tr[t] = t < kMaxA ? P.tab.tr0[t] : (t < 2 * kMaxA ? P.tab.tr1[t - kMaxA] : P.tab.Dh[u / kMaxA][u % kMaxA]);
  }
  // per face: the neighbour's trial levels (0 on a boundary face) and its
  // coupling table, read once (uniform) before the staging loop
  int nckf[6], coff[6], soff[6];
#pragma unroll
  for (int g = 0; g < 6; ++g) {
    const int k = Ie->nb[g];
    nckf[g] = k >= 0 ? P.info[k].q * P.info[k].nsub + 1 : 0;
    coff[g] = R->c_off[g];
    soff[g] = R->s_off[g];
  }
  const int doff = R->d_off, noff = R->n_off;
  for (int t = tid; t < nrow * q * TW; t += NT) {
    const int r = t / (q * TW), rest = t - r * q * TW, i = rest / TW, M = rest - i * TW;
    const int I = jsub * q + i;
    int off = -1;
    if (r < 2) {
      if (M < ncol) off = (r == 0 ? doff : noff) + I * ncol + M;
    } else {
      const int g = r < 8 ? r - 2 : r - 8;
      int nck = nckf[0], co = coff[0], so = soff[0];
#pragma unroll
      for (int h = 1; h < 6; ++h) {  // selects, no indexed private array
        nck = g == h ? nckf[h] : nck;
        co = g == h ? coff[h] : co;
        so = g == h ? soff[h] : so;
      }
      if (r < 8) {
        if (M < nck) off = co + I * nck + M;
      } else if (nck > 0 && M < ncol) {
        off = so + I * ncol + M;  // D_h's own part (interior faces)
      }
    }
    tb[t] = off >= 0 ? P.bank[off] : T(0);
  }
  // the trial levels of this sub-interval (own tables have no other columns
  // in its rows), and this thread's position and its own levels in registers
  int lev[QM];
#pragma unroll
  for (int m = 0; m < QM; ++m) lev[m] = m <= q ? local_trial_level(q, ns, jsub, m) : 0;
  const int s = tid;
  const bool pos = s < a3;
  const int s0 = s % A, s1 = (s / A) % A, s2 = s / a2;
  auto si = [&](int axis) { return axis == 0 ? s0 : (axis == 1 ? s1 : s2); };  // no private array
  // (a = 9, 768 threads: too few registers per thread; read the levels at each use)
  constexpr bool REG = NT <= 512;
  constexpr int UF = REG ? 6 : 1, UM = REG ? QM : 1;  // unrolled (register operands) or rolled loops
  auto load_own = [&](int fc, int m) {
    return (pos && m <= q && lev[m] >= m0) ? xe[((int64_t)fc * nst + lev[m] - m0) * a3 + s] : T(0);
  };
  T xo[REG ? 6 : 1][REG ? QM : 1];
  if constexpr (REG) {
#pragma unroll
    for (int fc = 0; fc < 6; ++fc)
#pragma unroll
      for (int m = 0; m < QM; ++m) xo[fc][m] = load_own(fc, m);
  }
  auto own_level = [&](int fc, int m) {
    if constexpr (REG) return xo[fc][m]; else return load_own(fc, m);
  };
  __syncthreads();
  if (staged) {
    for (int t = tid; t < (dis ? 12 : 6) * TW; t += NT) {
      const int g = t / TW, M = t - g * TW;  // g >= 6: D_h's own-part rows of face g - 6
      bool any = false;
      for (int i = 0; i < q; ++i) any = any || tb[((2 + g) * q + i) * TW + M] != T(0);
      used[t] = any ? 1 : 0;
    }
    __syncthreads();
    if (dis) {
      for (int t = tid; t < nf; t += NT) {
        for (int i = 0; i < q; ++i) opt[i * nf + t] = T(0);
        const int g = t / (4 * a2);
        if (Ie->nb[g] < 0) continue;
        const int rest = t - g * 4 * a2, ft = rest / a2, jj = rest - ft * a2;
        const int fu = jj % A, fv = jj / A;
        const int alpha = g >> 1, side = g & 1;
        const int ua = alpha == 0 ? 1 : 0, va = alpha == 2 ? 1 : 2;
        const int fld = (ft >> 1) == 0 ? 1 : 0, d = (ft & 1) == 0 ? ua : va;
        const T* xs = xe + (int64_t)(3 * fld + d) * nst * a3 + fu * axis_stride(ua, a) + fv * axis_stride(va, a);
        const int sn = axis_stride(alpha, a);
        const T* S = tb + (8 + g) * q * TW;
        const unsigned char* use = used + (6 + g) * TW;
        for (int M = m0; M < ncol; ++M) {
          if (!use[M]) continue;
          const T* xp = xs + (int64_t)(M - m0) * a3;
          T v = T(0);
#pragma unroll
          for (int l = 0; l < A; ++l) v += tr[side * kMaxA + l] * xp[l * sn];
          for (int i = 0; i < q; ++i) opt[i * nf + t] += S[i * TW + M] * v;
        }
      }
    }
    for (int t = tid; t < nf; t += NT) {
      for (int i = 0; i < q; ++i) nbt[i * nf + t] = T(0);
      const int g = t / (4 * a2), k = Ie->nb[g];
      if (k < 0) continue;
      const int rest = t - g * 4 * a2, ft = rest / a2, jj = rest - ft * a2;
      const int fu = jj % A, fv = jj / A;
      const bool slot_u = (ft & 1) == 0;
      const int fld = (ft >> 1) == 0 ? 1 : 0;
      const uint8_t code = Ie->orient[g];
      const int fo = code & 7, alo = fo >> 1, sdo = fo & 1;
      const int uo = alo == 0 ? 1 : 0, vo = alo == 2 ? 1 : 2;
      const bool swap = (code & kOrientSwap) != 0, flu = (code & kOrientFlipU) != 0, flv = (code & kOrientFlipV) != 0;
      const int mu_ax = swap ? vo : uo, mv_ax = swap ? uo : vo;
      const int cn = slot_u ? mu_ax : mv_ax;
      const ElemInfo* Ik = P.info + k;
      const int ak = Ik->a, ak3 = ak * ak * ak;
      if (fu >= ak || fv >= ak) continue;
      const int nck = Ik->q * Ik->nsub + 1;
      const T* xk = P.x + (P.resid ? Ik->trial_off : Ik->unk_off) + (int64_t)(3 * fld + cn) * (nck - m0) * ak3 +
                    fu * axis_stride(mu_ax, ak) + fv * axis_stride(mv_ax, ak);
      const int snk = axis_stride(alo, ak);
      const bool neg = (slot_u ? flu : flv) ^ (flu && (fu & 1)) ^ (flv && (fv & 1));
      const T* C = tb + (2 + g) * q * TW;
      const unsigned char* use = used + g * TW;
      for (int M = m0; M < nck; ++M) {
        if (!use[M]) continue;
        const T* xp = xk + (int64_t)(M - m0) * ak3;
        T v = T(0);
        for (int l = 0; l < ak; ++l) v += tr[sdo * kMaxA + l] * xp[l * snk];
        if (neg) v = -v;
        for (int i = 0; i < q; ++i) nbt[i * nf + t] += C[i * TW + M] * v;
      }
    }
  }
  for (int i = 0; i < q; ++i) {
    const int I = jsub * q + i;
    const T* tD = tb + i * TW;
    const T* tN = tb + (q + i) * TW;
    __syncthreads();  // staging done, or the previous level's readers of xn and fl are done
    if (pos) {
#pragma unroll UF
      for (int fc = 0; fc < 6; ++fc) {
        T v = T(0);
#pragma unroll UM
        for (int m = 0; m < QM; ++m)
          if (m <= q) v += tN[lev[m]] * own_level(fc, m);
        xn[fc * a3 + s] = v;
      }
    }
    __syncthreads();
    for (int t = tid; t < nf; t += NT) {
      const int g = t / (4 * a2), rest = t - g * 4 * a2, ft = rest / a2, jj = rest - ft * a2;
      const int fu = jj % A, fv = jj / A;
      const int alpha = g >> 1, side = g & 1;
      const int ua = alpha == 0 ? 1 : 0, va = alpha == 2 ? 1 : 2;
      const int which = ft >> 1;           // 0: F (H traces), 1: G (E traces)
      const bool slot_u = (ft & 1) == 0;   // tangential component along u (else v)
      const int fld = which == 0 ? 1 : 0;  // field of the traces
      const int d = slot_u ? ua : va;
      // own trace of the contracted field
      const T* own = xn + (3 * fld + d) * a3 + fu * axis_stride(ua, a) + fv * axis_stride(va, a);
      const int sn = axis_stride(alpha, a);
      T ts = T(0);
#pragma unroll
      for (int l = 0; l < A; ++l) ts += tr[side * kMaxA + l] * own[l * sn];
      const int k = Ie->nb[g];
      T val;
      if (k < 0) {
        val = which == 0 ? ts : -ts;
      } else {
        T tn = T(0);
        if (staged) {
          tn = nbt[i * nf + t];
        } else {
          const uint8_t code = Ie->orient[g];
          const int fo = code & 7, alo = fo >> 1, sdo = fo & 1;
          const int uo = alo == 0 ? 1 : 0, vo = alo == 2 ? 1 : 2;
          const bool swap = (code & kOrientSwap) != 0, flu = (code & kOrientFlipU) != 0,
                     flv = (code & kOrientFlipV) != 0;
          const int mu_ax = swap ? vo : uo, mv_ax = swap ? uo : vo;  // the neighbour's axes matched with our u, v
          const int cn = slot_u ? mu_ax : mv_ax;
          const ElemInfo* Ik = P.info + k;
          const int ak = Ik->a, ak3 = ak * ak * ak;
          if (fu < ak && fv < ak) {
            const int nck = Ik->q * Ik->nsub + 1;  // the neighbour's trial levels
            const T* C = tb + ((2 + g) * q + i) * TW;
            const T* xk = P.x + (P.resid ? Ik->trial_off : Ik->unk_off) + (int64_t)(3 * fld + cn) * (nck - m0) * ak3 +
                          fu * axis_stride(mu_ax, ak) + fv * axis_stride(mv_ax, ak);
            const int snk = axis_stride(alo, ak);
            for (int M = m0; M < nck; ++M) {
              const T w = C[M];
              if (w == T(0)) continue;
              const T* xp = xk + (int64_t)(M - m0) * ak3;
              T v = T(0);
              for (int l = 0; l < ak; ++l) v += tr[sdo * kMaxA + l] * xp[l * snk];
              tn += w * v;
            }
            // covariant component along a reversed axis, and odd modes along reversed axes
            const bool neg = (slot_u ? flu : flv) ^ (flu && (fu & 1)) ^ (flv && (fv & 1));
            if (neg) tn = -tn;
          }
        }
        val = T(0.5) * ((which == 0 ? ts : -ts) + tn);
        if (dis) {
          // D_h jump: own trace against the projected test function minus the neighbour's
          T own_p = T(0);
          if (staged) {
            own_p = opt[i * nf + t];
          } else {
            const T* S = tb + ((8 + g) * q + i) * TW;
            const T* xs = xe + (int64_t)(3 * fld + d) * nst * a3 + fu * axis_stride(ua, a) + fv * axis_stride(va, a);
            for (int M = m0; M < ncol; ++M) {
              const T w = S[M];
              if (w == T(0)) continue;
              const T* xp = xs + (int64_t)(M - m0) * a3;
              T v = T(0);
#pragma unroll
              for (int l = 0; l < A; ++l) v += tr[side * kMaxA + l] * xp[l * sn];
              own_p += w * v;
            }
          }
          jm[t] = own_p - tn;
        }
      }
      if (dis && k < 0) jm[t] = ts;  // PEC face: the own trace, not projected
      fl[t] = val;
    }
    __syncthreads();
    if (!pos) continue;
#pragma unroll UF
    for (int fc = 0; fc < 6; ++fc) {
      const int f = fc / 3, c = fc - 3 * f;
      // mass: the metric block of field f applied to the D-contracted levels
      T xd[3];
#pragma unroll
      for (int dd = 0; dd < 3; ++dd) {
        T v = T(0);
#pragma unroll UM
        for (int m = 0; m < QM; ++m)
          if (m <= q) v += tD[lev[m]] * own_level(3 * f + dd, m);
        xd[dd] = v;
      }
      const double* Mf = Me + 6 * f;
      const T mass = (T)Mf[c == 0 ? 0 : (c == 1 ? 3 : 4)] * xd[0] + (T)Mf[c == 0 ? 3 : (c == 1 ? 1 : 5)] * xd[1] +
                     (T)Mf[c == 0 ? 4 : (c == 1 ? 5 : 2)] * xd[2];
      // curl of the other field's contracted level
      const int c1 = (c + 1) % 3, c2 = (c + 2) % 3;
      const T* src = xn + (f == 0 ? 3 : 0) * a3;
      const int st1 = axis_stride(c1, a), st2 = axis_stride(c2, a);
      const int j1 = si(c1), j2 = si(c2);
      const int b1 = s - j1 * st1, b2 = s - j2 * st2;
      T curl = T(0);
#pragma unroll
      for (int n = 0; n < A; ++n) {
        const T d1 = f == 0 ? dh[n * kMaxA + j1] : dh[j1 * kMaxA + n];
        const T d2 = f == 0 ? dh[n * kMaxA + j2] : dh[j2 * kMaxA + n];
        curl += d1 * src[c2 * a3 + b1 + n * st1] - d2 * src[c1 * a3 + b2 + n * st2];
      }
      // lifts of the face values
      T lift = T(0);
#pragma unroll
      for (int alpha = 0; alpha < 3; ++alpha) {
        if (alpha == c) continue;
        const int d = 3 - c - alpha;
        const int ua = alpha == 0 ? 1 : 0, va = alpha == 2 ? 1 : 2;
        const int slot = d == ua ? 0 : 1;
        const T epsv = alpha == (c + 2) % 3 ? T(1) : T(-1);  // eps(c, d, alpha)
        const int jj = si(ua) + a * si(va);
        const int l = si(alpha);
        const int ft = (f == 0 ? 0 : 2) + slot;  // E rows lift F, H rows G
#pragma unroll
        for (int side = 0; side < 2; ++side) {
          const T sl = side ? tr[kMaxA + l] : -tr[l];  // sigma L_l(side)
          lift += (f == 0 ? epsv : -epsv) * sl * fl[((2 * alpha + side) * 4 + ft) * a2 + jj];
        }
      }
      // D_h: alpha_f L_{s_alpha}(side) (K J)_c over the four faces whose normal
      // is not c, jumps of field f itself (alpha_H = 0 on PEC faces)
      T dl = T(0);
      if (dis) {
        const T* dc = P.diss + (int64_t)Mesh::kDissWords * e;
#pragma unroll
        for (int alpha = 0; alpha < 3; ++alpha) {
          if (alpha == c) continue;
          const int ua = alpha == 0 ? 1 : 0, va = alpha == 2 ? 1 : 2;
          const int slot_c = c == ua ? 0 : 1;
          const T kcc = dc[12 + 3 * alpha + (c == (alpha + 1) % 3 ? 0 : 1)], kco = dc[12 + 3 * alpha + 2];
          const int jj = si(ua) + a * si(va);
          const int l = si(alpha);
          const int ftb = f == 0 ? 2 : 0;  // E rows: E jumps; H rows: H jumps
#pragma unroll
          for (int side = 0; side < 2; ++side) {
            const int g = 2 * alpha + side;
            const T* J = jm + (g * 4 + ftb) * a2 + jj;
            dl += dc[6 * f + g] * tr[side * kMaxA + l] * (kcc * J[slot_c * a2] + kco * J[(1 - slot_c) * a2]);
          }
        }
      }
      const int64_t o = ((int64_t)fc * nt + I) * a3 + s;
      T out = mass + P.dt * (curl + lift + dl);
      if (le) out -= le[o];
      ye[o] = out;
    }
  }
}

// P^{-1} of meshes with local time steps (every element; P = D_u (x) mass per
// element): the 3x3 inverse metric per spatial mode and level as on other
// meshes, and with n > 1 sub-intervals P's time factor is not the identity:
// row (j, 0) is l_1 - l_0 of sub-interval j, so the value at the right end of
// sub-interval j (unknown level (j + 1) q, or 0 for the slab end) is the sum
// of rows (0, 0) .. (j, 0), and rows (j, i > 0) give the interior levels
// j q + i as they are.  z = P^{-1} x on the unknowns layout.
template <typename T>
__global__ void precond_scale_local_kernel(const ElemInfo* info, const ElemMetric* metric, int64_t ne, const T* x,
                                           T* z, const int* skip) {
  if (skip && *skip == 0) return;
  const int64_t e = blockIdx.x;
  if (e >= ne) return;
  const ElemInfo I = info[e];
  const int a3 = I.a * I.a * I.a;
  const double* mm = metric[e].m;
  const int q = I.q, ns = I.nsub, nl = q * ns;
  for (int idx = threadIdx.x; idx < 2 * a3; idx += blockDim.x) {
    const int f = idx / a3, s = idx - f * a3;
    const double* Mi = mm + 12 + 6 * f;
    const T* xb = x + I.unk_off + (int64_t)3 * f * nl * a3 + s;
    T* zb = z + I.unk_off + (int64_t)3 * f * nl * a3 + s;
    double cum0 = 0.0, cum1 = 0.0, cum2 = 0.0;
    for (int L = 0; L < nl; ++L) {
      const double v0 = xb[(int64_t)L * a3], v1 = xb[(int64_t)(nl + L) * a3], v2 = xb[(int64_t)(2 * nl + L) * a3];
      const double w0 = Mi[0] * v0 + Mi[3] * v1 + Mi[4] * v2;
      const double w1 = Mi[3] * v0 + Mi[1] * v1 + Mi[5] * v2;
      const double w2 = Mi[4] * v0 + Mi[5] * v1 + Mi[2] * v2;
      const bool node = ns > 1 && L % q == 0;  // one sub-interval: P's time factor is the identity
      int o = L;
      if (node) {
        cum0 += w0;
        cum1 += w1;
        cum2 += w2;
        o = L + q < nl ? L + q : 0;
      }
      zb[(int64_t)o * a3] = (T)(node ? cum0 : w0);
      zb[(int64_t)(nl + o) * a3] = (T)(node ? cum1 : w1);
      zb[(int64_t)(2 * nl + o) * a3] = (T)(node ? cum2 : w2);
    }
  }
}

}  // namespace

int launch_precond_scale_local(const Mesh* m, int prec, const void* x, void* z, hipStream_t s, const int* skip) {
  const dim3 grid((unsigned)m->ne), block(256);
  if (prec == STDG_FP64)
    hipLaunchKernelGGL(precond_scale_local_kernel<double>, grid, block, 0, s, m->d_info, m->d_metric, m->ne,
                       (const double*)x, (double*)z, skip);
  else
    hipLaunchKernelGGL(precond_scale_local_kernel<float>, grid, block, 0, s, m->d_info, m->d_metric, m->ne,
                       (const float*)x, (float*)z, skip);
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "precond_scale_local launch");
}

template <typename T>
int launch_local_time(const Mesh* m, double dt, int mode, const T* x, const T* load, T* y, hipStream_t s,
                      const int* skip) {
  if (m->lt.empty()) return STDG_OK;
  if (!m->d_lt || !m->d_lt_work) return fail(STDG_E_ARG, "local time steps: device records missing");
  if (mode != STDG_OPERATOR && mode != STDG_RESIDUAL)
    return fail(STDG_E_ARG, "local time steps: preconditioned applies take the P^{-1} pre-pass");
  LParams<T> P;
  P.info = m->d_info;
  P.metric = m->d_metric;
  P.rec = m->d_lt;
  if constexpr (sizeof(T) == 8) P.diss = m->d_diss; else P.diss = m->d_diss32;
  P.bank = (const T*)(sizeof(T) == 8 ? m->d_ltb64 : m->d_ltb32);
  P.x = x;
  P.load = load;
  P.y = y;
  P.skip = skip;
  P.dt = (T)dt;
  P.resid = mode == STDG_RESIDUAL ? 1 : 0;
  if constexpr (sizeof(T) == 8) fill_tables_f64(&P.tab); else fill_tables_f32(&P.tab);
  // one launch per a (rows grouped by a on upload), dynamic LDS and the
  // register arrays sized for the largest q among its rows
  using K = void (*)(LParams<T>);
#define STDG_LT_ROW(AA) {local_time_kernel<T, AA, 3, false>, local_time_kernel<T, AA, 5, false>, \
                         local_time_kernel<T, AA, 7, false>}
  static const K kern[kMaxA + 1][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr},
                                       STDG_LT_ROW(2), STDG_LT_ROW(3), STDG_LT_ROW(4), STDG_LT_ROW(5),
                                       STDG_LT_ROW(6), STDG_LT_ROW(7), STDG_LT_ROW(8), STDG_LT_ROW(9)};
#undef STDG_LT_ROW
#define STDG_LT_ROW(AA) {local_time_kernel<T, AA, 3, true>, local_time_kernel<T, AA, 5, true>, \
                         AA <= kMaxDissLocalA7 ? local_time_kernel<T, AA <= kMaxDissLocalA7 ? AA : 2, 7, true> : nullptr}
  static const K kern_d[kMaxA + 1][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr},
                                         STDG_LT_ROW(2), STDG_LT_ROW(3), STDG_LT_ROW(4), STDG_LT_ROW(5),
                                         STDG_LT_ROW(6), STDG_LT_ROW(7), STDG_LT_ROW(8), STDG_LT_ROW(9)};
#undef STDG_LT_ROW
  static_assert(kMaxQ + 1 <= 7, "local-time kernels hold at most 7 trial levels per sub-interval");
  static const int nthreads[kMaxA + 1] = {0, 0, LCfg<2>::NT, LCfg<3>::NT, LCfg<4>::NT, LCfg<5>::NT,
                                          LCfg<6>::NT, LCfg<7>::NT, LCfg<8>::NT, LCfg<9>::NT};
  for (int a = 2; a <= kMaxA; ++a) {
    const int64_t b0 = m->lt_a_off[a], b1 = m->lt_a_off[a + 1];
    if (b1 == b0) continue;
    const int qmax = m->lt_a_qmax[a];
    const size_t a2 = (size_t)a * a, a3 = a2 * a;
    const bool dis = P.diss != nullptr;
    const size_t base = 2 * kMaxA + kMaxA * kMaxA + (size_t)(dis ? 14 : 8) * qmax * (kMaxLocalLevels + 1) + 6 * a3 +
                        (dis ? 48 : 24) * a2;
    const size_t full = base + (size_t)(dis ? 2 : 1) * qmax * 24 * a2;
    constexpr size_t kLdsCap = 65536;
    P.staged = full * sizeof(T) <= kLdsCap ? 1 : 0;
    P.work = m->d_lt_work + b0;
    const size_t lds = (P.staged ? full : base) * sizeof(T);
    const int qb = qmax <= 2 ? 0 : (qmax <= 4 ? 1 : 2);
    const K k = dis ? kern_d[a][qb] : kern[a][qb];
    if (!k) return fail(STDG_E_UNSUPPORTED, "local time steps with D_h: no kernel for p = " + std::to_string(a - 1));
    hipLaunchKernelGGL(k, dim3((unsigned)(b1 - b0)), dim3((unsigned)nthreads[a]), lds, s, P);
  }
  hipError_t e = hipGetLastError();
  return e == hipSuccess ? STDG_OK : hip_fail(e, "local-time kernel");
}

template int launch_local_time<float>(const Mesh*, double, int, const float*, const float*, float*, hipStream_t,
                                      const int*);
template int launch_local_time<double>(const Mesh*, double, int, const double*, const double*, double*, hipStream_t,
                                       const int*);

}  // namespace stdg
