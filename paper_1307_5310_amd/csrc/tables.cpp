// 1D factor tables of the tensor-product bases (Section 5.1-5.2), from closed
// forms of the Legendre identities on [0, 1]:
//   orthonormal Legendre L_j(xi) = sqrt(2j+1) P_j(2 xi - 1);
//   l_0 = 1 - xi, l_1 = xi, l_m = int_0^xi L_{m-1}
//       = (L_m / sqrt(2m+1) - L_{m-2} / sqrt(2m-3)) / (2 sqrt(2m-1))   (m >= 2);
//   N[i][m] = int L_i l_m  (curl and flux factor in time, carries dt);
//   int L_i l_m' = delta_{m,i+1} - delta_{i0} delta_{m0}  (the mass factor is a
//       shift, used directly by the kernels, no table);
//   Dh[n][j] = int L_n L_j' = 2 sqrt((2n+1)(2j+1)) for n < j, j - n odd;
//   traces L_j(0) = (-1)^j sqrt(2j+1), L_j(1) = sqrt(2j+1);
// and the Gauss-Legendre mass rule of trilinear elements (n = p + 2 points).
#include <algorithm>
#include <cmath>
#include <cstring>

#include "internal.h"

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

namespace stdg {

static void fill_double(Tables<double>* t) {
  std::memset(t, 0, sizeof(*t));
  for (int i = 0; i < kMaxQ; ++i) {
    for (int m = 0; m <= kMaxQ; ++m) {
      double v = 0.0;
      if (m == 0) {
        if (i == 0) v = 0.5;
        if (i == 1) v = -0.5 / std::sqrt(3.0);
      } else if (m == 1) {
        if (i == 0) v = 0.5;
        if (i == 1) v = 0.5 / std::sqrt(3.0);
      } else {
        if (i == m) v = 1.0 / (2.0 * std::sqrt((2.0 * m - 1.0) * (2.0 * m + 1.0)));
        if (i == m - 2) v = -1.0 / (2.0 * std::sqrt((2.0 * m - 1.0) * (2.0 * m - 3.0)));
      }
      t->N[i][m] = v;
    }
  }
  for (int n = 0; n < kMaxA; ++n)
    for (int j = 0; j < kMaxA; ++j)
      t->Dh[n][j] = (n < j && ((j - n) & 1)) ? 2.0 * std::sqrt((2.0 * n + 1.0) * (2.0 * j + 1.0)) : 0.0;
  for (int j = 0; j < kMaxA; ++j) {
    t->tr1[j] = std::sqrt(2.0 * j + 1.0);
    t->tr0[j] = (j & 1) ? -t->tr1[j] : t->tr1[j];
  }
}

void fill_tables_f64(Tables<double>* t) { fill_double(t); }

void fill_tables_f32(Tables<float>* t) {
  Tables<double> d;
  fill_double(&d);
  for (int i = 0; i < kMaxQ; ++i)
    for (int m = 0; m <= kMaxQ; ++m) t->N[i][m] = (float)d.N[i][m];
  for (int n = 0; n < kMaxA; ++n)
    for (int j = 0; j < kMaxA; ++j) t->Dh[n][j] = (float)d.Dh[n][j];
  for (int j = 0; j < kMaxA; ++j) {
    t->tr0[j] = (float)d.tr0[j];
    t->tr1[j] = (float)d.tr1[j];
  }
}

void gauss_rule01(int n, double* x, double* w) {
  // roots of P_n on [-1, 1] from the Chebyshev-like initial guesses, refined
  // by Newton's method; mapped to [0, 1] with weights halved
  for (int i = 0; i < n; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pm = n == 1 ? 1.0 : p0;
      dp = n * (z * p1 - pm) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pm = n == 1 ? 1.0 : p0;
      dp = n * (z * p1 - pm) / (z * z - 1.0);
    }
    x[i] = 0.5 * (1.0 - z);
    w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
  }
}

static double legendre01(int j, double xi) {
  const double u = 2.0 * xi - 1.0;
  double p0 = 1.0, p1 = u;
  if (j == 0) return 1.0;
  for (int k = 1; k < j; ++k) {
    const double p2 = ((2.0 * k + 1.0) * u * p1 - k * p0) / (k + 1.0);
    p0 = p1;
    p1 = p2;
  }
  return std::sqrt(2.0 * j + 1.0) * p1;
}

void fill_qtables_f64(int a, QTables<double>* t) {
  std::memset(t, 0, sizeof(*t));
  const int n = a + 1;
  double x[kMaxA + 1], w[kMaxA + 1];
  gauss_rule01(n, x, w);
  for (int g = 0; g < n; ++g) {
    t->x[g] = x[g];
    for (int j = 0; j < a; ++j) t->B[g * a + j] = std::sqrt(w[g]) * legendre01(j, x[g]);
  }
}

void fill_qtables_f32(int a, QTables<float>* t) {
  QTables<double> d;
  fill_qtables_f64(a, &d);
  for (int i = 0; i < (kMaxA + 1) * kMaxA; ++i) t->B[i] = (float)d.B[i];
  for (int i = 0; i <= kMaxA; ++i) t->x[i] = (float)d.x[i];
}

void fill_half_tables_f64(double* S) {
  // exact: the integrand has degree < 2 kMaxA, the rule 2 kMaxA points
  const int n = 2 * kMaxA;
  double x[2 * kMaxA], w[2 * kMaxA];
  gauss_rule01(n, x, w);
  for (int h = 0; h < 2; ++h)
    for (int k = 0; k < kMaxA; ++k)
      for (int m = 0; m < kMaxA; ++m) {
        double v = 0.0;
        for (int g = 0; g < n; ++g) v += w[g] * legendre01(k, x[g]) * legendre01(m, 0.5 * (x[g] + h));
        S[(h * kMaxA + k) * kMaxA + m] = v;
      }
}

void fill_face_rule_f64(int n, FaceRule<double>* r) {
  std::memset(r, 0, sizeof(*r));
  if (n < 1 || n > kMaxFaceQ) return;
  double x[kMaxFaceQ], w[kMaxFaceQ];
  gauss_rule01(n, x, w);
  for (int k = 0; k < n; ++k) {
    r->x[k] = x[k];
    r->w[k] = w[k];
    for (int j = 0; j < kMaxA; ++j) r->L[k * kMaxA + j] = legendre01(j, x[k]);
  }
}

void fill_face_rule_f32(int n, FaceRule<float>* r) {
  FaceRule<double> d;
  fill_face_rule_f64(n, &d);
  for (int k = 0; k < kMaxFaceQ; ++k) {
    r->x[k] = (float)d.x[k];
    r->w[k] = (float)d.w[k];
  }
  for (int i = 0; i < kMaxFaceQ * kMaxA; ++i) r->L[i] = (float)d.L[i];
}

// Local time steps (Section 2.2): tables of a slab interval bisected into n
// equal sub-intervals, in the unit slab coordinate s, with the flattened trial
// levels of local_trial_level.  Own terms: on sub-interval j the mass factor
// is the shift delta_{m,i+1} - delta_{i0} delta_{m0} and the curl and flux
// factor N[i][m] / n (the sub-interval has length 1 / n).
static double ilegendre01(int m, double xi) {
  if (m == 0) return 1.0 - xi;
  if (m == 1) return xi;
  return (legendre01(m, xi) / std::sqrt(2.0 * m + 1.0) - legendre01(m - 2, xi) / std::sqrt(2.0 * m - 3.0)) /
         (2.0 * std::sqrt(2.0 * m - 1.0));
}

int local_time_tables(int q, int n, std::vector<double>* bank, int32_t* d_off, int32_t* n_off) {
  Tables<double> t;
  fill_double(&t);
  const int rows = n * q, cols = 1 + n * q;
  *d_off = (int32_t)bank->size();
  bank->resize(bank->size() + 2 * (size_t)rows * cols, 0.0);
  *n_off = *d_off + rows * cols;
  double* D = bank->data() + *d_off;
  double* N = bank->data() + *n_off;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < q; ++i) {
      const int I = j * q + i;
      D[I * cols + local_trial_level(q, n, j, i + 1)] += 1.0;
      if (i == 0) D[I * cols + local_trial_level(q, n, j, 0)] -= 1.0;
      for (int m = 0; m <= q; ++m) N[I * cols + local_trial_level(q, n, j, m)] += t.N[i][m] / n;
    }
  return *d_off;
}

// Coupling of S_h across a face between partitions of n and nk sub-intervals
// (powers of two, so they nest): C[(j, i)][M'] = int_0^1 (pi L_i^(j)) phi'_M'
// ds, pi the L2 projection onto the common temporal test space, piecewise
// P_{r-1} (r = min(q, qk)) on the coarser partition.
//   n <= nk: L_i^(j) already lies on the coarser partition, so pi keeps it for
//     i < r and removes it otherwise; the integral runs over the nk / n
//     sub-intervals of the neighbour inside sub-interval j (Gauss rule).
//   n > nk: sub-interval j lies in the neighbour's sub-interval c; pi L_i^(j)
//     = sum_{rho < r} beta_rho L_rho^(c) with beta_rho = nk int_{I_j} L_i^(j)
//     L_rho^(c), and int_{I_c} L_rho^(c) l_m'^(c) = N[rho][m'] / nk.
int local_coupling_table(int q, int n, int qk, int nk, std::vector<double>* bank) {
  Tables<double> t;
  fill_double(&t);
  const int rows = n * q, cols = 1 + nk * qk, r = std::min(q, qk);
  const int off = (int)bank->size();
  bank->resize(bank->size() + (size_t)rows * cols, 0.0);
  double* C = bank->data() + off;
  const int ng = q + qk + 2;
  double xg[32], wg[32];
  gauss_rule01(ng, xg, wg);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < r; ++i) {
      double* row = C + (size_t)(j * q + i) * cols;
      if (n <= nk) {
        const int ratio = nk / n;
        for (int jr = 0; jr < ratio; ++jr) {
          const int jk = j * ratio + jr;
          for (int m = 0; m <= qk; ++m) {
            // s = (jk + xi) / nk, n s - j = (jr + xi) / ratio
            double v = 0.0;
            for (int g = 0; g < ng; ++g) v += wg[g] * legendre01(i, (jr + xg[g]) / ratio) * ilegendre01(m, xg[g]);
            row[local_trial_level(qk, nk, jk, m)] += v / nk;
          }
        }
      } else {
        const int ratio = n / nk, c = j / ratio, jr = j - c * ratio;
        for (int rho = 0; rho < r; ++rho) {
          // beta = nk int_{I_j} L_i(n s - j) L_rho(nk s - c) ds, s = (j + xi) / n
          double beta = 0.0;
          for (int g = 0; g < ng; ++g) beta += wg[g] * legendre01(i, xg[g]) * legendre01(rho, (jr + xg[g]) / ratio);
          beta *= (double)nk / n;
          for (int m = 0; m <= qk; ++m) row[local_trial_level(qk, nk, c, m)] += beta * t.N[rho][m] / nk;
        }
      }
    }
  return off;
}

// D_h's own part with local time steps: T[(j, i)][M] = int_0^1 (pi L_i^(j)) phi_M ds
// for the element's own trial levels (q, n), pi the projection onto piecewise
// P_{r-1} on npj <= n equal sub-intervals (the common temporal test space of
// a face's pair).  npj == n: pi keeps L_i^(j) for i < r.  npj < n: sub-interval
// j lies in the coarse interval c; pi L_i^(j) = sum_{rho < r} beta_rho L_rho^(c),
// beta_rho = npj int_{I_j} L_i^(j) L_rho^(c), integrated against the own trial
// functions of every sub-interval inside I_c (Gauss rule).
int local_projected_table(int q, int n, int r, int npj, std::vector<double>* bank) {
  Tables<double> t;
  fill_double(&t);
  const int rows = n * q, cols = 1 + n * q;
  const int off = (int)bank->size();
  bank->resize(bank->size() + (size_t)rows * cols, 0.0);
  double* T = bank->data() + off;
  const int ng = 2 * q + 2;
  double xg[32], wg[32];
  gauss_rule01(ng, xg, wg);
  const int ratio = n / npj;
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < q; ++i) {
      double* row = T + (size_t)(j * q + i) * cols;
      if (npj == n) {
        if (i >= r) continue;
        for (int m = 0; m <= q; ++m) row[local_trial_level(q, n, j, m)] += t.N[i][m] / n;
        continue;
      }
      const int c = j / ratio, jr = j - c * ratio;
      for (int rho = 0; rho < r; ++rho) {
        double beta = 0.0;  // npj int_{I_j} L_i(n s - j) L_rho(npj s - c) ds, s = (j + xi) / n
        for (int g = 0; g < ng; ++g) beta += wg[g] * legendre01(i, xg[g]) * legendre01(rho, (jr + xg[g]) / ratio);
        beta *= (double)npj / n;
        for (int jj = 0; jj < ratio; ++jj) {
          const int jt = c * ratio + jj;  // own sub-interval inside I_c
          for (int m = 0; m <= q; ++m) {
            // int_{I_jt} L_rho(npj s - c) l_m(n s - jt) ds, s = (jt + xi) / n, npj s - c = (jj + xi) / ratio
            double v = 0.0;
            for (int g = 0; g < ng; ++g) v += wg[g] * legendre01(rho, (jj + xg[g]) / ratio) * ilegendre01(m, xg[g]);
            row[local_trial_level(q, n, jt, m)] += beta * v / n;
          }
        }
      }
    }
  return off;
}

}  // namespace stdg
