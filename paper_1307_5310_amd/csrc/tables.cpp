// 1D factor tables of the tensor-product bases (Section 5.1-5.2), from closed
// forms of the Legendre identities on [0, 1]:
//   orthonormal Legendre L_j(xi) = sqrt(2j+1) P_j(2 xi - 1);
//   l_0 = 1 - xi, l_1 = xi, l_m = int_0^xi L_{m-1}
//       = (L_m / sqrt(2m+1) - L_{m-2} / sqrt(2m-3)) / (2 sqrt(2m-1))   (m >= 2);
//   N[i][m] = int L_i l_m  (curl and flux factor in time, carries dt);
//   int L_i l_m' = delta_{m,i+1} - delta_{i0} delta_{m0}  (the mass factor is a
//       shift, used directly by the kernels, no table);
//   Dh[n][j] = int L_n L_j' = 2 sqrt((2n+1)(2j+1)) for n < j, j - n odd;
//   traces L_j(0) = (-1)^j sqrt(2j+1), L_j(1) = sqrt(2j+1).
#include <cmath>
#include <cstring>

#include "internal.h"

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

}  // namespace stdg
