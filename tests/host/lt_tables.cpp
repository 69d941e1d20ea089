// Prints the library's local-time tables (own D and N, and the S_h coupling)
// for the (q, n, q', n') given on the command line, one table per line:
//   D <q> <n> v...   N <q> <n> v...   C <q> <n> <q'> <n'> v...   P <q> <n> <r> <n_p> v...
// (row-major, n q rows).  Host code only; no device.
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "../../paper_1307_5310_amd/csrc/internal.h"

namespace stdg {
std::string g_err;
void set_error(const std::string& m) { g_err = m; }
int fail(int status, const std::string& m) { g_err = m; return status; }
int hip_fail(hipError_t, const char* what) { g_err = what; return STDG_E_DEVICE; }
}  // namespace stdg

int main(int argc, char** argv) {
  if (argc != 5) return 2;
  const int q = std::atoi(argv[1]), n = std::atoi(argv[2]), qk = std::atoi(argv[3]), nk = std::atoi(argv[4]);
  std::vector<double> bank;
  int32_t d_off = 0, n_off = 0;
  stdg::local_time_tables(q, n, &bank, &d_off, &n_off);
  const int c_off = stdg::local_coupling_table(q, n, qk, nk, &bank);
  const int rows = n * q, cols = 1 + n * q, ccols = 1 + nk * qk;
  std::printf("D %d %d", q, n);
  for (int i = 0; i < rows * cols; ++i) std::printf(" %.17g", bank[d_off + i]);
  std::printf("\nN %d %d", q, n);
  for (int i = 0; i < rows * cols; ++i) std::printf(" %.17g", bank[n_off + i]);
  std::printf("\nC %d %d %d %d", q, n, qk, nk);
  for (int i = 0; i < rows * ccols; ++i) std::printf(" %.17g", bank[c_off + i]);
  std::printf("\n");
  // D_h's own part: the own trial against the test function projected onto
  // the common space of (q, n) and (q', n')
  const int r = q < qk ? q : qk, npj = n < nk ? n : nk;
  const int p_off = stdg::local_projected_table(q, n, r, npj, &bank);
  std::printf("P %d %d %d %d", q, n, r, npj);
  for (int i = 0; i < rows * cols; ++i) std::printf(" %.17g", bank[p_off + i]);
  std::printf("\n");
  return 0;
}
