// Slab solve (placeholder until the GMRES solver lands).
#include "internal.h"

using namespace stdg;

extern "C" int stdg_slab_solve(const stdg_mesh* mesh, double t0, double dt, const double* load_dev,
                               const stdg_solve_opts* opts, double* state_dev, double* slab_U_dev,
                               stdg_solve_info* info, void* stream) {
  (void)mesh; (void)t0; (void)dt; (void)load_dev; (void)opts; (void)state_dev; (void)slab_U_dev; (void)info;
  (void)stream;
  return fail(STDG_E_UNSUPPORTED, "stdg_slab_solve: not available in this build");
}
