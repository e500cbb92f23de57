// Matrix-free CG and FP32 iterative-refinement solver (placeholder).
#include "internal.h"

extern "C" dg_status dg_solve(const dg_mesh*, int, const double*, double*, const void*, const dg_solve_params*,
                              dg_solve_info*, void*) {
  dg_set_error("dg_solve is not built yet");
  return DG_ERR_UNSUPPORTED;
}
