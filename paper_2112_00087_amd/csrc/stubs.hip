#include "ops.h"
int schwarz_solve(hz_ctx, const hz_solve_opts&, const z_t*, z_t*, hz_solve_info*) {
  return hz_fail(HZ_ERR_INVALID, "Schwarz method not available");
}
