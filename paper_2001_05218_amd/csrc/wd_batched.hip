// Batched multi-RHS solver (placeholder until the persistent kernel lands).
#include <hip/hip_runtime.h>

#include "../../include/wilson.h"
#include "wd_internal.hpp"

namespace wd {
size_t batched_workspace_bytes(const Geom& g, int nrhs, int hist_len) {
  (void)g; (void)nrhs; (void)hist_len;
  return 256;
}
}  // namespace wd

extern "C" int cg_solve_batched(const wd_lattice*, double, const void*, int32_t, const void*, void*,
                                const wd_cg_params*, wd_cg_result*, void*, size_t, void*) {
  return WD_ERR_INVALID;
}
