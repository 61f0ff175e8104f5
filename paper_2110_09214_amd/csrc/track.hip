// Transport step (in progress).
#include "obem_internal.hpp"

extern "C" obem_status track_step(obem_ctx *ctx, obem_meshh *, obem_particles *, const obem_gas *,
                                  const obem_step_params *, int64_t *, double *, obem_step_stats *) {
  return obem::fail(ctx, OBEM_EINVAL, "track_step: not available in this build");
}
