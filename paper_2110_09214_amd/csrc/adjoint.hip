// Adjoint of the field evaluation (in progress).
#include "obem_internal.hpp"

extern "C" obem_status field_eval_backward(obem_ctx *ctx, const obem_meshh *, const double *, int64_t,
                                           const double *, const double *, const double *, const double *, int64_t,
                                           const double *, const double *, const double *, double, obem_precision,
                                           unsigned, const double *, const double *, const double *, double *,
                                           double *, double *, double *, double *, double *, double *) {
  return obem::fail(ctx, OBEM_EINVAL, "field_eval_backward: not available in this build");
}
