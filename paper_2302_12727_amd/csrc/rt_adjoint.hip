// Adjoint of one RT step (placeholder until the VJP kernels land).
#include "rt_internal.h"

rt_status rt_adjoint_impl(rt_ctx *ctx, const void *, const double *, const double *,
                          const void *, const uint8_t *, const void *, void *, double *) {
    return rt_fail(ctx, RT_ESTATE, "adjoint not available");
}
