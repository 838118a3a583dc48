// Ivanova effective surfaces (Part II eq:IvanovaAij): the per-particle sums
// of kernel gradients they need, and the switch between the surface kinds.
// The pair formula itself is in rt_pair.h (pair_geometry_ivanova64).
#include "rt_internal.h"

using namespace gearrt;

namespace {

// g_i = sum_k grad W_k(x_i) over the gather neighbours of i (r_ik < H_i),
// grad W_k(x_i) = (sigma / H_i^4) w'(r_ik / H_i) (x_i - x_k) / r_ik, written
// to ivan[i][0..2] (ivan[i][3] = 0) and to slots 13-15 of the geometry record,
// where the FP64 transports find a neighbour's with the rest of its record.
__global__ __launch_bounds__(kBlock) void k_ivanova_sums(
    int64_t n, double *__restrict__ geo, const double *__restrict__ xs,
    const int32_t *__restrict__ nbr, const int64_t *__restrict__ wave_base,
    const int32_t *__restrict__ n_gath, double box, double *__restrict__ ivan) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ibox = 1.0 / box;
    const double iH = geo[(int64_t)kRec * i + R_IH];
    const double f0 = kSigma3 * iH * iH * iH * iH;
    const double px = xs[3 * i], py = xs[3 * i + 1], pz = xs[3 * i + 2];
    const int64_t base = wave_base[i >> 6] + (i & 63);
    const int32_t ng = n_gath[i];
    double gx = 0.0, gy = 0.0, gz = 0.0;
    for (int32_t k = 0; k < ng; ++k) {
        const int64_t j = nbr[base + 64 * (int64_t)k];
        const double sx = min_image(xs[3 * j] - px, box, ibox);
        const double sy = min_image(xs[3 * j + 1] - py, box, ibox);
        const double sz = min_image(xs[3 * j + 2] - pz, box, ibox);
        const double r2 = sx * sx + sy * sy + sz * sz;
        if (!(r2 > 0.0)) continue;
        const double ir = rsq64(r2);
        const double f = -f0 * kern_dw(r2 * ir * iH) * ir;   // times s = x_j - x_i
        gx += f * sx;
        gy += f * sy;
        gz += f * sz;
    }
    double *o = ivan + 4 * i;
    o[0] = gx;
    o[1] = gy;
    o[2] = gz;
    o[3] = 0.0;
    double *r = geo + (int64_t)kRec * i;
    r[13] = gx;
    r[14] = gy;
    r[15] = gz;
}

}  // namespace

rt_status rt_ivanova_impl(rt_ctx *ctx) {
    const int64_t n = ctx->p.n;
    if (!ctx->ivan) {
        rt_status rs = rt_alloc(ctx, (void **)&ctx->ivan, sizeof(double) * 4 * n);
        if (rs != RT_OK) return rs;
    }
    k_ivanova_sums<<<(unsigned)((n + kBlock - 1) / kBlock), kBlock, 0, ctx->stream>>>(
        n, ctx->geo, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath, ctx->p.box, ctx->ivan);
    RT_HIP(hipGetLastError());
    return RT_OK;
}

rt_status rt_set_surfaces_impl(rt_ctx *ctx, int32_t kind) {
    if (kind == RT_IVANOVA) {
        rt_status rs = rt_ivanova_impl(ctx);
        if (rs != RT_OK) return rs;
    }
    ctx->surfaces = kind;
    return RT_OK;
}
