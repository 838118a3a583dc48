// Drift correction of the radiation state (Part III "Dealing With Particle
// Drifts"): a particle moved by dx carries its state extrapolated with its own
// gradients (eq:gradient), U(x + dx) = U(x) + grad U . dx per component.
#include "rt_pair.h"

using namespace gearrt;

namespace {

// One thread per state (particle k, group g), block b owning the kBlock G
// states from b kBlock G on in G rounds of consecutive states.  The moved
// state is computed in FP64 and guarded as the transport's updated state.
// Block partials [nb][2G]: photon totals (columns 0..G-1) and the energy the
// guard adds (columns G..2G-1).
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_drift(int64_t n, const T *__restrict__ UD,
                                                  const double *__restrict__ dx,
                                                  const double *__restrict__ vol, double c,
                                                  T *__restrict__ Uout, double *__restrict__ partials,
                                                  unsigned long long *__restrict__ counts) {
    __shared__ double smem[(kBlock / 64) * 2 * G];
    __shared__ unsigned long long scnt[2];
    if (threadIdx.x < 2) scnt[threadIdx.x] = 0;
    const int64_t ns = n * G;
    const int64_t s0 = (int64_t)blockIdx.x * kBlock * G + threadIdx.x;
    double red[2 * G];
#pragma unroll
    for (int p = 0; p < 2 * G; ++p) red[p] = 0.0;
    int cE = 0, cF = 0;
#pragma unroll
    for (int r = 0; r < G; ++r) {
        const int64_t s = s0 + (int64_t)r * kBlock;
        if (s >= ns) break;
        const int64_t k = s / G;
        const int g = (int)(s - k * G);
        const double d0 = dx[3 * k], d1 = dx[3 * k + 1], d2 = dx[3 * k + 2];
        const T *rec = UD + s * 16;
        double q[4];
#pragma unroll
        for (int m = 0; m < 4; ++m)
            q[m] = (double)rec[m] + (double)rec[4 + 3 * m] * d0 + (double)rec[5 + 3 * m] * d1 +
                   (double)rec[6 + 3 * m] * d2;
        const double Epre = q[0];
        const int f = guard64(q[0], q[1], q[2], q[3], c);
        cE += f & 1;
        cF += f >> 1;
        T *o = Uout + s * 4;
#pragma unroll
        for (int m = 0; m < 4; ++m) o[m] = (T)q[m];
        const double V = vol[k];
#pragma unroll
        for (int p = 0; p < G; ++p) {
            red[p] += p == g ? V * (double)o[0] : 0.0;
            red[G + p] += (p == g && (f & 1)) ? -Epre * V : 0.0;
        }
    }
    if (partials)
        block_reduce_store<2 * G>(red, partials + (int64_t)blockIdx.x * 2 * G, smem,
                                  [](int p) { return p; });
    if (counts) {
        const int64_t v0 = wave_sum_i64(cE), v1 = wave_sum_i64(cF);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&scnt[0], (unsigned long long)v0);
            atomicAdd(&scnt[1], (unsigned long long)v1);
        }
        __syncthreads();
        if (threadIdx.x < 2 && scnt[threadIdx.x])
            atomicAdd(&counts[RT_CNT_CELL_E + threadIdx.x], scnt[threadIdx.x]);
    }
}

template <typename T, int G>
void launch_drift(rt_ctx *ctx, const T *UD, const double *dx, T *Uout, double *part,
                  int64_t *counts, int64_t nb) {
    k_drift<T, G><<<(unsigned)nb, kBlock, 0, ctx->stream>>>(ctx->p.n, UD, dx, ctx->vol,
                                                            ctx->p.c_red, Uout, part,
                                                            (unsigned long long *)counts);
}

}  // namespace

rt_status rt_drift_impl(rt_ctx *ctx, const void *UD, const double *dx, void *U_out, double *Q,
                        int64_t *counts, double *ledger) {
    const int64_t n = ctx->p.n;
    const int64_t nb = (n + kBlock - 1) / kBlock;   // the rows of the partials buffer
    double *part = (Q || ledger) ? ctx->partials : nullptr;
    rt_timer_begin(ctx, "drift");
#define RT_DRIFT_CASE(GG)                                                                     \
    case GG:                                                                                  \
        if (ctx->p.precision == RT_FP64)                                                      \
            launch_drift<double, GG>(ctx, (const double *)UD, dx, (double *)U_out, part,      \
                                     counts, nb);                                             \
        else                                                                                  \
            launch_drift<float, GG>(ctx, (const float *)UD, dx, (float *)U_out, part, counts, \
                                    nb);                                                      \
        break;
    switch (ctx->p.groups) {
        RT_DRIFT_CASE(1)
        RT_DRIFT_CASE(2)
        RT_DRIFT_CASE(3)
        RT_DRIFT_CASE(4)
        RT_DRIFT_CASE(5)
        RT_DRIFT_CASE(6)
        RT_DRIFT_CASE(7)
        RT_DRIFT_CASE(8)
        default: break;
    }
#undef RT_DRIFT_CASE
    rt_timer_end(ctx, "drift");
    RT_HIP(hipGetLastError());
    if (part) {
        rt_finalize_partials(ctx, nb, Q, ledger);
        RT_HIP(hipGetLastError());
    }
    return RT_OK;
}
