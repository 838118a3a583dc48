// Individual power-of-two time steps (Part II "Individual time steps",
// eq:meshless-explicit-individual-timesteps; Part III eq:transport-update-
// explicit, whose exchanges are time integrated with min{dt_k, dt_l}; the
// factor-4 limiter of Part III "Dynamic Sub-Cycling").
//
// Time bins: dt_i = dt 2^b_i (dt the smallest CFL step, as rt_build_cells
// computes it), b_i the largest n <= max_bin with dt 2^n <= C_cfl dx_i / c,
// then lowered until interacting particles are at most 2 bins apart.  The
// bins live in slot 12 of the geometry records, and with the smallest bin of
// each particle's neighbourhood in bin8 (n bytes each; all 0 after
// rt_build_cells: the global step).  Slots 13-15 of the records hold the
// Ivanova kernel-gradient sums.  A tick t advances the time by dt; particle i ends a step at the end
// of tick t when (t + 1) is a multiple of 2^b_i.
#include "rt_internal.h"

using namespace gearrt;

namespace {

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

__device__ __forceinline__ bool ends_step(int64_t tick, int32_t b) {
    return ((tick + 1) & ((int64_t(1) << b) - 1)) == 0;
}

// own CFL bin (eq:rt-cfl with the particle's own dx)
__global__ void k_bins_init(int64_t n, const double *__restrict__ geo,
                            const double *__restrict__ dtp, double cfl, double c, int32_t nmax,
                            int32_t *__restrict__ bin) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double dx = cbrt(geo[(int64_t)kRec * i + R_V] * (3.0 / (4.0 * kPi)));
    const double tau = cfl * dx / c, dt = dtp[0];
    int32_t b = 0;
    while (b < nmax && ldexp(dt, b + 1) <= tau) ++b;
    bin[i] = b;
}

// one Jacobi sweep of b_i <- min(b_i, min_j b_j + 2) over the symmetric lists
__global__ void k_bins_limit(int64_t n, const int32_t *__restrict__ nbr,
                             const int64_t *__restrict__ wave_base,
                             const int32_t *__restrict__ n_nbr, const int32_t *__restrict__ bin,
                             int32_t *__restrict__ out, int32_t *__restrict__ changed) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t base = wave_base[i >> 6] + (i & 63);
    int32_t m = bin[i];
    const int32_t nn = n_nbr[i];
    for (int32_t k = 0; k < nn; ++k) m = min(m, bin[nbr[base + 64 * (int64_t)k]] + 2);
    out[i] = m;
    if (m != bin[i]) atomicOr(changed, 1);
}

// bins into the geometry records (slot 12), into bin8 with the smallest bin of
// each neighbourhood (bin8[n + i]), and into the FP32 records (slot F_BIN) of
// FP32C contexts
__global__ void k_bins_store(int64_t n, const int32_t *__restrict__ nbr,
                             const int64_t *__restrict__ wave_base,
                             const int32_t *__restrict__ n_nbr, const int32_t *__restrict__ bin,
                             double *__restrict__ geo, float *__restrict__ geo32,
                             uint8_t *__restrict__ bin8) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t base = wave_base[i >> 6] + (i & 63);
    int32_t m = bin[i];
    const int32_t nn = n_nbr[i];
    for (int32_t k = 0; k < nn; ++k) m = min(m, bin[nbr[base + 64 * (int64_t)k]]);
    geo[(int64_t)kRec * i + 12] = (double)bin[i];
    if (geo32) geo32[(int64_t)F_REC * i + F_BIN] = (float)bin[i];
    bin8[i] = (uint8_t)bin[i];
    bin8[n + i] = (uint8_t)m;
}

__global__ void k_bins_max(int64_t n, const int32_t *__restrict__ bin, int32_t *__restrict__ top) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicMax(top, bin[i]);
}

// injection for the particles that end a step in this tick, each with its dt
template <typename T>
__global__ void k_inject_binned(int32_t ngas, int G, const int32_t *__restrict__ gptr,
                                const int32_t *__restrict__ gas, const int32_t *__restrict__ src,
                                const double *__restrict__ coef, const double *__restrict__ L,
                                const double *__restrict__ dtp, const double *__restrict__ geo,
                                int64_t tick, T *__restrict__ U) {
    const int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ngas) return;
    const int64_t g = gas[t];
    const int32_t b = (int32_t)geo[(int64_t)kRec * g + 12];
    if (!ends_step(tick, b)) return;
    const double dtg = ldexp(dtp[0], b);
    for (int grp = 0; grp < G; ++grp) {
        double s = 0.0;
        for (int32_t e = gptr[t]; e < gptr[t + 1]; ++e) s += coef[e] * L[(int64_t)src[e] * G + grp];
        T *E = U + (g * G + grp) * 4;
        E[0] = (T)((double)E[0] + dtg * s);
    }
}

// the stored state of the particles that ended a step follows their update;
// the bins come from the compact copy (one byte per particle) once
// rt_time_bins has run, else from the geometry records
template <typename T>
__global__ void k_refresh(int64_t n, int G, const uint8_t *__restrict__ bin8,
                          const double *__restrict__ geo, int64_t tick, const T *__restrict__ U,
                          T *__restrict__ UD) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * G) return;
    const int64_t i = t / G;
    const int32_t b = bin8 ? (int32_t)bin8[i] : (int32_t)geo[(int64_t)kRec * i + 12];
    if (!ends_step(tick, b)) return;
#pragma unroll
    for (int m = 0; m < 4; ++m) UD[t * 16 + m] = U[t * 4 + m];
}

}  // namespace

rt_status rt_time_bins_impl(rt_ctx *ctx, int32_t max_bin, int32_t *bins_out, int64_t *cycle) {
    const int64_t n = ctx->p.n;
    int32_t *work = nullptr;
    rt_status rs = rt_alloc(ctx, (void **)&work, sizeof(int32_t) * (2 * n + 2));
    if (rs != RT_OK) return rs;
    int32_t *b = work, *b2 = work + n, *flag = work + 2 * n;
    hipStream_t st = ctx->stream;
    k_bins_init<<<nblk(n), kBlock, 0, st>>>(n, ctx->geo, ctx->dt_dev, ctx->p.cfl, ctx->p.c_red,
                                            max_bin, b);
    // the limiter lowers a bin by one hop per sweep: at most max_bin / 2 + 1
    // sweeps change anything
    int32_t changed = 1, sweeps = 0;
    while (changed) {
        if (sweeps > max_bin + 2) {
            rt_free(ctx, work);
            return rt_fail(ctx, RT_EHIP, "time-bin limiter did not converge");
        }
        RT_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
        k_bins_limit<<<nblk(n), kBlock, 0, st>>>(n, ctx->nbr, ctx->wave_base, ctx->n_nbr, b, b2,
                                                 flag);
        RT_HIP(hipMemcpyAsync(&changed, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RT_HIP(hipStreamSynchronize(st));
        int32_t *tmp = b;
        b = b2;
        b2 = tmp;
        ++sweeps;
    }
    if (!ctx->bin8 && (rs = rt_alloc(ctx, (void **)&ctx->bin8, 2 * (size_t)n)) != RT_OK) {
        rt_free(ctx, work);
        return rs;
    }
    k_bins_store<<<nblk(n), kBlock, 0, st>>>(n, ctx->nbr, ctx->wave_base, ctx->n_nbr, b, ctx->geo,
                                             ctx->geo32, ctx->bin8);
    RT_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), st));
    k_bins_max<<<nblk(n), kBlock, 0, st>>>(n, b, flag);
    int32_t top = 0;
    RT_HIP(hipMemcpyAsync(&top, flag, sizeof(int32_t), hipMemcpyDeviceToHost, st));
    if (bins_out)
        RT_HIP(hipMemcpyAsync(bins_out, b, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    RT_HIP(hipStreamSynchronize(st));
    RT_HIP(hipGetLastError());
    rt_free(ctx, work);
    ctx->bin_top = top;
    if (cycle) *cycle = int64_t(1) << top;
    return RT_OK;
}

rt_status rt_tick_impl(rt_ctx *ctx, void *U, const double *L, int64_t tick, void *UD,
                       double *acc, double *Q, int64_t *counts, double *ledger) {
    const int64_t n = ctx->p.n;
    const int G = ctx->p.groups;
    const bool f64 = ctx->p.precision == RT_FP64;
    if (ctx->S > 0 && ctx->n_inj_gas > 0 && L) {
        if (f64)
            k_inject_binned<double><<<nblk(ctx->n_inj_gas), kBlock, 0, ctx->stream>>>(
                ctx->n_inj_gas, G, ctx->inj_gptr, ctx->inj_gas, ctx->inj_src, ctx->inj_coef, L,
                ctx->dt_dev, ctx->geo, tick, (double *)U);
        else
            k_inject_binned<float><<<nblk(ctx->n_inj_gas), kBlock, 0, ctx->stream>>>(
                ctx->n_inj_gas, G, ctx->inj_gptr, ctx->inj_gas, ctx->inj_src, ctx->inj_coef, L,
                ctx->dt_dev, ctx->geo, tick, (float *)U);
        RT_HIP(hipGetLastError());
    }
    rt_status rs = f64 ? rt_tick_step_impl(ctx, (double *)U, (double *)UD, ctx->dt_dev, tick, acc,
                                           Q, counts, ledger)
                       : rt_tick_step32_impl(ctx, (float *)U, (float *)UD, ctx->dt_dev, tick,
                                             acc, Q, counts, ledger);
    if (rs != RT_OK) return rs;
    if (f64)
        k_refresh<double><<<nblk(n * G), kBlock, 0, ctx->stream>>>(n, G, ctx->bin8, ctx->geo, tick,
                                                                   (const double *)U,
                                                                   (double *)UD);
    else
        k_refresh<float><<<nblk(n * G), kBlock, 0, ctx->stream>>>(n, G, ctx->bin8, ctx->geo, tick,
                                                                  (const float *)U, (float *)UD);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
