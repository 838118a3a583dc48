// C ABI of the photon-transport library: argument validation, context
// lifetime, stream binding, queries and event timing.  The arithmetic lives in
// rt_build.hip, rt_step.hip and rt_adjoint.hip.
#include <string.h>

#include <algorithm>
#include <vector>

#include "rt_internal.h"

using namespace gearrt;

static std::string g_create_err;

rt_status rt_fail(rt_ctx *ctx, rt_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    else g_create_err = msg;
    return st;
}

bool rt_try_alloc(rt_ctx *ctx, void **ptr, size_t bytes) {
    *ptr = nullptr;
    if (bytes == 0) bytes = 8;
    if (hipMalloc(ptr, bytes) != hipSuccess) {
        *ptr = nullptr;
        (void)hipGetLastError();
        return false;
    }
    ctx->allocs[*ptr] = bytes;
    ctx->device_bytes += (int64_t)bytes;
    ctx->device_peak = std::max(ctx->device_peak, ctx->device_bytes);
    return true;
}

rt_status rt_alloc(rt_ctx *ctx, void **ptr, size_t bytes) {
    if (rt_try_alloc(ctx, ptr, bytes)) return RT_OK;
    return rt_fail(ctx, RT_ENOMEM, "hipMalloc of " + std::to_string(bytes ? bytes : 8) +
                                       " bytes failed");
}

void rt_free(rt_ctx *ctx, void *ptr) {
    if (!ptr) return;
    auto it = ctx->allocs.find(ptr);
    if (it != ctx->allocs.end()) {
        ctx->device_bytes -= (int64_t)it->second;
        ctx->allocs.erase(it);
    }
    (void)hipFree(ptr);
}

void rt_timer_begin(rt_ctx *ctx, const char *) {
    if (!ctx->timing) return;
    if (ctx->ev_used + 2 > ctx->ev_pool.size()) {
        for (int k = 0; k < 64; ++k) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            ctx->ev_pool.push_back(e);
        }
    }
    hipEvent_t a = ctx->ev_pool[ctx->ev_used++];
    (void)hipEventRecord(a, ctx->stream);
    ctx->ev_open.push_back(a);
}

void rt_timer_end(rt_ctx *ctx, const char *name) {
    if (!ctx->timing || ctx->ev_open.empty()) return;
    if (ctx->ev_used + 1 > ctx->ev_pool.size()) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        ctx->ev_pool.push_back(e);
    }
    hipEvent_t b = ctx->ev_pool[ctx->ev_used++];
    (void)hipEventRecord(b, ctx->stream);
    ctx->trecs.push_back({name, ctx->ev_open.back(), b});
    ctx->ev_open.pop_back();
}

static bool finite_pos(double v) { return v > 0.0 && v < 1e300; }

extern "C" {

rt_status rt_create(const rt_params *p, rt_ctx **out) {
    if (!out) return rt_fail(nullptr, RT_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return rt_fail(nullptr, RT_EINVAL, "params is NULL");
    if (p->n < 1 || p->n > (int64_t(1) << 28))
        return rt_fail(nullptr, RT_EINVAL, "n must be in [1, 2^28]");
    if (p->groups < 1 || p->groups > 8) return rt_fail(nullptr, RT_EINVAL, "groups must be in [1, 8]");
    if (p->precision != RT_FP64 && p->precision != RT_FP32C)
        return rt_fail(nullptr, RT_EINVAL, "precision must be RT_FP64 or RT_FP32C");
    if (!finite_pos(p->box)) return rt_fail(nullptr, RT_EINVAL, "box must be positive");
    if (!finite_pos(p->eta)) return rt_fail(nullptr, RT_EINVAL, "eta must be positive");
    if (!finite_pos(p->kappa)) return rt_fail(nullptr, RT_EINVAL, "kappa must be positive");
    if (!finite_pos(p->c_red)) return rt_fail(nullptr, RT_EINVAL, "c_red must be positive");
    if (!finite_pos(p->cfl)) return rt_fail(nullptr, RT_EINVAL, "cfl must be positive");
    rt_ctx *ctx = new (std::nothrow) rt_ctx();
    if (!ctx) return rt_fail(nullptr, RT_ENOMEM, "host allocation failed");
    ctx->p = *p;
    ctx->stream = (hipStream_t)p->hip_stream;
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return rt_fail(nullptr, RT_EHIP, "no HIP device");
    }
    rt_status rs;
    if ((rs = rt_alloc(ctx, (void **)&ctx->status, sizeof(int32_t))) != RT_OK ||
        (rs = rt_alloc(ctx, (void **)&ctx->dt_dev, sizeof(double))) != RT_OK) {
        g_create_err = ctx->err;
        rt_destroy(ctx);
        return rs;
    }
    if (hipMemset(ctx->status, 0, sizeof(int32_t)) != hipSuccess) {
        rt_destroy(ctx);
        return rt_fail(nullptr, RT_EHIP, "hipMemset failed");
    }
    rt_adjoint_static_init(ctx);
    *out = ctx;
    return RT_OK;
}

void rt_destroy(rt_ctx *ctx) {
    if (!ctx) return;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    void *bufs[] = {ctx->xs, ctx->geo, ctx->geo32, ctx->perm32, ctx->keys, ctx->dt_dev,
                    ctx->h_iters, ctx->node_lo, ctx->node_hi, ctx->node_hmax, ctx->n_nbr,
                    ctx->n_gath, ctx->wave_base, ctx->nbr, ctx->src_h, ctx->inj_gptr,
                    ctx->inj_gas, ctx->inj_src, ctx->inj_coef, ctx->inj_xi, ctx->src_ptr,
                    ctx->src_gas, ctx->src_coef, ctx->status, ctx->partials, ctx->scan_tmp,
                    ctx->adj_buf, ctx->hll_table, ctx->hll_table32, ctx->vol, ctx->ivan,
                    ctx->bin8, ctx->task, ctx->n_task, ctx->tstat, ctx->uoff, ctx->urow, ctx->gloc,
                    ctx->uown, ctx->ublk, ctx->goff, ctx->aoff, ctx->arow, ctx->agloc,
                    ctx->aown, ctx->ablk};
    for (void *b : bufs) rt_free(ctx, b);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

const char *rt_last_error(const rt_ctx *ctx) {
    return ctx ? ctx->err.c_str() : g_create_err.c_str();
}

rt_status rt_set_stream(rt_ctx *ctx, void *s) {
    if (!ctx) return RT_EINVAL;
    ctx->stream = (hipStream_t)s;
    ctx->p.hip_stream = s;
    return RT_OK;
}

rt_status rt_build_cells(rt_ctx *ctx, const double *x, const double *h_in, int64_t *perm,
                         double *h, double *V, double *dt) {
    if (!ctx) return RT_EINVAL;
    if (!x || !h || !V) return rt_fail(ctx, RT_EINVAL, "x, h and V are required");
    return rt_build_impl(ctx, x, h_in, perm, h, V, dt);
}

rt_status rt_set_h_iterations(rt_ctx *ctx, int32_t max_iter) {
    if (!ctx) return RT_EINVAL;
    if (max_iter < 1 || max_iter > 10000)
        return rt_fail(ctx, RT_EINVAL, "max_iter must be in 1 .. 10000");
    ctx->h_iter_cap = max_iter;
    return RT_OK;
}

rt_status rt_set_sources(rt_ctx *ctx, int32_t n_src, const double *xs, double eta_star) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (n_src < 0 || n_src > (1 << 20)) return rt_fail(ctx, RT_EINVAL, "n_src out of range");
    if (n_src > 0 && !xs) return rt_fail(ctx, RT_EINVAL, "xs is NULL");
    if (n_src > 0 && !finite_pos(eta_star)) return rt_fail(ctx, RT_EINVAL, "eta_star must be positive");
    return rt_sources_impl(ctx, n_src, xs, eta_star);
}

rt_status rt_inject(rt_ctx *ctx, void *U, const double *L, const double *dt) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (ctx->S == 0) return RT_OK;
    if (!U || !L || !dt) return rt_fail(ctx, RT_EINVAL, "U, L and dt are required");
    return rt_inject_impl(ctx, U, L, dt);
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

static bool overlap(const void *a, size_t na, const void *b, size_t nb) {
    const char *x = (const char *)a, *y = (const char *)b;
    return x < y + nb && y < x + na;
}

rt_status rt_gradient(rt_ctx *ctx, const void *U, void *UD) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (!U || !UD) return rt_fail(ctx, RT_EINVAL, "U and UD are required");
    size_t es = ctx->p.precision == RT_FP64 ? 8 : 4;
    size_t nu = es * 4 * ctx->p.groups * ctx->p.n;
    if (overlap(U, nu, UD, 4 * nu)) return rt_fail(ctx, RT_EINVAL, "U and UD overlap");
    if (!aligned16(U) || !aligned16(UD))
        return rt_fail(ctx, RT_EINVAL, "U and UD must be 16-byte aligned");
    return rt_gradient_impl(ctx, U, UD);
}

rt_status rt_transport(rt_ctx *ctx, const void *UD, const double *dt, void *U_out,
                       double *photon_total, int64_t *counts, double *ledger,
                       void *U_unguarded) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (!UD || !dt || !U_out) return rt_fail(ctx, RT_EINVAL, "UD, dt and U_out are required");
    size_t es = ctx->p.precision == RT_FP64 ? 8 : 4;
    size_t nu = es * 4 * ctx->p.groups * ctx->p.n;
    if (overlap(UD, 4 * nu, U_out, nu)) return rt_fail(ctx, RT_EINVAL, "UD and U_out overlap");
    if (U_unguarded && overlap(U_unguarded, nu, U_out, nu))
        return rt_fail(ctx, RT_EINVAL, "U_unguarded and U_out overlap");
    if (!aligned16(UD)) return rt_fail(ctx, RT_EINVAL, "UD must be 16-byte aligned");
    return rt_transport_impl(ctx, UD, dt, U_out, photon_total, counts, ledger, U_unguarded);
}

rt_status rt_photon_total(rt_ctx *ctx, const void *U, double *Q) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (!U || !Q) return rt_fail(ctx, RT_EINVAL, "U and Q are required");
    return rt_total_impl(ctx, U, Q);
}

rt_status rt_set_riemann(rt_ctx *ctx, int32_t solver) {
    if (!ctx) return RT_EINVAL;
    if (solver != RT_GLF && solver != RT_HLL)
        return rt_fail(ctx, RT_EINVAL, "solver must be RT_GLF or RT_HLL");
    return rt_set_riemann_impl(ctx, solver);
}

rt_status rt_set_surfaces(rt_ctx *ctx, int32_t kind) {
    if (!ctx) return RT_EINVAL;
    if (kind != RT_HOPKINS && kind != RT_IVANOVA)
        return rt_fail(ctx, RT_EINVAL, "kind must be RT_HOPKINS or RT_IVANOVA");
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    return rt_set_surfaces_impl(ctx, kind);
}

rt_status rt_get_hll_table(rt_ctx *ctx, double *tab) {
    if (!tab) return rt_fail(ctx, RT_EINVAL, "tab is NULL");
    std::vector<double> t = rt_hll_speed_table(RT_HLL_NF, RT_HLL_NMU);
    memcpy(tab, t.data(), sizeof(double) * t.size());
    return RT_OK;
}

rt_status rt_photon_groups(int32_t G, const double *edges_eV, double T_bb, double *sigma_N,
                           double *sigma_E, double *eps, double *frac) {
    if (G < 1 || G > 64) return rt_fail(nullptr, RT_EINVAL, "G must be in 1 .. 64");
    if (!edges_eV || !sigma_N || !sigma_E || !eps)
        return rt_fail(nullptr, RT_EINVAL, "edges_eV, sigma_N, sigma_E and eps are required");
    if (!finite_pos(T_bb)) return rt_fail(nullptr, RT_EINVAL, "T_bb must be positive");
    if (!finite_pos(edges_eV[0])) return rt_fail(nullptr, RT_EINVAL, "edges_eV[0] must be positive");
    for (int32_t i = 0; i < G; ++i) {
        if (!(edges_eV[i + 1] > edges_eV[i]))
            return rt_fail(nullptr, RT_EINVAL, "edges_eV must increase");
        if (i + 1 < G && !finite_pos(edges_eV[i + 1]))
            return rt_fail(nullptr, RT_EINVAL, "only the last edge may be infinite");
    }
    std::string err;
    rt_status rs = rt_photon_groups_impl(G, edges_eV, T_bb, sigma_N, sigma_E, eps, frac, err);
    if (rs != RT_OK) return rt_fail(nullptr, rs, err);
    return RT_OK;
}

rt_status rt_absorb(rt_ctx *ctx, void *U, int32_t J, const double *n_old, const double *n_new,
                    const double *sigma, const double *dt, double *photon_total,
                    double *absorbed) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (!U || !n_old || !sigma || !dt)
        return rt_fail(ctx, RT_EINVAL, "U, n_old, sigma and dt are required");
    if (J < 1 || J > 8) return rt_fail(ctx, RT_EINVAL, "J must be in 1 .. 8");
    size_t es = ctx->p.precision == RT_FP64 ? 8 : 4;
    size_t nu = es * 4 * ctx->p.groups * ctx->p.n, nn = sizeof(double) * J * ctx->p.n;
    if (overlap(U, nu, n_old, nn) || (n_new && overlap(U, nu, n_new, nn)) ||
        overlap(U, nu, sigma, sizeof(double) * J * ctx->p.groups))
        return rt_fail(ctx, RT_EINVAL, "n_old, n_new and sigma must not overlap U");
    return rt_absorb_impl(ctx, U, J, n_old, n_new, sigma, dt, photon_total, absorbed);
}

rt_status rt_drift(rt_ctx *ctx, const void *UD, const double *dx, void *U_out,
                   double *photon_total, int64_t *counts, double *ledger) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (!UD || !dx || !U_out) return rt_fail(ctx, RT_EINVAL, "UD, dx and U_out are required");
    size_t es = ctx->p.precision == RT_FP64 ? 8 : 4;
    size_t nu = es * 4 * ctx->p.groups * ctx->p.n, nx = sizeof(double) * 3 * ctx->p.n;
    if (overlap(UD, 4 * nu, U_out, nu) || overlap(dx, nx, U_out, nu))
        return rt_fail(ctx, RT_EINVAL, "U_out must not overlap UD or dx");
    if (!aligned16(UD)) return rt_fail(ctx, RT_EINVAL, "UD must be 16-byte aligned");
    return rt_drift_impl(ctx, UD, dx, U_out, photon_total, counts, ledger);
}

rt_status rt_time_bins(rt_ctx *ctx, int32_t max_bin, int32_t *bins, int64_t *cycle_ticks) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (max_bin < 0 || max_bin > 30) return rt_fail(ctx, RT_EINVAL, "max_bin must be in 0 .. 30");
    return rt_time_bins_impl(ctx, max_bin, bins, cycle_ticks);
}

rt_status rt_tick(rt_ctx *ctx, void *U, const double *L, int64_t tick, void *UD,
                  double *acc, double *photon_total, int64_t *counts, double *ledger) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (!U || !UD || !acc) return rt_fail(ctx, RT_EINVAL, "U, UD and acc are required");
    if (tick < 0) return rt_fail(ctx, RT_EINVAL, "tick must be >= 0");
    if (ctx->S > 0 && !L) return rt_fail(ctx, RT_EINVAL, "L is required when sources are set");
    const size_t es = ctx->p.precision == RT_FP64 ? sizeof(double) : sizeof(float);
    const size_t nu = es * 4 * ctx->p.groups * ctx->p.n, na = sizeof(double) * 4 * ctx->p.groups * ctx->p.n;
    if (overlap(UD, 4 * nu, U, nu) || overlap(UD, 4 * nu, acc, na) || overlap(U, nu, acc, na))
        return rt_fail(ctx, RT_EINVAL, "U, UD and acc must not overlap");
    if (!aligned16(U) || !aligned16(UD))
        return rt_fail(ctx, RT_EINVAL, "U and UD must be 16-byte aligned");
    return rt_tick_impl(ctx, U, L, tick, UD, acc, photon_total, counts, ledger);
}

rt_status rt_adjoint(rt_ctx *ctx, const void *U_pre, const double *L, const double *dt,
                     const void *UD, const void *U_unguarded, const void *lam_next, void *lam,
                     double *dL_dL) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (!dt || !lam_next || !lam) return rt_fail(ctx, RT_EINVAL, "dt, lam_next and lam are required");
    if (!UD && !U_pre) return rt_fail(ctx, RT_EINVAL, "U_pre is required when UD is NULL");
    if (ctx->S > 0 && !L) return rt_fail(ctx, RT_EINVAL, "L is required when sources are set");
    if (UD && !aligned16(UD)) return rt_fail(ctx, RT_EINVAL, "UD must be 16-byte aligned");
    return rt_adjoint_impl(ctx, U_pre, L, dt, UD, U_unguarded, lam_next, lam, dL_dL);
}

rt_status rt_adjoint_static(rt_ctx *ctx, const double *L, const double *dt, const void *UD,
                            const void *U_unguarded, const void *lam_next, void *lam,
                            double *dL_dL) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    if (!dt || !UD || !U_unguarded || !lam_next || !lam)
        return rt_fail(ctx, RT_EINVAL, "dt, UD, U_unguarded, lam_next and lam are required");
    if (ctx->S > 0 && !L) return rt_fail(ctx, RT_EINVAL, "L is required when sources are set");
    if (!aligned16(UD)) return rt_fail(ctx, RT_EINVAL, "UD must be 16-byte aligned");
    return rt_adjoint_static_impl(ctx, L, dt, UD, U_unguarded, lam_next, lam, dL_dL);
}

rt_status rt_sync(rt_ctx *ctx) {
    if (!ctx) return RT_EINVAL;
    RT_HIP(hipStreamSynchronize(ctx->stream));
    RT_HIP(hipGetLastError());
    int32_t st = 0;
    RT_HIP(hipMemcpy(&st, ctx->status, sizeof(int32_t), hipMemcpyDeviceToHost));
    if (st) RT_HIP(hipMemset(ctx->status, 0, sizeof(int32_t)));
    if (st & ST_NOCONV) return rt_fail(ctx, RT_ENOCONV, "smoothing length did not converge");
    if (st & ST_SINGULAR) return rt_fail(ctx, RT_ESINGULAR, "E_i not positive definite");
    if (st & ST_BIGH) return rt_fail(ctx, RT_EINVAL, "compact support reaches half the box");
    if (st & ST_NONFINITE)
        return rt_fail(ctx, RT_ENONFINITE, "a state or gradient record is NaN or infinite");
    return RT_OK;
}

rt_status rt_get_stats(rt_ctx *ctx, rt_stats *out) {
    if (!ctx || !out) return RT_EINVAL;
    memset(out, 0, sizeof *out);
    out->n = ctx->p.n;
    out->n_entries = ctx->n_entries;
    out->n_pairs = ctx->n_entries / 2;
    out->n_gather = ctx->n_gather_entries;
    out->sell_slots = ctx->slots;
    out->max_neighbours = ctx->max_nbr;
    out->h_iter_max = ctx->h_iter_max;
    out->n_inject = ctx->n_inj;
    out->device_bytes = ctx->device_bytes;
    out->device_bytes_peak = ctx->device_peak;
    out->h_list_overflow = ctx->h_list_overflow;
    out->union_blocks = ctx->uoff ? ctx->nwaves - ctx->n_ublk : 0;
    out->union_staged_blocks = ctx->uoff ? ctx->n_ublk : 0;
    out->adj_union_blocks = ctx->aoff ? ctx->nwaves - ctx->n_ablk : 0;
    out->adj_union_staged_blocks = ctx->aoff ? ctx->n_ablk : 0;
    if (ctx->tstat) {
        int64_t t[2];
        RT_HIP(hipStreamSynchronize(ctx->stream));
        RT_HIP(hipMemcpy(t, ctx->tstat, sizeof t, hipMemcpyDeviceToHost));
        out->task_longest = t[0];
        out->task_bound = t[1];
    }
    return RT_OK;
}

rt_status rt_get_geometry(rt_ctx *ctx, double *B, int32_t *n_nbr, int32_t *n_gath) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    const int64_t n = ctx->p.n;
    RT_HIP(hipStreamSynchronize(ctx->stream));
    if (B) {
        // B_i = E_i^{-1} = Bv_i / (V_i^2 sigma / H_i^3)
        std::vector<double> rec((size_t)n * kRec), out((size_t)n * 6);
        RT_HIP(hipStreamSynchronize(ctx->stream));
        RT_HIP(hipMemcpy(rec.data(), ctx->geo, sizeof(double) * kRec * n, hipMemcpyDeviceToHost));
        for (int64_t i = 0; i < n; ++i) {
            const double *r = &rec[(size_t)i * kRec];
            double iH = r[R_IH], V = r[R_V];
            double f = 1.0 / (V * V * kSigma3 * iH * iH * iH);
            for (int a = 0; a < 6; ++a) out[(size_t)i * 6 + a] = r[R_B + a] * f;
        }
        RT_HIP(hipMemcpy(B, out.data(), sizeof(double) * 6 * n, hipMemcpyHostToDevice));
    }
    if (n_nbr) RT_HIP(hipMemcpy(n_nbr, ctx->n_nbr, sizeof(int32_t) * n, hipMemcpyDeviceToDevice));
    if (n_gath) RT_HIP(hipMemcpy(n_gath, ctx->n_gath, sizeof(int32_t) * n, hipMemcpyDeviceToDevice));
    return RT_OK;
}

rt_status rt_get_neighbours(rt_ctx *ctx, int64_t *ptr, int32_t *idx) {
    if (!ctx) return RT_EINVAL;
    if (!ctx->built) return rt_fail(ctx, RT_ESTATE, "rt_build_cells has not run");
    const int64_t n = ctx->p.n;
    RT_HIP(hipStreamSynchronize(ctx->stream));
    std::vector<int32_t> nn(n), table((size_t)std::max<int64_t>(ctx->slots, 1));
    std::vector<int64_t> wb(ctx->nwaves + 1), hp(n + 1);
    RT_HIP(hipMemcpy(nn.data(), ctx->n_nbr, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
    RT_HIP(hipMemcpy(wb.data(), ctx->wave_base, sizeof(int64_t) * (ctx->nwaves + 1), hipMemcpyDeviceToHost));
    RT_HIP(hipMemcpy(table.data(), ctx->nbr, sizeof(int32_t) * std::max<int64_t>(ctx->slots, 1),
                     hipMemcpyDeviceToHost));
    hp[0] = 0;
    for (int64_t i = 0; i < n; ++i) hp[i + 1] = hp[i] + nn[i];
    std::vector<int32_t> hi((size_t)std::max<int64_t>(hp[n], 1));
    for (int64_t i = 0; i < n; ++i) {
        int64_t base = wb[i >> 6] + (i & 63);
        for (int32_t k = 0; k < nn[i]; ++k) hi[hp[i] + k] = table[base + 64 * (int64_t)k];
    }
    if (ptr) RT_HIP(hipMemcpy(ptr, hp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice));
    if (idx && hp[n] > 0) RT_HIP(hipMemcpy(idx, hi.data(), sizeof(int32_t) * hp[n], hipMemcpyHostToDevice));
    return RT_OK;
}

rt_status rt_get_sources(rt_ctx *ctx, int32_t *gas, int32_t *src, double *xi, double *h_src) {
    if (!ctx) return RT_EINVAL;
    RT_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->S == 0) return RT_OK;
    std::vector<int32_t> gp(ctx->n_inj_gas + 1), g(ctx->n_inj_gas), full(ctx->n_inj);
    RT_HIP(hipMemcpy(gp.data(), ctx->inj_gptr, sizeof(int32_t) * (ctx->n_inj_gas + 1), hipMemcpyDeviceToHost));
    RT_HIP(hipMemcpy(g.data(), ctx->inj_gas, sizeof(int32_t) * ctx->n_inj_gas, hipMemcpyDeviceToHost));
    for (int32_t t = 0; t < ctx->n_inj_gas; ++t)
        for (int32_t e = gp[t]; e < gp[t + 1]; ++e) full[e] = g[t];
    if (gas) RT_HIP(hipMemcpy(gas, full.data(), sizeof(int32_t) * ctx->n_inj, hipMemcpyHostToDevice));
    if (src) RT_HIP(hipMemcpy(src, ctx->inj_src, sizeof(int32_t) * ctx->n_inj, hipMemcpyDeviceToDevice));
    if (xi) RT_HIP(hipMemcpy(xi, ctx->inj_xi, sizeof(double) * ctx->n_inj, hipMemcpyDeviceToDevice));
    if (h_src) RT_HIP(hipMemcpy(h_src, ctx->src_h, sizeof(double) * ctx->S, hipMemcpyDeviceToDevice));
    return RT_OK;
}

rt_status rt_timing(rt_ctx *ctx, int32_t on) {
    if (!ctx) return RT_EINVAL;
    if (on) {
        RT_HIP(hipStreamSynchronize(ctx->stream));
        ctx->trecs.clear();
        ctx->ev_open.clear();
        ctx->ev_used = 0;
    }
    ctx->timing = on ? 1 : 0;
    return RT_OK;
}

rt_status rt_get_timing(rt_ctx *ctx, const char *kernel, double *ms_total, int64_t *launches) {
    if (!ctx || !kernel) return RT_EINVAL;
    RT_HIP(hipStreamSynchronize(ctx->stream));
    double ms = 0.0;
    int64_t cnt = 0;
    for (auto &r : ctx->trecs) {
        if (r.name != kernel) continue;
        float t = 0.0f;
        RT_HIP(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        ++cnt;
    }
    if (ms_total) *ms_total = ms;
    if (launches) *launches = cnt;
    return RT_OK;
}

}  // extern "C"
