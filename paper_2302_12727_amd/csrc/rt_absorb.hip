// Photo-absorption: the photon removal of the thermochemistry step (Part III
// "Third step: Thermochemistry") and the group constants it needs (Part III
// "Discretization of Frequencies": eq:sigma_N, the energy-weighted average
// beside it and the mean photon energy, for the blackbody spectrum
// eq:blackbody and the photo-ionization cross-section fits
// eq:sigma-parametrizaiton with tab:cross-sections).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "rt_pair.h"

using namespace gearrt;

// ---------------------------------------------------------------------------
// group constants (host)

namespace {

constexpr double kKB = 1.380649e-16;        // erg / K
constexpr double kEV = 1.602176634e-12;     // erg
constexpr int kSpecies = 3;                 // H0, He0, He+
// ionization energies in eV (eq:nuIonHI, eq:nuIonHeI, eq:nuIonHeII)
constexpr double kEion[kSpecies] = {13.60, 24.59, 54.42};
// fit parameters of tab:cross-sections per species: E_0 [eV], sigma_0 [cm^2]
// (the fits' sigma_0 in Mb already multiplied by 1e-18), y_a, P, y_w, y_0, y_1
constexpr double kFit[kSpecies][7] = {
    {0.4298, 5.475e-14, 32.88, 2.963, 0.0, 0.0, 0.0},
    {13.61, 9.492e-16, 1.469, 3.188, 2.039, 0.4434, 2.136},
    {1.720, 1.369e-14, 32.88, 2.963, 0.0, 0.0, 0.0},
};

// photo-ionization cross section of species j at photon energy E [eV], cm^2
double cross_section(int j, double E) {
    if (E < kEion[j]) return 0.0;
    const double *p = kFit[j];
    const double x = E / p[0] - p[5];
    const double y = std::sqrt(x * x + p[6] * p[6]);
    const double F = ((x - 1.0) * (x - 1.0) + p[4] * p[4]) * std::pow(y, 0.5 * p[3] - 5.5) *
                     std::pow(1.0 + std::sqrt(y / p[2]), -p[3]);
    return p[1] * F;
}

// nodes and weights of the n-point Gauss-Legendre rule on [-1, 1]: roots of
// P_n by Newton's method from the usual cosine guesses, P_n and P_n' from the
// three-term recurrence
struct GaussRule {
    std::vector<double> x, w;
    explicit GaussRule(int n) : x(n), w(n) {
        for (int i = 0; i < n; ++i) {
            double z = std::cos(M_PI * (i + 0.75) / (n + 0.5)), dp = 1.0;
            for (int it = 0; it < 100; ++it) {
                double p0 = 1.0, p1 = z;
                for (int k = 2; k <= n; ++k) {
                    const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                    p0 = p1;
                    p1 = p2;
                }
                dp = n * (z * p1 - p0) / (z * z - 1.0);
                const double dz = p1 / dp;
                z -= dz;
                if (std::fabs(dz) < 1e-16) break;
            }
            x[i] = z;
            w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
        }
    }
};

// int_a^b f(x) dx: panels of width <= 1/2 between the break points, 16-point
// Gauss-Legendre on each
template <class F>
double integrate(const GaussRule &q, double a, double b, const std::vector<double> &breaks, F f) {
    std::vector<double> pts{a};
    for (double p : breaks)
        if (p > a && p < b) pts.push_back(p);
    pts.push_back(b);
    double tot = 0.0;
    for (size_t s = 0; s + 1 < pts.size(); ++s) {
        const double lo = pts[s], hi = pts[s + 1];
        const int np = std::max(1, (int)std::ceil((hi - lo) / 0.5));
        const double hw = 0.5 * (hi - lo) / np;
        for (int p = 0; p < np; ++p) {
            const double mid = lo + (2 * p + 1) * hw;
            double acc = 0.0;
            for (size_t k = 0; k < q.x.size(); ++k) acc += q.w[k] * f(mid + hw * q.x[k]);
            tot += hw * acc;
        }
    }
    return tot;
}

}  // namespace

rt_status rt_photon_groups_impl(int32_t G, const double *edges, double T_bb, double *sigma_N,
                                double *sigma_E, double *eps, double *frac, std::string &err) {
    // work in x = E / (k_B T): the blackbody energy density per dx is
    // proportional to x^3 / (e^x - 1) and the photon number to x^2 / (e^x - 1);
    // beyond 80 past a group's lower edge both are below 1e-28 of the group's
    // integral
    const double kT = kKB * T_bb / kEV;   // eV
    const GaussRule q(16);
    std::vector<double> xb(kSpecies);
    for (int j = 0; j < kSpecies; ++j) xb[j] = kEion[j] / kT;
    auto number = [](double x) { return x * x / std::expm1(x); };
    auto energy = [](double x) { return x * x * x / std::expm1(x); };
    const double x0 = edges[0] / kT;
    const double n_all = integrate(q, x0, x0 + 80.0, {}, number);
    for (int32_t i = 0; i < G; ++i) {
        const double a = edges[i] / kT;
        const double b = std::isinf(edges[i + 1]) ? a + 80.0 : std::min(edges[i + 1] / kT, a + 80.0);
        const double ni = integrate(q, a, b, {}, number);
        const double ei = integrate(q, a, b, {}, energy);
        if (!(ni > 0.0) || !(ei > 0.0) || !std::isfinite(ni) || !std::isfinite(ei)) {
            err = "group " + std::to_string(i) + " holds no photons of this spectrum";
            return RT_EINVAL;
        }
        eps[i] = ei / ni * kKB * T_bb;
        if (frac) frac[i] = ni / n_all;
        for (int j = 0; j < kSpecies; ++j) {
            auto sig = [&](double x) { return cross_section(j, x * kT); };
            sigma_N[i * kSpecies + j] =
                integrate(q, a, b, xb, [&](double x) { return number(x) * sig(x); }) / ni;
            sigma_E[i * kSpecies + j] =
                integrate(q, a, b, xb, [&](double x) { return energy(x) * sig(x); }) / ei;
        }
    }
    return RT_OK;
}

// ---------------------------------------------------------------------------
// photon removal (device)

namespace {

// One thread per state (particle k, group g) of the [n][G] states: block b
// owns the kBlock G states from b kBlock G on, in G rounds of kBlock
// consecutive states (consecutive lanes read consecutive states), all rounds'
// loads issued before the first use.  U_kg *= max(0, 1 - c dt sum_j sigma_gj
// nbar_kj), nbar the average of the densities at the two ends of the step.
// Block partials [nb][2G]: photon totals after the removal (columns 0..G-1)
// and the removed energy sum_k V_k dE_kg (columns G..2G-1).
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_absorb(int64_t n, int J, const double *__restrict__ vol,
                                                   const double *__restrict__ n_old,
                                                   const double *__restrict__ n_new,
                                                   const double *__restrict__ sigma,
                                                   const double *__restrict__ dtp, double c,
                                                   T *__restrict__ U, double *__restrict__ partials) {
    __shared__ double ssig[8 * 8];
    __shared__ double smem[(kBlock / 64) * 2 * G];
    if (threadIdx.x < G * J) ssig[threadIdx.x] = sigma[threadIdx.x];
    __syncthreads();
    const double cdt = c * dtp[0];
    const int64_t ns = n * G;
    const int64_t s0 = (int64_t)blockIdx.x * kBlock * G + threadIdx.x;
    double red[2 * G];
#pragma unroll
    for (int p = 0; p < 2 * G; ++p) red[p] = 0.0;
#pragma unroll
    for (int r = 0; r < G; ++r) {
        const int64_t s = s0 + (int64_t)r * kBlock;
        if (s >= ns) break;
        const int64_t k = s / G;
        const int g = (int)(s - k * G);
        double kap = 0.0;
        for (int j = 0; j < J; ++j) {
            const double nb = n_new ? 0.5 * (n_old[k * J + j] + n_new[k * J + j]) : n_old[k * J + j];
            kap += ssig[g * J + j] * nb;
        }
        const double f = fmax(1.0 - cdt * kap, 0.0);
        T *u = U + s * 4;
        const double E0 = (double)u[0];
        const T E1 = (T)(E0 * f);
        u[0] = E1;
        u[1] = (T)((double)u[1] * f);
        u[2] = (T)((double)u[2] * f);
        u[3] = (T)((double)u[3] * f);
        const double V = vol[k];
#pragma unroll
        for (int p = 0; p < G; ++p) {
            red[p] += p == g ? V * (double)E1 : 0.0;
            red[G + p] += p == g ? V * (E0 - (double)E1) : 0.0;
        }
    }
    block_reduce_store<2 * G>(red, partials + (int64_t)blockIdx.x * 2 * G, smem,
                              [](int p) { return p; });
}

template <typename T, int G>
void launch_absorb(rt_ctx *ctx, T *U, int J, const double *n_old, const double *n_new,
                   const double *sigma, const double *dt, int64_t nb) {
    k_absorb<T, G><<<(unsigned)nb, kBlock, 0, ctx->stream>>>(ctx->p.n, J, ctx->vol, n_old, n_new,
                                                             sigma, dt, ctx->p.c_red, U,
                                                             ctx->partials);
}

}  // namespace

rt_status rt_absorb_impl(rt_ctx *ctx, void *U, int32_t J, const double *n_old,
                         const double *n_new, const double *sigma, const double *dt, double *Q,
                         double *absorbed) {
    const int64_t n = ctx->p.n;
    const int G = ctx->p.groups;
    // one block per kBlock particles: the rows of the partials buffer
    const int64_t nb = (n + kBlock - 1) / kBlock;
    rt_timer_begin(ctx, "absorb");
#define RT_ABSORB_CASE(GG)                                                                  \
    case GG:                                                                                \
        if (ctx->p.precision == RT_FP64)                                                    \
            launch_absorb<double, GG>(ctx, (double *)U, J, n_old, n_new, sigma, dt, nb);    \
        else                                                                                \
            launch_absorb<float, GG>(ctx, (float *)U, J, n_old, n_new, sigma, dt, nb);      \
        break;
    switch (G) {
        RT_ABSORB_CASE(1)
        RT_ABSORB_CASE(2)
        RT_ABSORB_CASE(3)
        RT_ABSORB_CASE(4)
        RT_ABSORB_CASE(5)
        RT_ABSORB_CASE(6)
        RT_ABSORB_CASE(7)
        RT_ABSORB_CASE(8)
        default: break;
    }
#undef RT_ABSORB_CASE
    rt_timer_end(ctx, "absorb");
    RT_HIP(hipGetLastError());
    if (Q || absorbed) {
        rt_finalize_partials(ctx, nb, Q, absorbed);
        RT_HIP(hipGetLastError());
    }
    return RT_OK;
}
