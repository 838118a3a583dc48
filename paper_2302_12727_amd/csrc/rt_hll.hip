// Wave speeds of the HLL Riemann solver (Part III eq:riemann-HLL): the
// extreme eigenvalues of the Jacobian of the M1 flux (F.n, c^2 P n) with
// respect to (E, F).  They depend only on the reduced flux f = |F|/(cE) and on
// mu = cos(theta), theta the angle between F and the interface normal, and are
// tabulated in units of c on a grid uniform in f on [0, 1] and in mu on
// [-1, 1], [i][j][2] = (l_min, l_max), interpolated bilinearly in the
// transport kernel, as the thesis tabulates and interpolates them.
//
// The table is computed here on the host.  For 0 < f < 1 the Jacobian at
// E = 1, F = f e_x, n = (mu, sqrt(1 - mu^2), 0) (c = 1) has the double
// eigenvalue m = 3 f mu / (2 + sqrt(4 - 3 f^2)) (the two modes transverse to
// the plane of F and n) and two simple extreme ones, l1 + l2 = tr J - 2 m and
// l1^2 + l2^2 = tr J^2 - 2 m^2; at f = 0 the speeds are -+1/sqrt(3) and at
// f = 1 every eigenvalue is mu (free streaming).
#include <cmath>
#include <vector>

#include "rt_internal.h"

namespace {

// Jacobian of the M1 flux (division-free form: flux_v = a n + b F with
// a = E/3 - |F|^2/D, b = 3 (F.n)/D, D = 2E + R, R = sqrt(4E^2 - 3|F|^2), c = 1)
void m1_jacobian(double E, const double F[3], const double n[3], double J[4][4]) {
    const double F2 = F[0] * F[0] + F[1] * F[1] + F[2] * F[2];
    const double Fn = F[0] * n[0] + F[1] * n[1] + F[2] * n[2];
    const double R = std::sqrt(4.0 * E * E - 3.0 * F2);
    const double D = 2.0 * E + R;
    const double b = 3.0 * Fn / D;
    const double dD_dE = 2.0 + 4.0 * E / R;
    double dD_dF[3], da_dF[3], db_dF[3];
    for (int j = 0; j < 3; ++j) dD_dF[j] = -3.0 * F[j] / R;
    const double da_dE = 1.0 / 3.0 + F2 / (D * D) * dD_dE;
    const double db_dE = -3.0 * Fn / (D * D) * dD_dE;
    for (int j = 0; j < 3; ++j) {
        da_dF[j] = -2.0 * F[j] / D + F2 / (D * D) * dD_dF[j];
        db_dF[j] = 3.0 * n[j] / D - 3.0 * Fn / (D * D) * dD_dF[j];
    }
    J[0][0] = 0.0;
    for (int j = 0; j < 3; ++j) J[0][1 + j] = n[j];
    for (int i = 0; i < 3; ++i) {
        J[1 + i][0] = da_dE * n[i] + db_dE * F[i];
        for (int j = 0; j < 3; ++j)
            J[1 + i][1 + j] = da_dF[j] * n[i] + db_dF[j] * F[i] + (i == j ? b : 0.0);
    }
}

}  // namespace

std::vector<double> rt_hll_speed_table(int nf, int nmu) {
    std::vector<double> tab((size_t)nf * nmu * 2);
    for (int i = 0; i < nf; ++i) {
        const double f = (double)i / (nf - 1);
        for (int j = 0; j < nmu; ++j) {
            const double mu = -1.0 + 2.0 * j / (nmu - 1);
            double lo, hi;
            if (i == 0) {
                hi = 1.0 / std::sqrt(3.0);
                lo = -hi;
            } else if (i == nf - 1) {
                lo = hi = mu;
            } else {
                const double n[3] = {mu, std::sqrt(std::fmax(0.0, 1.0 - mu * mu)), 0.0};
                const double F[3] = {f, 0.0, 0.0};
                double J[4][4];
                m1_jacobian(1.0, F, n, J);
                double tr = 0.0, tr2 = 0.0;
                for (int a = 0; a < 4; ++a) {
                    tr += J[a][a];
                    for (int b = 0; b < 4; ++b) tr2 += J[a][b] * J[b][a];
                }
                const double m = 3.0 * f * mu / (2.0 + std::sqrt(4.0 - 3.0 * f * f));
                const double s1 = tr - 2.0 * m, s2 = tr2 - 2.0 * m * m;
                const double disc = std::fmax(2.0 * s2 - s1 * s1, 0.0);   // (l1 - l2)^2
                lo = 0.5 * (s1 - std::sqrt(disc));
                hi = 0.5 * (s1 + std::sqrt(disc));
            }
            tab[((size_t)i * nmu + j) * 2 + 0] = lo;
            tab[((size_t)i * nmu + j) * 2 + 1] = hi;
        }
    }
    return tab;
}

rt_status rt_set_riemann_impl(rt_ctx *ctx, int32_t solver) {
    if (solver == RT_HLL && !ctx->hll_table) {
        std::vector<double> tab = rt_hll_speed_table(RT_HLL_NF, RT_HLL_NMU);
        std::vector<float> tab32(tab.begin(), tab.end());
        rt_status rs = rt_alloc(ctx, (void **)&ctx->hll_table, sizeof(double) * tab.size());
        if (rs != RT_OK) return rs;
        rs = rt_alloc(ctx, (void **)&ctx->hll_table32, sizeof(float) * tab32.size());
        if (rs != RT_OK) return rs;
        RT_HIP(hipMemcpy(ctx->hll_table, tab.data(), sizeof(double) * tab.size(),
                         hipMemcpyHostToDevice));
        RT_HIP(hipMemcpy(ctx->hll_table32, tab32.data(), sizeof(float) * tab32.size(),
                         hipMemcpyHostToDevice));
    }
    ctx->solver = solver;
    return RT_OK;
}
