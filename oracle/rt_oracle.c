/*
 * Reference (oracle) implementation of the particle-based M1 photon transport
 * step of Gear-RT -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 C.  Every function is a direct transcription of a
 * definition of the thesis (arXiv:2302.12727), cited by part, chapter and
 * equation label.  There is no blocking, fusion or reordering beyond the
 * definitions: each per-particle sum is a loop over that particle's neighbour
 * list in increasing partner index order.  OpenMP only distributes independent
 * particles over threads; results do not depend on the thread count.
 *
 * Only the tests, the smoke check and the CPU baseline of the benchmark may
 * load this library.  It shares no code with the HIP library.
 *
 * Readings of points the thesis leaves open are marked "(reading)".
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Kernel: cubic B-spline, Part II "Partition of unity", eq:cubic-spline-kernel.
 * q = r/H; W = sigma/H^3 * w(q), sigma = 16/pi in three dimensions.
 * At q = 0 the first branch is taken (w(0) = 1/2, by continuity).            */
double orc_w(double q)
{
    if (q <= 0.5) {
        double a = 1.0 - q, b = 0.5 - q;
        return a * a * a - 4.0 * b * b * b;
    }
    if (q < 1.0) {
        double a = 1.0 - q;
        return a * a * a;
    }
    return 0.0;
}

/* dw/dq of the same polynomial pieces. */
double orc_dw(double q)
{
    if (q <= 0.5) {
        double a = 1.0 - q, b = 0.5 - q;
        return -3.0 * a * a + 12.0 * b * b;
    }
    if (q < 1.0) {
        double a = 1.0 - q;
        return -3.0 * a * a;
    }
    return 0.0;
}

double orc_W(double r, double H)
{
    return (16.0 / ORC_PI) / (H * H * H) * orc_w(r / H);
}

/* Periodic minimum-image separation x_b - x_a in a box of side L
 * (reading: the transport tests of the thesis stay away from boundaries;
 * periodic boxes use the nearest image). */
static void sep(const double *xa, const double *xb, const double *box, double *s)
{
    for (int d = 0; d < 3; ++d) {
        double v = xb[d] - xa[d];
        if (box[d] > 0.0) v -= box[d] * nearbyint(v / box[d]);
        s[d] = v;
    }
}

/* ------------------------------------------------------------------------ */
/* Smoothing length.  Part II "Neighbor search", eq:number-of-neighbors:
 * N_ngb = (4 pi/3) (kappa eta)^3 with kappa = H/h.  The smoothing length of a
 * particle is the root of  g(h) = h^3 * sum_j W(r_j, kappa h) - eta^3  over
 * the given candidate distances (reading: number density estimated with the
 * kernel sum, self term included by the caller for gas particles).  Solved by
 * Newton-Raphson safeguarded by bisection, as the thesis prescribes.
 *
 * dist: n rows of k candidate distances, ascending.  A row is valid for any
 * h <= dist[k-1]/kappa.  status[i]: 0 converged, 1 candidate set too small,
 * 2 no convergence in 200 iterations.                                        */
static void g_and_dg(const double *d, int32_t k, double h, double kappa,
                     double eta3, double *g, double *dg)
{
    const double pref = (16.0 / ORC_PI) / (kappa * kappa * kappa);
    double s = 0.0, ds = 0.0;
    const double H = kappa * h;
    for (int32_t m = 0; m < k; ++m) {
        double q = d[m] / H;
        if (q >= 1.0) break;
        s += orc_w(q);
        ds += orc_dw(q) * (-q / h);
    }
    *g = pref * s - eta3;
    *dg = pref * ds;
}

int32_t orc_solve_h(int64_t n, int32_t k, const double *dist, double eta,
                    double kappa, double *h_out, int32_t *status, int32_t *iters)
{
    const double eta3 = eta * eta * eta;
    const double nngb = 4.0 * ORC_PI / 3.0 * pow(kappa * eta, 3.0);
    int32_t bad = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : bad)
    for (int64_t i = 0; i < n; ++i) {
        const double *d = dist + i * (int64_t)k;
        double hi = d[k - 1] / kappa, lo = 0.0, g, dg;
        status[i] = 0;
        g_and_dg(d, k, hi, kappa, eta3, &g, &dg);
        if (!(g >= 0.0)) { status[i] = 1; h_out[i] = hi; iters[i] = 0; ++bad; continue; }
        int32_t guess = (int32_t)nngb;
        if (guess > k - 1) guess = k - 1;
        double h = d[guess] / kappa;
        if (!(h > lo && h < hi)) h = 0.5 * (lo + hi);
        int32_t it = 0, ok = 0;
        for (it = 0; it < 200; ++it) {
            g_and_dg(d, k, h, kappa, eta3, &g, &dg);
            if (g == 0.0) { ok = 1; break; }
            if (g < 0.0) lo = h; else hi = h;
            double hn = (dg > 0.0) ? h - g / dg : -1.0;
            if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
            if (fabs(hn - h) <= 4.0 * 2.220446049250313e-16 * h ||
                hi - lo <= 4.0 * 2.220446049250313e-16 * hi) {
                h = hn; ok = 1; break;
            }
            h = hn;
        }
        h_out[i] = h;
        iters[i] = it;
        if (!ok) { status[i] = 2; ++bad; }
    }
    return bad;
}

/* ------------------------------------------------------------------------ */
/* Gather lists G(i) = { j != i : r_ij < H_i } taken from k-nearest candidate
 * rows (idx/dist as returned by a k-d tree query).  Two passes: counts, then
 * fill; ptr has n+1 entries.  Entries of a row are sorted by partner index.  */
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

int64_t orc_gather_count(int64_t n, int32_t k, const int64_t *idx, const double *dist,
                         const double *H, int64_t *ptr)
{
    ptr[0] = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int32_t m = 0; m < k; ++m) {
            int64_t j = idx[i * k + m];
            if (j != i && dist[i * k + m] < H[i]) ++c;
        }
        ptr[i + 1] = ptr[i] + c;
    }
    return ptr[n];
}

void orc_gather_fill(int64_t n, int32_t k, const int64_t *idx, const double *dist,
                     const double *H, const int64_t *ptr, int64_t *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t o = ptr[i];
        for (int32_t m = 0; m < k; ++m) {
            int64_t j = idx[i * k + m];
            if (j != i && dist[i * k + m] < H[i]) out[o++] = j;
        }
        qsort(out + ptr[i], (size_t)(ptr[i + 1] - ptr[i]), sizeof(int64_t), cmp_i64);
    }
}

/* Symmetric lists N(i) = G(i) union { j : i in G(j) } = { j : r_ij < max(H_i, H_j) }
 * (reading: a pair exchanges flux whenever one of the two kernels reaches
 * the other particle, i.e. whenever A_ij is non-zero).  tptr/tidx is the
 * transpose of G; both rows are merged without duplicates.                   */
void orc_transpose(int64_t n, const int64_t *gptr, const int64_t *gidx,
                   int64_t *tptr, int64_t *tidx, int64_t *fill /* scratch n */)
{
    memset(tptr, 0, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = gptr[i]; e < gptr[i + 1]; ++e) tptr[gidx[e] + 1]++;
    for (int64_t i = 0; i < n; ++i) tptr[i + 1] += tptr[i];
    for (int64_t i = 0; i < n; ++i) fill[i] = tptr[i];
    for (int64_t i = 0; i < n; ++i)            /* increasing i => rows sorted */
        for (int64_t e = gptr[i]; e < gptr[i + 1]; ++e) tidx[fill[gidx[e]]++] = i;
}

static int64_t merge_rows(const int64_t *a, int64_t na, const int64_t *b, int64_t nb,
                          int64_t *out)
{
    int64_t i = 0, j = 0, c = 0;
    while (i < na || j < nb) {
        int64_t v;
        if (j >= nb || (i < na && a[i] < b[j])) v = a[i++];
        else if (i >= na || b[j] < a[i]) v = b[j++];
        else { v = a[i]; ++i; ++j; }
        if (out) out[c] = v;
        ++c;
    }
    return c;
}

int64_t orc_sym_count(int64_t n, const int64_t *gptr, const int64_t *gidx,
                      const int64_t *tptr, const int64_t *tidx, int64_t *sptr)
{
    sptr[0] = 0;
    for (int64_t i = 0; i < n; ++i)
        sptr[i + 1] = sptr[i] + merge_rows(gidx + gptr[i], gptr[i + 1] - gptr[i],
                                           tidx + tptr[i], tptr[i + 1] - tptr[i], NULL);
    return sptr[n];
}

void orc_sym_fill(int64_t n, const int64_t *gptr, const int64_t *gidx,
                  const int64_t *tptr, const int64_t *tidx, const int64_t *sptr,
                  int64_t *sidx)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        merge_rows(gidx + gptr[i], gptr[i + 1] - gptr[i], tidx + tptr[i],
                   tptr[i + 1] - tptr[i], sidx + sptr[i]);
}

/* ------------------------------------------------------------------------ */
/* Static geometry, Part II "Partition of unity" and "Finite volume particle
 * methods following Hopkins":
 *   omega(x_i) = sum_j W(x_i - x_j, h_i)   (eq:omega, self term included)
 *   V_i        = 1/omega(x_i)              (eq:particle-volume)
 *   psi_j(x_i) = W(r_ij, H_i) / omega(x_i) (eq:psi)
 *   E_i^{ab}   = sum_j (x_j-x_i)^a (x_j-x_i)^b psi_j(x_i)   (eq:matrix_E)
 * The inverse B_i = E_i^{-1} (eq:matrix_B) is taken by the caller.          */
void orc_geometry(int64_t n, const double *x, const double *H, const double *box,
                  const int64_t *gptr, const int64_t *gidx, double *omega,
                  double *V, double *E /* n x 9 */)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double w = orc_W(0.0, H[i]);
        for (int64_t e = gptr[i]; e < gptr[i + 1]; ++e) {
            double s[3];
            sep(x + 3 * i, x + 3 * gidx[e], box, s);
            double r = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
            w += orc_W(r, H[i]);
        }
        omega[i] = w;
        V[i] = 1.0 / w;
        double Ei[9] = {0};
        for (int64_t e = gptr[i]; e < gptr[i + 1]; ++e) {
            double s[3];
            sep(x + 3 * i, x + 3 * gidx[e], box, s);
            double r = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
            double psi = orc_W(r, H[i]) / w;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) Ei[3 * a + b] += s[a] * s[b] * psi;
        }
        memcpy(E + 9 * i, Ei, sizeof Ei);
    }
}

/* psi_tilde_j(x_i) = B_i (x_j - x_i) psi_j(x_i)   (eq:psitilde)            */
static void psitilde(const double *Bi, const double *s, double psi, double *out)
{
    for (int a = 0; a < 3; ++a)
        out[a] = (Bi[3 * a + 0] * s[0] + Bi[3 * a + 1] * s[1] + Bi[3 * a + 2] * s[2]) * psi;
}

/* ------------------------------------------------------------------------ */
/* Least-squares gradient, eq:gradient:
 *   d q / d x^a |_i = sum_j (q_j - q_i) psi_tilde_j^a(x_i)
 * over the gather neighbours of i, for every group and q in (E, Fx, Fy, Fz).
 * U is n x G x 4, dU is n x G x 4 x 3.                                       */
void orc_gradient(int64_t n, int32_t G, const double *x, const double *H,
                  const double *V, const double *B, const double *box,
                  const int64_t *gptr, const int64_t *gidx, const double *U,
                  double *dU)
{
    const int64_t nq = 4 * (int64_t)G;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double *out = dU + i * nq * 3;
        for (int64_t m = 0; m < nq * 3; ++m) out[m] = 0.0;
        for (int64_t e = gptr[i]; e < gptr[i + 1]; ++e) {
            int64_t j = gidx[e];
            double s[3], pt[3];
            sep(x + 3 * i, x + 3 * j, box, s);
            double r = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
            double psi = orc_W(r, H[i]) * V[i];
            psitilde(B + 9 * i, s, psi, pt);
            for (int64_t q = 0; q < nq; ++q) {
                double dq = U[j * nq + q] - U[i * nq + q];
                for (int a = 0; a < 3; ++a) out[3 * q + a] += dq * pt[a];
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* minmod, Part I TVD flux limiters (minmod(a, b)) and eq:rt-minmod.
 * (reading: at |a| = |b| with ab > 0 both branches give the same value.)   */
double orc_minmod(double a, double b)
{
    if (a * b <= 0.0) return 0.0;
    return (fabs(a) <= fabs(b)) ? a : b;
}

/* M1 closure, Part III "The M1 closure" (eq:eddington-freq) per photon group
 * (eq:eddington-group):  P = D E,
 *   D = (1-chi)/2 I + (3 chi - 1)/2 n (x) n,  n = F/|F|,
 *   chi = (3 + 4 f^2) / (5 + 2 sqrt(4 - 3 f^2)),  f = |F|/(c E).
 * Returns the flux of the state (E, F) projected on the unit normal nh:
 *   out[0] = F . nh,  out[1..3] = c^2 P nh.
 * For F = 0 the closure reduces to D = I/3 (Appendix E).  A state with E = 0
 * carries no flux.                                                            */
void orc_m1_flux(const double *q, const double *nh, double c, double *out)
{
    double E = q[0];
    const double *F = q + 1;
    if (!(E > 0.0)) { out[0] = out[1] = out[2] = out[3] = 0.0; return; }
    double Fn = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
    double D[9];
    if (Fn > 0.0) {
        double f = Fn / (c * E);
        double chi = (3.0 + 4.0 * f * f) / (5.0 + 2.0 * sqrt(4.0 - 3.0 * f * f));
        double nF[3] = {F[0] / Fn, F[1] / Fn, F[2] / Fn};
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                D[3 * a + b] = (a == b ? 0.5 * (1.0 - chi) : 0.0) +
                               0.5 * (3.0 * chi - 1.0) * nF[a] * nF[b];
    } else {
        for (int a = 0; a < 9; ++a) D[a] = 0.0;
        D[0] = D[4] = D[8] = 1.0 / 3.0;
    }
    out[0] = F[0] * nh[0] + F[1] * nh[1] + F[2] * nh[2];
    for (int a = 0; a < 3; ++a)
        out[1 + a] = c * c * E * (D[3 * a + 0] * nh[0] + D[3 * a + 1] * nh[1] + D[3 * a + 2] * nh[2]);
}

/* Face-state guard (reading: the thesis sets negative energy densities to
 * zero; a state with E = 0 gets F = 0, and a flux above the free-streaming
 * limit |F| = cE is scaled back onto it).  Returns bit 0 if E was clipped,
 * bit 1 if F was rescaled.                                                   */
static int guard_state(double *q, double c)
{
    int fired = 0;
    if (q[0] < 0.0) { q[0] = 0.0; fired |= 1; }
    if (q[0] == 0.0) { q[1] = q[2] = q[3] = 0.0; return fired; }
    double Fn = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double lim = c * q[0];
    if (Fn > lim) {
        double sc = lim / Fn;
        q[1] *= sc; q[2] *= sc; q[3] *= sc;
        fired |= 2;
    }
    return fired;
}

/* GLF Riemann solver, eq:riemann-GLF:
 *   Phi = (Flux_L + Flux_R)/2 - c/2 (U_R - U_L)
 * with the fluxes projected on the unit normal nh of the effective surface. */
void orc_glf(const double *qL, const double *qR, const double *nh, double c, double *phi)
{
    double fL[4], fR[4];
    orc_m1_flux(qL, nh, c, fL);
    orc_m1_flux(qR, nh, c, fR);
    for (int m = 0; m < 4; ++m) phi[m] = 0.5 * (fL[m] + fR[m]) - 0.5 * c * (qR[m] - qL[m]);
}

/* HLL Riemann solver, eq:riemann-HLL:
 *   Phi = (l+ Flux_L - l- Flux_R + l+ l- (U_R - U_L)) / (l+ - l-),
 *   l+ = max(0, l_max), l- = min(0, l_min),
 * l_min, l_max the extreme eigenvalues of the flux Jacobian along nh.  They
 * depend on the reduced flux f = |F|/(cE) and the angle between F and the
 * interface only, and are tabulated and interpolated, as the thesis does
 * (table in units of c).  Readings: the table is uniform in f on [0, 1] (nf
 * nodes) and in mu = cos(theta) on [-1, 1] (nmu nodes), [i][j][2] = (l_min,
 * l_max) at (f_i, mu_j), interpolated bilinearly; a state with no flux
 * (E = 0 or F = 0) is looked up at f = 0; l_max is the larger of the two face
 * states' and l_min the smaller (the wave speeds must bound both states).    */
static void hll_speeds(const double *q, const double *nh, double c, const double *tab,
                       int32_t nf, int32_t nmu, double *lmin, double *lmax)
{
    double E = q[0];
    double Fn = sqrt(q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    double f = 0.0, mu = 0.0;
    if (E > 0.0 && Fn > 0.0) {
        f = Fn / (c * E);
        if (f > 1.0) f = 1.0;
        mu = (q[1] * nh[0] + q[2] * nh[1] + q[3] * nh[2]) / Fn;
        if (mu > 1.0) mu = 1.0;
        if (mu < -1.0) mu = -1.0;
    }
    double x = f * (nf - 1), y = 0.5 * (mu + 1.0) * (nmu - 1);
    int32_t i = (int32_t)x, j = (int32_t)y;
    if (i > nf - 2) i = nf - 2;
    if (j > nmu - 2) j = nmu - 2;
    double tx = x - i, ty = y - j;
    for (int k = 0; k < 2; ++k) {
        double v00 = tab[((int64_t)i * nmu + j) * 2 + k];
        double v10 = tab[((int64_t)(i + 1) * nmu + j) * 2 + k];
        double v01 = tab[((int64_t)i * nmu + j + 1) * 2 + k];
        double v11 = tab[((int64_t)(i + 1) * nmu + j + 1) * 2 + k];
        double v = (1.0 - tx) * (1.0 - ty) * v00 + tx * (1.0 - ty) * v10 +
                   (1.0 - tx) * ty * v01 + tx * ty * v11;
        if (k == 0) *lmin = c * v; else *lmax = c * v;
    }
}

void orc_hll(const double *qL, const double *qR, const double *nh, double c,
             const double *tab, int32_t nf, int32_t nmu, double *phi)
{
    double fL[4], fR[4], a0, a1, b0, b1;
    orc_m1_flux(qL, nh, c, fL);
    orc_m1_flux(qR, nh, c, fR);
    hll_speeds(qL, nh, c, tab, nf, nmu, &a0, &a1);
    hll_speeds(qR, nh, c, tab, nf, nmu, &b0, &b1);
    double lmax = a1 > b1 ? a1 : b1, lmin = a0 < b0 ? a0 : b0;
    double lp = lmax > 0.0 ? lmax : 0.0, lm = lmin < 0.0 ? lmin : 0.0;
    if (!(lp - lm > 0.0)) {
        for (int m = 0; m < 4; ++m) phi[m] = 0.5 * (fL[m] + fR[m]);
        return;
    }
    for (int m = 0; m < 4; ++m)
        phi[m] = (lp * fL[m] - lm * fR[m] + lp * lm * (qR[m] - qL[m])) / (lp - lm);
}

/* Effective surface of the Hopkins formulation, eq:HopkinsAij:
 *   A_kl = V_k psi_tilde_l(x_k) - V_l psi_tilde_k(x_l).                      */
void orc_surface(const double *xk, const double *xl, double Hk, double Hl, double Vk,
                 double Vl, const double *Bk, const double *Bl, const double *box,
                 double *A)
{
    double s[3], ms[3], tl[3], tk[3];
    sep(xk, xl, box, s);
    ms[0] = -s[0]; ms[1] = -s[1]; ms[2] = -s[2];
    double r = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    psitilde(Bk, s, orc_W(r, Hk) * Vk, tl);    /* psi_tilde_l(x_k) */
    psitilde(Bl, ms, orc_W(r, Hl) * Vl, tk);   /* psi_tilde_k(x_l) */
    for (int a = 0; a < 3; ++a) A[a] = Vk * tl[a] - Vl * tk[a];
}

/* ------------------------------------------------------------------------ */
/* Ivanova effective surfaces, Part II eq:IvanovaAij:
 *   A_ij = V_i grad psi_j(x_i) - V_j grad psi_i(x_j),
 * with the analytic gradients of the partition of unity of the appendix
 * "Full Expressions For Partitions of Unity And Their Gradients":
 *   grad psi_j(x_i) = grad W_j(x_i) / omega_i
 *                     - W(r_ij, H_i) sum_k grad W_k(x_i) / omega_i^2,
 *   grad W_j(x_i)   = (sigma / H_i^4) w'(r_ij / H_i) (x_i - x_j) / r_ij,
 * the kernel evaluated with particle i's compact support radius H_i (the
 * appendix holds h at h(x_i) = h_i), the sum over the gather neighbours of i
 * (r_ik < H_i; the self term has no gradient), and 1/omega_i = V_i.         */
static void grad_W(const double *xi, const double *xj, double Hi, const double *box,
                   double *out)
{
    double s[3];
    sep(xi, xj, box, s);                      /* s = x_j - x_i */
    double r = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    if (!(r > 0.0)) { out[0] = out[1] = out[2] = 0.0; return; }
    double f = (16.0 / ORC_PI) / (Hi * Hi * Hi * Hi) * orc_dw(r / Hi) / r;
    for (int a = 0; a < 3; ++a) out[a] = -f * s[a];
}

/* gsum[i] = sum_k grad W_k(x_i) over the gather neighbours of i            */
void orc_ivanova_sums(int64_t n, const double *x, const double *H, const double *box,
                      const int64_t *gptr, const int64_t *gidx, double *gsum)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        double g[3] = {0.0, 0.0, 0.0}, d[3];
        for (int64_t e = gptr[i]; e < gptr[i + 1]; ++e) {
            grad_W(x + 3 * i, x + 3 * gidx[e], H[i], box, d);
            for (int a = 0; a < 3; ++a) g[a] += d[a];
        }
        for (int a = 0; a < 3; ++a) gsum[3 * i + a] = g[a];
    }
}

/* grad psi_j(x_i) (zero beyond the support of W(., H_i))                    */
void orc_grad_psi(const double *xi, const double *xj, double Hi, double Vi,
                  const double *gsum_i, const double *box, double *out)
{
    double s[3], gW[3];
    sep(xi, xj, box, s);
    double r = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
    grad_W(xi, xj, Hi, box, gW);
    double W = orc_W(r, Hi);
    for (int a = 0; a < 3; ++a) out[a] = Vi * gW[a] - Vi * Vi * W * gsum_i[a];
}

void orc_surface_ivanova(const double *xk, const double *xl, double Hk, double Hl, double Vk,
                         double Vl, const double *gk, const double *gl, const double *box,
                         double *A)
{
    double pl[3], pk[3];
    orc_grad_psi(xk, xl, Hk, Vk, gk, box, pl);     /* grad psi_l(x_k) */
    orc_grad_psi(xl, xk, Hl, Vl, gl, box, pk);     /* grad psi_k(x_l) */
    for (int a = 0; a < 3; ++a) A[a] = Vk * pl[a] - Vl * pk[a];
}

/* ------------------------------------------------------------------------ */
/* One transport step, Part III "Second step: transport":
 *   U_k(t + dt) = U_k(t) - (1/V_k) sum_l dt Flux_kl . A_kl
 * (eq:transport-update-explicit with one global time step) where Flux_kl is
 * the GLF solution of the Riemann problem between the states extrapolated to
 * the interface x_kl = x_k + h_k/(h_k+h_l) (x_l - x_k) (eq:rt-riemann-problem),
 * particle k being the left state.  Slopes are limited with minmod (reading:
 * the two gradients are projected on the pair separation s = x_l - x_k and the
 * limited slope m = minmod(grad q_k . s, grad q_l . s) replaces both, so
 *   q_L = q_k + h_k/(h_k+h_l) m,   q_R = q_l - h_l/(h_k+h_l) m).
 * The face states are guarded (guard_state) before the solver; after the
 * update the new state is guarded again and the energy this adds is booked.
 *
 * counts[4] (summed over the step): [0] face states with E clipped,
 * [1] face states with F rescaled, [2] updated states with E clipped,
 * [3] updated states with F rescaled.  ledger[G]: sum_k V_k * (energy density
 * added by clipping E < 0 of the updated state).                            */
static void transport_core(int64_t n, int32_t G, const double *x, const double *h,
                           const double *H, const double *V, const double *B,
                           const double *box, const int64_t *sptr, const int64_t *sidx,
                           double c, double dt, const double *U, const double *dU,
                           double *Uout, int64_t *counts, double *ledger,
                           const double *tab, int32_t nf, int32_t nmu, const double *gsum);

void orc_transport(int64_t n, int32_t G, const double *x, const double *h,
                   const double *H, const double *V, const double *B,
                   const double *box, const int64_t *sptr, const int64_t *sidx,
                   double c, double dt, const double *U, const double *dU, double *Uout,
                   int64_t *counts, double *ledger)
{
    transport_core(n, G, x, h, H, V, B, box, sptr, sidx, c, dt, U, dU, Uout, counts, ledger,
                   NULL, 0, 0, NULL);
}

/* The same step with the HLL solver (table as orc_hll) instead of GLF.      */
void orc_transport_hll(int64_t n, int32_t G, const double *x, const double *h,
                       const double *H, const double *V, const double *B,
                       const double *box, const int64_t *sptr, const int64_t *sidx,
                       double c, double dt, const double *U, const double *dU, double *Uout,
                       int64_t *counts, double *ledger, const double *tab, int32_t nf,
                       int32_t nmu)
{
    transport_core(n, G, x, h, H, V, B, box, sptr, sidx, c, dt, U, dU, Uout, counts, ledger,
                   tab, nf, nmu, NULL);
}

/* The same step with the Ivanova surfaces (gsum from orc_ivanova_sums) in
 * place of the Hopkins ones, GLF (tab NULL) or HLL.                         */
void orc_transport_ivanova(int64_t n, int32_t G, const double *x, const double *h,
                           const double *H, const double *V, const double *B,
                           const double *box, const int64_t *sptr, const int64_t *sidx,
                           double c, double dt, const double *U, const double *dU,
                           double *Uout, int64_t *counts, double *ledger, const double *tab,
                           int32_t nf, int32_t nmu, const double *gsum)
{
    transport_core(n, G, x, h, H, V, B, box, sptr, sidx, c, dt, U, dU, Uout, counts, ledger,
                   tab, nf, nmu, gsum);
}

static void transport_core(int64_t n, int32_t G, const double *x, const double *h,
                           const double *H, const double *V, const double *B,
                           const double *box, const int64_t *sptr, const int64_t *sidx,
                           double c, double dt, const double *U, const double *dU,
                           double *Uout, int64_t *counts, double *ledger,
                           const double *tab, int32_t nf, int32_t nmu, const double *gsum)
{
    const int64_t nq = 4 * (int64_t)G;
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    double *led = (double *)calloc((size_t)n * (size_t)G, sizeof(double));
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : c0, c1, c2, c3)
    for (int64_t k = 0; k < n; ++k) {
        double *acc = (double *)calloc((size_t)nq, sizeof(double));
        for (int64_t e = sptr[k]; e < sptr[k + 1]; ++e) {
            int64_t l = sidx[e];
            double A[3], s[3];
            if (gsum)
                orc_surface_ivanova(x + 3 * k, x + 3 * l, H[k], H[l], V[k], V[l],
                                    gsum + 3 * k, gsum + 3 * l, box, A);
            else
                orc_surface(x + 3 * k, x + 3 * l, H[k], H[l], V[k], V[l], B + 9 * k,
                            B + 9 * l, box, A);
            double An = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
            if (!(An > 0.0)) continue;
            double nh[3] = {A[0] / An, A[1] / An, A[2] / An};
            sep(x + 3 * k, x + 3 * l, box, s);
            double wk = h[k] / (h[k] + h[l]);
            double wl = h[l] / (h[k] + h[l]);
            for (int32_t g = 0; g < G; ++g) {
                double qL[4], qR[4], phi[4];
                for (int m = 0; m < 4; ++m) {
                    const double *gk = dU + (k * nq + 4 * g + m) * 3;
                    const double *gl = dU + (l * nq + 4 * g + m) * 3;
                    double dk = gk[0] * s[0] + gk[1] * s[1] + gk[2] * s[2];
                    double dl = gl[0] * s[0] + gl[1] * s[1] + gl[2] * s[2];
                    double mm = orc_minmod(dk, dl);
                    qL[m] = U[k * nq + 4 * g + m] + wk * mm;
                    qR[m] = U[l * nq + 4 * g + m] - wl * mm;
                }
                int fl = guard_state(qL, c), fr = guard_state(qR, c);
                c0 += (fl & 1) + (fr & 1);
                c1 += ((fl >> 1) & 1) + ((fr >> 1) & 1);
                if (tab) orc_hll(qL, qR, nh, c, tab, nf, nmu, phi);
                else orc_glf(qL, qR, nh, c, phi);
                for (int m = 0; m < 4; ++m) acc[4 * g + m] += An * phi[m];
            }
        }
        for (int32_t g = 0; g < G; ++g) {
            double q[4];
            for (int m = 0; m < 4; ++m) q[m] = U[k * nq + 4 * g + m] - dt / V[k] * acc[4 * g + m];
            double Epre = q[0];
            int f = guard_state(q, c);
            if (f & 1) { c2++; led[k * G + g] = -Epre * V[k]; }
            c3 += (f >> 1) & 1;
            for (int m = 0; m < 4; ++m) Uout[k * nq + 4 * g + m] = q[m];
        }
        free(acc);
    }
    counts[0] += c0; counts[1] += c1; counts[2] += c2; counts[3] += c3;
    for (int32_t g = 0; g < G; ++g) {
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k) s += led[k * G + g];
        ledger[g] += s;
    }
    free(led);
}

/* ------------------------------------------------------------------------ */
/* Injection, Part III "First step: injection":
 *   E_g(t + dt) = E_g(t) + dt * sum_s xi_sg L_s / V_g
 * with xi_sg = mu_a psi(x_s - x_g, h_s) and the octant correction
 * mu_a = sum_b w_b / (q_nz w_a)  (eq:isotropy-correction-with-zero).
 * (reading: sources give luminosities; dividing by V_g turns the energy
 * dt xi L into an energy density so that sum_g V_g dE_g = dt L exactly.)
 * Entries are applied in the given order (sorted by gas, then source).      */
void orc_inject(int64_t nent, int32_t G, const int64_t *src, const int64_t *gas,
                const double *xi, const double *V, const double *L, double dt,
                double *U)
{
    for (int64_t e = 0; e < nent; ++e) {
        int64_t s = src[e], g = gas[e];
        for (int32_t grp = 0; grp < G; ++grp)
            U[(g * G + grp) * 4] += dt * xi[e] * L[s * G + grp] / V[g];
    }
}

/* Injection weights of one source: psi_sg = W(r_sg, H_s) / sum_g' W(r_sg', H_s)
 * over the gas particles within H_s; octant a(g) from the signs of
 * x_g - x_s (components >= 0 count as "+", reading), w_a = sum_{g in a} psi_sg,
 * q_nz = number of octants holding particles, xi_sg = mu_a psi_sg.           */
int32_t orc_source_weights(int32_t m, const double *xs, const double *xg /* m x 3 */,
                           double Hs, const double *box, double *xi)
{
    double wsum = 0.0, wa[8] = {0};
    int cnt[8] = {0};
    int *oct = (int *)malloc(sizeof(int) * (size_t)(m > 0 ? m : 1));
    for (int32_t e = 0; e < m; ++e) {
        double s[3];
        sep(xs, xg + 3 * e, box, s);
        double r = sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]);
        xi[e] = orc_W(r, Hs);
        wsum += xi[e];
        oct[e] = (s[0] >= 0.0) | ((s[1] >= 0.0) << 1) | ((s[2] >= 0.0) << 2);
    }
    if (!(wsum > 0.0)) { free(oct); return -1; }
    for (int32_t e = 0; e < m; ++e) {
        xi[e] /= wsum;               /* psi_sg */
        if (xi[e] > 0.0) { wa[oct[e]] += xi[e]; cnt[oct[e]]++; }
    }
    int qnz = 0;
    double wtot = 0.0;
    for (int a = 0; a < 8; ++a) if (cnt[a] > 0) { qnz++; wtot += wa[a]; }
    for (int32_t e = 0; e < m; ++e) {
        if (xi[e] > 0.0) xi[e] *= wtot / (qnz * wa[oct[e]]);
    }
    free(oct);
    return qnz;
}

/* ------------------------------------------------------------------------ */
/* Photon budget Q_g = sum_k V_k E_kg with Neumaier-compensated summation.   */
void orc_photon_total(int64_t n, int32_t G, const double *V, const double *U, double *Q)
{
    for (int32_t g = 0; g < G; ++g) {
        double s = 0.0, comp = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double v = V[k] * U[(k * G + g) * 4];
            double t = s + v;
            if (fabs(s) >= fabs(v)) comp += (s - t) + v;
            else comp += (v - t) + s;
            s = t;
        }
        Q[g] = s + comp;
    }
}

/* Global time step, eq:rt-cfl: dt = C_cfl * min_i dx_i / c with
 * dx_i = (V_i / (4 pi/3))^{1/3} (reading: one global step, see the text on
 * individual time steps for the general case).                              */
double orc_dt(int64_t n, const double *V, double cfl, double c)
{
    double m = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        double dx = cbrt(V[i] / (4.0 * ORC_PI / 3.0));
        if (dx < m) m = dx;
    }
    return cfl * m / c;
}

/* ------------------------------------------------------------------------ */
/* Individual time steps (Part II "Individual time steps",
 * eq:meshless-explicit-individual-timesteps; Part III eq:transport-update-
 * explicit, whose exchanges are time integrated with min{dt_k, dt_l}; the
 * limiter of Part III "Dynamic Sub-Cycling": interacting particles differ by at
 * most a factor 4 in time step).
 *
 * Time bins: dt_i = dtmin 2^b_i, b_i the largest n <= nmax with
 * dtmin 2^n <= C_cfl dx_i / c (eq:rt-cfl), then lowered until every
 * interacting pair has |b_k - b_l| <= 2 (the greatest such assignment).     */
void orc_bins(int64_t n, const double *V, double cfl, double c, double dtmin, int32_t nmax,
              const int64_t *sptr, const int64_t *sidx, int32_t *bin)
{
    for (int64_t i = 0; i < n; ++i) {
        double tau = cfl * cbrt(V[i] / (4.0 * ORC_PI / 3.0)) / c;
        int32_t b = 0;
        while (b < nmax && dtmin * ldexp(1.0, b + 1) <= tau) ++b;
        bin[i] = b;
    }
    int changed = 1;
    while (changed) {
        changed = 0;
        for (int64_t i = 0; i < n; ++i) {
            int32_t m = bin[i];
            for (int64_t e = sptr[i]; e < sptr[i + 1]; ++e) {
                int32_t lim = bin[sidx[e]] + 2;
                if (lim < m) m = lim;
            }
            if (m < bin[i]) { bin[i] = m; changed = 1; }
        }
    }
}

/* Particle i ends a step at the end of tick t (time (t+1) dtmin) when
 * (t+1) is a multiple of 2^b_i.                                             */
static int orc_active(int64_t t, int32_t b) { return ((t + 1) % ((int64_t)1 << b)) == 0; }

/* Injection for the particles that end a step in tick t, each with its own
 * dt_g: E_g += dt_g sum_s xi_sg L_s / V_g.                                  */
void orc_inject_binned(int64_t nent, int32_t G, const int64_t *src, const int64_t *gas,
                       const double *xi, const double *V, const double *L, double dtmin,
                       const int32_t *bin, int64_t t, double *U)
{
    for (int64_t e = 0; e < nent; ++e) {
        int64_t s = src[e], g = gas[e];
        if (!orc_active(t, bin[g])) continue;
        double dtg = dtmin * ldexp(1.0, bin[g]);
        for (int32_t grp = 0; grp < G; ++grp)
            U[(g * G + grp) * 4] += dtg * xi[e] * L[s * G + grp] / V[g];
    }
}

/* Transport of tick t.  Every pair whose smaller bin ends a step in this tick
 * exchanges dt_kl |A| Phi_kl, dt_kl = dtmin 2^min(b_k, b_l), computed from the
 * current states U and the stored gradients dU (as orc_transport), into the
 * flux sums acc of both particles (each particle sums its own side).  A
 * particle that ends a step applies U_k - acc_k / V_k, is guarded as in
 * orc_transport, and clears acc_k; the others keep accumulating.  Uout gets
 * the new states of the active particles and U of the others.  gsum (from
 * orc_ivanova_sums) selects the Ivanova surfaces, NULL the Hopkins ones.    */
void orc_transport_binned(int64_t n, int32_t G, const double *x, const double *h,
                          const double *H, const double *V, const double *B,
                          const double *box, const int64_t *sptr, const int64_t *sidx,
                          double c, double dtmin, const int32_t *bin, int64_t t,
                          const double *U, const double *dU, double *acc, double *Uout,
                          int64_t *counts, double *ledger, const double *tab, int32_t nf,
                          int32_t nmu, const double *gsum)
{
    const int64_t nq = 4 * (int64_t)G;
    int64_t c0 = 0, c1 = 0, c2 = 0, c3 = 0;
    double *led = (double *)calloc((size_t)n * (size_t)G, sizeof(double));
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : c0, c1, c2, c3)
    for (int64_t k = 0; k < n; ++k) {
        double *ak = acc + k * nq;
        for (int64_t e = sptr[k]; e < sptr[k + 1]; ++e) {
            int64_t l = sidx[e];
            int32_t bmin = bin[k] < bin[l] ? bin[k] : bin[l];
            if (!orc_active(t, bmin)) continue;
            double dtkl = dtmin * ldexp(1.0, bmin);
            double A[3], s[3];
            if (gsum)
                orc_surface_ivanova(x + 3 * k, x + 3 * l, H[k], H[l], V[k], V[l],
                                    gsum + 3 * k, gsum + 3 * l, box, A);
            else
                orc_surface(x + 3 * k, x + 3 * l, H[k], H[l], V[k], V[l], B + 9 * k,
                            B + 9 * l, box, A);
            double An = sqrt(A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
            if (!(An > 0.0)) continue;
            double nh[3] = {A[0] / An, A[1] / An, A[2] / An};
            sep(x + 3 * k, x + 3 * l, box, s);
            double wk = h[k] / (h[k] + h[l]);
            double wl = h[l] / (h[k] + h[l]);
            for (int32_t g = 0; g < G; ++g) {
                double qL[4], qR[4], phi[4];
                for (int m = 0; m < 4; ++m) {
                    const double *gk = dU + (k * nq + 4 * g + m) * 3;
                    const double *gl = dU + (l * nq + 4 * g + m) * 3;
                    double dk = gk[0] * s[0] + gk[1] * s[1] + gk[2] * s[2];
                    double dl = gl[0] * s[0] + gl[1] * s[1] + gl[2] * s[2];
                    double mm = orc_minmod(dk, dl);
                    qL[m] = U[k * nq + 4 * g + m] + wk * mm;
                    qR[m] = U[l * nq + 4 * g + m] - wl * mm;
                }
                int fl = guard_state(qL, c), fr = guard_state(qR, c);
                c0 += (fl & 1) + (fr & 1);
                c1 += ((fl >> 1) & 1) + ((fr >> 1) & 1);
                if (tab) orc_hll(qL, qR, nh, c, tab, nf, nmu, phi);
                else orc_glf(qL, qR, nh, c, phi);
                for (int m = 0; m < 4; ++m) ak[4 * g + m] += dtkl * An * phi[m];
            }
        }
        for (int32_t g = 0; g < G; ++g) {
            double q[4];
            if (!orc_active(t, bin[k])) {
                for (int m = 0; m < 4; ++m) Uout[k * nq + 4 * g + m] = U[k * nq + 4 * g + m];
                continue;
            }
            for (int m = 0; m < 4; ++m) q[m] = U[k * nq + 4 * g + m] - ak[4 * g + m] / V[k];
            double Epre = q[0];
            int f = guard_state(q, c);
            if (f & 1) { c2++; led[k * G + g] = -Epre * V[k]; }
            c3 += (f >> 1) & 1;
            for (int m = 0; m < 4; ++m) {
                Uout[k * nq + 4 * g + m] = q[m];
                ak[4 * g + m] = 0.0;
            }
        }
    }
    counts[0] += c0; counts[1] += c1; counts[2] += c2; counts[3] += c3;
    for (int32_t g = 0; g < G; ++g) {
        double s = 0.0;
        for (int64_t k = 0; k < n; ++k) s += led[k * G + g];
        ledger[g] += s;
    }
    free(led);
}

/* ------------------------------------------------------------------------ */
/* Drift correction (Part III "Dealing With Particle Drifts"): a particle
 * moved by dx carries U(x + dx) = U(x) + grad U(x) . dx per component, with
 * the gradients of eq:gradient (dU [n][G][4][3], as orc_gradient writes
 * them).  Reading: the moved state is guarded like the updated state of a
 * transport step (guard_state); counts[2], counts[3] and ledger[G] are
 * accumulated as there.                                                     */
void orc_drift(int64_t n, int32_t G, const double *U, const double *dU, const double *dx,
               const double *V, double c, double *Uout, int64_t *counts, double *ledger)
{
    for (int32_t g = 0; g < G; ++g) {
        double led = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double q[4];
            for (int m = 0; m < 4; ++m) {
                const double *gr = dU + ((k * G + g) * 4 + m) * 3;
                q[m] = U[(k * G + g) * 4 + m] + gr[0] * dx[3 * k] + gr[1] * dx[3 * k + 1] +
                       gr[2] * dx[3 * k + 2];
            }
            double Epre = q[0];
            int f = guard_state(q, c);
            if (f & 1) { counts[2]++; led += -Epre * V[k]; }
            counts[3] += (f >> 1) & 1;
            for (int m = 0; m < 4; ++m) Uout[(k * G + g) * 4 + m] = q[m];
        }
        ledger[g] += led;
    }
}

/* ------------------------------------------------------------------------ */
/* Photon removal of the thermochemistry step (Part III "Third step:
 * Thermochemistry"): forward Euler over dt with the number densities of the
 * absorbing species averaged over the step,
 *   E_kg(t+dt) = E_kg(t) (1 - c dt sum_j sigma_gj (n_kj(t) + n_kj(t+dt))/2),
 * and the same factor on F_kg.  sigma[G][J] is the number-weighted group
 * cross section (eq:sigma_N), n_old/n_new [n][J] the densities at the two
 * ends of the step (n_new NULL: constant densities).  Reading: a factor
 * below zero (more than all photons absorbed in one step) is taken as zero.
 * absorbed[G] += sum_k V_k (E_kg(t) - E_kg(t+dt)).                          */
void orc_absorb(int64_t n, int32_t G, int32_t J, const double *V, const double *U,
                const double *n_old, const double *n_new, const double *sigma, double c,
                double dt, double *Uout, double *absorbed)
{
    for (int32_t g = 0; g < G; ++g) {
        double lost = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double kappa = 0.0;
            for (int32_t j = 0; j < J; ++j) {
                double nbar = n_new ? 0.5 * (n_old[k * J + j] + n_new[k * J + j])
                                    : n_old[k * J + j];
                kappa += sigma[g * J + j] * nbar;
            }
            double f = 1.0 - c * dt * kappa;
            if (f < 0.0) f = 0.0;
            const double *q = U + (k * G + g) * 4;
            double *o = Uout + (k * G + g) * 4;
            for (int m = 0; m < 4; ++m) o[m] = q[m] * f;
            lost += V[k] * (q[0] - o[0]);
        }
        absorbed[g] += lost;
    }
}

/* Threads of the parallel loops that follow (timing of the baseline only;
 * every loop gives the same bits with any count). */
void orc_set_num_threads(int32_t t)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int32_t orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
