// Device functions of one neighbour pair, shared by the transport kernel and
// its adjoint: face guards, the M1 flux through an effective surface, minmod,
// the pair geometry, the LDS transpose of neighbour rows, and the
// vector-Jacobian products of the guard and of the flux.
#pragma once

#include "rt_internal.h"

namespace gearrt {
namespace {

// Face guard (reading of "negative energy densities are set to zero"): E < 0
// becomes 0 with F = 0, and a flux beyond the free-streaming limit is scaled
// to |F| = cE.  Returns bit0 / bit1 when the respective guard fired.
__device__ __forceinline__ int guard64(double &E, double &Fx, double &Fy, double &Fz, double c) {
    int fired = 0;
    if (E < 0.0) {
        E = 0.0;
        fired = 1;
    }
    if (E == 0.0) {
        Fx = Fy = Fz = 0.0;
        return fired;
    }
    const double F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const double lim = c * E;
    if (F2 > lim * lim) {
        const double sc = lim * rsq64(F2);
        Fx *= sc;
        Fy *= sc;
        Fz *= sc;
        fired |= 2;
    }
    return fired;
}

// Flux of a state through the (unnormalised) surface A, using the M1 closure
// (eq:eddington-group) rewritten without the 0/0 of n = F/|F| and without any
// division by E.  With f = |F|/(cE), the Eddington factor gives
//   (1 - chi)/2 = 1/3 - f^2/(2 + s),  (3 chi - 1)/(2 f^2) = 3/(2 + s),
//   s = sqrt(4 - 3 f^2);
// multiplying through by cE, with R = sqrt(4 (cE)^2 - 3 |F|^2) and
// D = 2 cE + R:
//   c^2 P A = (c^2 E/3 - c |F|^2/D) A + 3 c (F.A)/D F.
// out[0] = F.A, out[1..3] = c^2 P A.  Guarded states have |F| <= cE, so
// R >= cE; a state with E = 0 (and F = 0) has no flux (1/D replaced by 0).
__device__ __forceinline__ void m1_flux64(double E, double Fx, double Fy, double Fz, double Ax,
                                          double Ay, double Az, double c, double out[4]) {
    const double FA = Fx * Ax + Fy * Ay + Fz * Az;
    const double F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const double cE = c * E;
    const double R2 = __builtin_fma(-3.0, F2, 4.0 * cE * cE);
    const double R = R2 > 0.0 ? R2 * rsq64(R2) : 0.0;
    const double D = __builtin_fma(2.0, cE, R);
    const double iD = D > 0.0 ? rcp64(D) : 0.0;
    const double a = c * __builtin_fma(-F2, iD, cE * (1.0 / 3.0));
    const double b = 3.0 * c * FA * iD;
    out[0] = FA;
    out[1] = a * Ax + b * Fx;
    out[2] = a * Ay + b * Fy;
    out[3] = a * Az + b * Fz;
}

// HLL wave speeds of one face state (eq:riemann-HLL): the extreme eigenvalues
// of the M1 flux Jacobian along A/|A|, interpolated bilinearly in the table
// tab[RT_HLL_NF][RT_HLL_NMU] = (l_min, l_max)/c over f = |F|/(cE), clamped to
// 1, and mu = F.A/(|F||A|), clamped to [-1, 1]; a state with E <= 0 or F = 0
// is looked up at f = 0.  iAn = 1/|A|.  Every index stays in the table
// whatever the inputs (NaN compares false and fmin/fmax drop it).
__device__ __forceinline__ void hll_speeds64(double E, double Fx, double Fy, double Fz,
                                             double Ax, double Ay, double Az, double iAn,
                                             double c, const double2 *__restrict__ tab,
                                             double &lo, double &hi) {
    const double F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const double FA = Fx * Ax + Fy * Ay + Fz * Az;
    double f = 0.0, mu = 0.0;
    if (E > 0.0 && F2 > 0.0) {
        const double iF = rsq64(F2);
        f = fmin(F2 * iF * rcp64(c * E), 1.0);
        mu = fmin(fmax(FA * iF * iAn, -1.0), 1.0);
    }
    const double x = f * (RT_HLL_NF - 1), y = (mu + 1.0) * (0.5 * (RT_HLL_NMU - 1));
    const int i = max(min((int)x, RT_HLL_NF - 2), 0);
    const int j = max(min((int)y, RT_HLL_NMU - 2), 0);
    const double tx = x - i, ty = y - j;
    const double2 *t = tab + i * RT_HLL_NMU + j;
    const double2 v00 = t[0], v01 = t[1], v10 = t[RT_HLL_NMU], v11 = t[RT_HLL_NMU + 1];
    const double ux = 1.0 - tx, uy = 1.0 - ty;
    lo = c * (ux * (uy * v00.x + ty * v01.x) + tx * (uy * v10.x + ty * v11.x));
    hi = c * (ux * (uy * v00.y + ty * v01.y) + tx * (uy * v10.y + ty * v11.y));
}

// Weights of the numerical flux Phi.A = w1 F_L.A + w2 F_R.A + w3 (U_R - U_L)
// of the HLL solver (eq:riemann-HLL) from the face states' wave speeds; the
// GLF solver (eq:riemann-GLF) is w1 = w2 = 1/2, w3 = -c |A|/2.
__device__ __forceinline__ void hll_weights(double loL, double hiL, double loR, double hiR,
                                            double An, double &w1, double &w2, double &w3) {
    const double lp = fmax(fmax(hiL, hiR), 0.0), lm = fmin(fmin(loL, loR), 0.0);
    const double den = lp - lm;
    if (den > 0.0) {
        const double id = rcp64(den);
        w1 = lp * id;
        w2 = -lm * id;
        w3 = lp * lm * An * id;
    } else {
        w1 = w2 = 0.5;
        w3 = 0.0;
    }
}

// Vector-Jacobian products of the HLL wave speeds and weights (the adjoint of
// eq:riemann-HLL), with the derivative of the branch the forward takes at each
// kink: the speed a max/min selects (the first on ties), f and mu passed
// through while inside [0, 1] and [-1, 1], the table cell of the forward, and
// nothing where E or F is zero (f = mu = 0 there).
//
// hll_weights_vjp: cotangents of (loL, hiL, loR, hiR) from the cotangent sums
// S1 = m.F_L.A, S2 = m.F_R.A, S3 = m.(U_R - U_L) of the flux cotangent m.
__device__ __forceinline__ void hll_weights_vjp(double loL, double hiL, double loR, double hiR,
                                                double An, double S1, double S2, double S3,
                                                double &gloL, double &ghiL, double &gloR,
                                                double &ghiR) {
    gloL = ghiL = gloR = ghiR = 0.0;
    const double mx = hiL >= hiR ? hiL : hiR, mn = loL <= loR ? loL : loR;
    const double lp = mx > 0.0 ? mx : 0.0, lm = mn < 0.0 ? mn : 0.0;
    const double den = lp - lm;
    if (!(den > 0.0)) return;
    const double id = rcp64(den), id2 = id * id;
    // w1 = lp/den, w2 = -lm/den, w3 = lp lm |A|/den
    const double glp = (-lm * S1 + lm * S2 - An * lm * lm * S3) * id2;
    const double glm = (lp * S1 - lp * S2 + An * lp * lp * S3) * id2;
    if (mx > 0.0) (hiL >= hiR ? ghiL : ghiR) = glp;
    if (mn < 0.0) (loL <= loR ? gloL : gloR) = glm;
}
// hll_speeds64_vjp: adds to t (cotangent of the face state) the pull-back of
// the cotangents glo, ghi of the speeds hll_speeds64 returns for that state.
__device__ __forceinline__ void hll_speeds64_vjp(double E, double Fx, double Fy, double Fz,
                                                 double Ax, double Ay, double Az, double iAn,
                                                 double c, const double2 *__restrict__ tab,
                                                 double glo, double ghi, double (&t)[4]) {
    const double F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    if (!(E > 0.0 && F2 > 0.0)) return;
    const double FA = Fx * Ax + Fy * Ay + Fz * Az;
    const double iF = rsq64(F2), iE = rcp64(c * E);
    const double fr = F2 * iF * iE, mr = FA * iF * iAn;
    const double f = fmin(fr, 1.0), mu = fmin(fmax(mr, -1.0), 1.0);
    const double x = f * (RT_HLL_NF - 1), y = (mu + 1.0) * (0.5 * (RT_HLL_NMU - 1));
    const int i = max(min((int)x, RT_HLL_NF - 2), 0);
    const int j = max(min((int)y, RT_HLL_NMU - 2), 0);
    const double tx = x - i, ty = y - j;
    const double2 *tb = tab + i * RT_HLL_NMU + j;
    const double2 v00 = tb[0], v01 = tb[1], v10 = tb[RT_HLL_NMU], v11 = tb[RT_HLL_NMU + 1];
    const double ux = 1.0 - tx, uy = 1.0 - ty;
    // d(lo, hi)/dx and d(lo, hi)/dy of the bilinear form (times c)
    const double gx = glo * (uy * (v10.x - v00.x) + ty * (v11.x - v01.x)) +
                      ghi * (uy * (v10.y - v00.y) + ty * (v11.y - v01.y));
    const double gy = glo * (ux * (v01.x - v00.x) + tx * (v11.x - v10.x)) +
                      ghi * (ux * (v01.y - v00.y) + tx * (v11.y - v10.y));
    const double gf = c * gx * (RT_HLL_NF - 1), gm = c * gy * (0.5 * (RT_HLL_NMU - 1));
    if (fr <= 1.0) {            // f = |F|/(cE): df/dE = -f/E, df/dF = F/(|F| c E)
        const double k = gf * iF * iE;
        t[0] -= gf * fr * c * iE;
        t[1] += k * Fx;
        t[2] += k * Fy;
        t[3] += k * Fz;
    }
    if (mr >= -1.0 && mr <= 1.0) {   // mu = F.A/(|F||A|): dmu/dF = A/(|F||A|) - mu F/|F|^2
        const double a = gm * iF * iAn, b = gm * mr * iF * iF;
        t[1] += a * Ax - b * Fx;
        t[2] += a * Ay - b * Fy;
        t[3] += a * Az - b * Fz;
    }
}

__device__ __forceinline__ double minmod(double a, double b) {
    const double m = (fabs(a) <= fabs(b)) ? a : b;
    return (a * b > 0.0) ? m : 0.0;
}

// minmod(a, b) as the median of (a, b, 0): for a and b of one sign the median
// is the one nearer 0, otherwise 0; med3(a, b, 0) = max(min(a, b),
// min(max(a, b), 0)) takes four min/max instructions and no compare or
// select, and returns a, b or 0 exactly as minmod does.
__device__ __forceinline__ double minmod_med(double a, double b) {
    return fmax(fmin(a, b), fmin(fmax(a, b), 0.0));
}

// Face guard and M1 flux coefficients of one face state in one pass (the
// transport's inner loop): the guard of guard64 applied to q in place (the
// same bits returned), then FA = F.A and the coefficients of
// c^2 P A = a A + b F of m1_flux64, sharing |F|^2 and cE between them.  An
// E = 0 state with F != 0 takes the rescale branch with factor 0 (F -> 0, not
// counted, as guard64 does); the branches of m1_flux64 at R2 = 0 and D = 0
// (only E = 0 reaches them) become a floor at the smallest normal double,
// where F = 0 makes a = b = 0 all the same.  c3 = 3c.
__device__ __forceinline__ int face_m164(double (&q)[4], double Ax, double Ay, double Az,
                                         double c, double c3, double &FA, double &a,
                                         double &b) {
    int fired = 0;
    if (q[0] < 0.0) {
        q[0] = 0.0;
        fired = 1;
    }
    double F2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const double cE = c * q[0];
    const double lim2 = cE * cE;
    if (F2 > lim2) {
        const double sc = cE * rsq64(F2);
        q[1] *= sc;
        q[2] *= sc;
        q[3] *= sc;
        if (q[0] > 0.0) fired |= 2;
        F2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    }
    FA = q[1] * Ax + q[2] * Ay + q[3] * Az;
    const double R2 = __builtin_fma(-3.0, F2, 4.0 * lim2);
    const double R = R2 * rsq64(fmax(R2, 2.2250738585072014e-308));
    const double D = __builtin_fma(2.0, cE, R);
    const double iD = rcp64(fmax(D, 2.2250738585072014e-308));
    a = c * __builtin_fma(-F2, iD, cE * (1.0 / 3.0));
    b = c3 * FA * iD;
    return fired;
}

// Per-pair flux accumulation shared by the FP64 transport and its adjoint
// recompute: returns |A| and A in out-params, or |A| = 0 if the pair has no
// surface.
struct PairGeo {
    double sx, sy, sz, Ax, Ay, Az, An, fk, fl;
};

__device__ __forceinline__ void pair_geometry64(const double *__restrict__ rk,
                                                const double *__restrict__ rl, double box,
                                                double ibox, PairGeo &pg) {
    pg.sx = min_image(rl[0] - rk[0], box, ibox);
    pg.sy = min_image(rl[1] - rk[1], box, ibox);
    pg.sz = min_image(rl[2] - rk[2], box, ibox);
    const double r = sqrt64(pg.sx * pg.sx + pg.sy * pg.sy + pg.sz * pg.sz);
    const double wk = kern_w(r * rk[R_IH]);
    const double wl = kern_w(r * rl[R_IH]);
    // A_kl = (w_k Bv_k + w_l Bv_l) s   (eq:HopkinsAij, see the record layout)
    const double m00 = wk * rk[R_B + 0] + wl * rl[R_B + 0];
    const double m01 = wk * rk[R_B + 1] + wl * rl[R_B + 1];
    const double m02 = wk * rk[R_B + 2] + wl * rl[R_B + 2];
    const double m11 = wk * rk[R_B + 3] + wl * rl[R_B + 3];
    const double m12 = wk * rk[R_B + 4] + wl * rl[R_B + 4];
    const double m22 = wk * rk[R_B + 5] + wl * rl[R_B + 5];
    pg.Ax = m00 * pg.sx + m01 * pg.sy + m02 * pg.sz;
    pg.Ay = m01 * pg.sx + m11 * pg.sy + m12 * pg.sz;
    pg.Az = m02 * pg.sx + m12 * pg.sy + m22 * pg.sz;
    pg.An = sqrt64(pg.Ax * pg.Ax + pg.Ay * pg.Ay + pg.Az * pg.Az);
    // interface x_kl = x_k + h_k/(h_k+h_l) s  (eq:rt-riemann-problem)
    const double ih = rcp64(rk[R_H] + rl[R_H]);
    pg.fk = rk[R_H] * ih;
    pg.fl = rl[R_H] * ih;
}

// Ivanova effective surface (eq:IvanovaAij with the analytic gradients of the
// partition of unity): A_kl = V_k grad psi_l(x_k) - V_l grad psi_k(x_l) with
// grad psi_l(x_k) = V_k grad W_l(x_k) - V_k^2 W(r, H_k) g_k and
// grad W_l(x_k) = (sigma / H_k^4) w'(r / H_k) (x_k - x_l) / r, so that with
// s = x_l - x_k
//   A_kl = -(V_k^2 sigma w'_k / H_k^4 + V_l^2 sigma w'_l / H_l^4) s / r
//          - V_k^3 sigma w_k / H_k^3 g_k + V_l^3 sigma w_l / H_l^3 g_l.
// gk, gl: the kernel-gradient sums g of both particles.
__device__ __forceinline__ void pair_geometry_ivanova64(const double *__restrict__ rk,
                                                        const double *__restrict__ rl,
                                                        const double (&gk)[3],
                                                        const double (&gl)[3], double box,
                                                        double ibox, PairGeo &pg) {
    pg.sx = min_image(rl[0] - rk[0], box, ibox);
    pg.sy = min_image(rl[1] - rk[1], box, ibox);
    pg.sz = min_image(rl[2] - rk[2], box, ibox);
    const double r = sqrt64(pg.sx * pg.sx + pg.sy * pg.sy + pg.sz * pg.sz);
    const double ir = r > 0.0 ? rcp64(r) : 0.0;
    const double iHk = rk[R_IH], iHl = rl[R_IH], Vk = rk[R_V], Vl = rl[R_V];
    const double qk = r * iHk, ql = r * iHl;
    const double sk = kSigma3 * Vk * Vk * iHk * iHk * iHk, sl = kSigma3 * Vl * Vl * iHl * iHl * iHl;
    const double a = -(sk * iHk * kern_dw(qk) + sl * iHl * kern_dw(ql)) * ir;
    const double bk = sk * Vk * kern_w(qk), bl = sl * Vl * kern_w(ql);
    pg.Ax = a * pg.sx - bk * gk[0] + bl * gl[0];
    pg.Ay = a * pg.sy - bk * gk[1] + bl * gl[1];
    pg.Az = a * pg.sz - bk * gk[2] + bl * gl[2];
    pg.An = sqrt64(pg.Ax * pg.Ax + pg.Ay * pg.Ay + pg.Az * pg.Az);
    const double ih = rcp64(rk[R_H] + rl[R_H]);
    pg.fk = rk[R_H] * ih;
    pg.fl = rl[R_H] * ih;
}

// Block sum of NP per-lane values; value p goes to out[col(p)].
template <int NP, class Col>
__device__ __forceinline__ void block_reduce_store(double (&v)[NP], double *__restrict__ out,
                                                   double *smem, Col col) {
    // smem: [kBlock/64][NP]
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        double x = wave_sum(v[p]);
        if (lane == 0) smem[wv * NP + p] = x;
    }
    __syncthreads();
    if (threadIdx.x < NP) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += smem[w * NP + threadIdx.x];
        out[col((int)threadIdx.x)] = s;
    }
}

// LDS transpose of neighbour records.  A lane-per-particle gather makes every
// wave-wide load touch 64 different cache lines (one address-unit cycle each);
// instead the wave fetches the 64 records it needs in this iteration with
// coalesced loads (8 lanes per 128-byte line, 8 lines per instruction), writes
// them to its own LDS buffer, and each lane then reads its neighbour's record
// from LDS.  Records are padded to 17 doubles in LDS against bank conflicts.
constexpr int kStage = 17;

// Order LDS traffic of one wavefront: everything before is complete and
// visible to the other lanes of the wave before anything after is issued.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Copy one 16-double line per lane's neighbour (line base pointers src + 16 *
// row[m]) into the wave's stage buffer: 8 loads, each lane moving 16 bytes.
// The load and store halves are separate so that a kernel can put several
// loads in flight before it stores the first of them.
__device__ __forceinline__ void load_lines(const double *__restrict__ src, const int64_t (&row)[8],
                                           int lane, double2 (&v)[8]) {
    const int piece = lane & 7;
#pragma unroll
    for (int m = 0; m < 8; ++m)
        v[m] = *reinterpret_cast<const double2 *>(src + 16 * row[m] + 2 * piece);
}
__device__ __forceinline__ void store_lines(const double2 (&v)[8], double *sb, int lane) {
    const int piece = lane & 7, slot = lane >> 3;
    wave_lds_sync();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        double *d = sb + (8 * m + slot) * kStage + 2 * piece;
        d[0] = v[m].x;
        d[1] = v[m].y;
    }
    wave_lds_sync();
}
// Pointers to this lane's 16-byte piece of line `sel` of rows r[m] of a table
// of rows `stride` lines long, src + 16 (stride r[m] + sel) + 2 (lane % 8),
// for the 8 rows the lane helps to move.  The row offset is formed in 32 bits
// (stride r[m] < 2^31) and widened once: no 64-bit multiply per line, and the
// lines sel + 1, sel + 2, ... of the same rows are constant offsets.
__device__ __forceinline__ void row_ptrs(const double *__restrict__ src, const int32_t (&r)[8],
                                         int stride, int sel, int lane, const double *(&p)[8]) {
    const uint32_t extra = (uint32_t)sel * 16 + 2 * (lane & 7);
#pragma unroll
    for (int m = 0; m < 8; ++m)
        p[m] = src + (((size_t)(uint32_t)(r[m] * stride) << 4) + extra);
}
// Load the pieces at p[m] + 16 g (line g beyond the one p points into).
__device__ __forceinline__ void load_at(const double *const (&p)[8], int g, double2 (&v)[8]) {
#pragma unroll
    for (int m = 0; m < 8; ++m) v[m] = *reinterpret_cast<const double2 *>(p[m] + 16 * g);
}
// This lane's 16-byte pieces of line g of rows r[m] of a table of rows
// `stride` lines long, addressed either by 8 pointers (OFF32 false) or by 8
// byte offsets from the table's base (OFF32 true: the table is smaller than
// 4 GiB).  The offsets take half the registers of the pointers, and the base
// stays in scalar registers.
template <bool OFF32> struct RowLines;
template <> struct RowLines<false> {
    const double *p[8];
    __device__ __forceinline__ RowLines(const double *__restrict__ src, const int32_t (&r)[8],
                                        int stride, int lane) {
        row_ptrs(src, r, stride, 0, lane, p);
    }
    __device__ __forceinline__ void load(int g, double2 (&v)[8]) const { load_at(p, g, v); }
};
template <> struct RowLines<true> {
    const char *b;
    uint32_t o[8];
    __device__ __forceinline__ RowLines(const double *__restrict__ src, const int32_t (&r)[8],
                                        int stride, int lane)
        : b(reinterpret_cast<const char *>(src)) {
#pragma unroll
        for (int m = 0; m < 8; ++m) o[m] = (uint32_t)r[m] * (uint32_t)(128 * stride) + 16u * (lane & 7);
    }
    __device__ __forceinline__ void load(int g, double2 (&v)[8]) const {
#pragma unroll
        for (int m = 0; m < 8; ++m) v[m] = *reinterpret_cast<const double2 *>(b + o[m] + 128u * g);
    }
};
__device__ __forceinline__ void stage_lines(const double *__restrict__ src, const int64_t (&row)[8],
                                            double *sb, int lane) {
    double2 v[8];
    load_lines(src, row, lane, v);
    store_lines(v, sb, lane);
}

// Copy the 4-double row (row_stride doubles apart) of every lane's row index j
// into the wave's stage buffer: 2 loads, 2 lanes per row, 32 rows per load.
__device__ __forceinline__ void load_rows4(const double *__restrict__ src, int64_t row_stride,
                                           int64_t j, int lane, double2 (&v)[2]) {
    const int piece = lane & 1, slot = lane >> 1;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int64_t r = __shfl(j, 32 * m + slot, 64);
        v[m] = *reinterpret_cast<const double2 *>(src + row_stride * r + 2 * piece);
    }
}
__device__ __forceinline__ void store_rows4(const double2 (&v)[2], double *sb, int lane) {
    const int piece = lane & 1, slot = lane >> 1;
    wave_lds_sync();
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        double *d = sb + (32 * m + slot) * kStage + 2 * piece;
        d[0] = v[m].x;
        d[1] = v[m].y;
    }
    wave_lds_sync();
}
__device__ __forceinline__ void stage_rows4(const double *__restrict__ src, int64_t row_stride,
                                            int64_t j, double *sb, int lane) {
    double2 v[2];
    load_rows4(src, row_stride, j, lane, v);
    store_rows4(v, sb, lane);
}

// Vector-Jacobian product of guard64 at its input state q (before the guard):
// lam (cotangent of the output) is overwritten with the cotangent of q.
//   E < 0:        output constant  -> 0
//   E = 0:        F -> 0           -> (lam_E, 0)
//   |F| > cE:     F -> cE F/|F|    -> lam_E + c n.lam_F,  (cE/|F|)(I - n n^T) lam_F
//   otherwise identity.
__device__ __forceinline__ void guard64_vjp(const double q[4], double lam[4], double c) {
    const double E = q[0];
    if (E < 0.0) {
        lam[0] = lam[1] = lam[2] = lam[3] = 0.0;
        return;
    }
    if (E == 0.0) {
        lam[1] = lam[2] = lam[3] = 0.0;
        return;
    }
    const double F2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const double lim = c * E;
    if (F2 > lim * lim) {
        const double iF = rsq64(F2);
        const double nx = q[1] * iF, ny = q[2] * iF, nz = q[3] * iF;
        const double nl = nx * lam[1] + ny * lam[2] + nz * lam[3];
        const double sc = lim * iF;
        lam[0] += c * nl;
        lam[1] = sc * (lam[1] - nx * nl);
        lam[2] = sc * (lam[2] - ny * nl);
        lam[3] = sc * (lam[3] - nz * nl);
    }
}

// Vector-Jacobian product of m1_flux64 with respect to the (guarded) face
// state (E, F) for the cotangent nu = (nu0, nu_v) of (F.A, c^2 P A).  In the
// form above, flux_v = a A + b F with a = c^2 E/3 - c |F|^2/D,
// b = 3 c (F.A)/D, dD/dE = 2c + 4 c (cE)/R, dD/dF = -3 F/R.  With
// alpha = nu_v.A, beta = nu_v.F and K = c (alpha |F|^2 - 3 (F.A) beta)/D^2:
//   d/dE = alpha c^2/3 + K dD/dE
//   d/dF = (nu0 + 3 c beta/D) A + 3 c (F.A)/D nu_v - (2 c alpha/D + 3 K/R) F
// (at E = 0, where F = 0, 1/D and 1/R are replaced by 0: the one-sided limit).
// nuF, if given, receives nu . flux = nu0 (F.A) + a alpha + b beta.
__device__ __forceinline__ void m1_flux64_vjp(double E, double Fx, double Fy, double Fz, double Ax,
                                              double Ay, double Az, double c, const double nu[4],
                                              double out[4], double *nuF = nullptr) {
    const double FA = Fx * Ax + Fy * Ay + Fz * Az;
    const double F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const double cE = c * E;
    const double R2 = __builtin_fma(-3.0, F2, 4.0 * cE * cE);
    const double iR = R2 > 0.0 ? rsq64(R2) : 0.0;
    const double D = __builtin_fma(2.0, cE, R2 * iR);
    const double iD = D > 0.0 ? rcp64(D) : 0.0;
    const double al = nu[1] * Ax + nu[2] * Ay + nu[3] * Az;
    const double be = nu[1] * Fx + nu[2] * Fy + nu[3] * Fz;
    const double K = c * iD * iD * __builtin_fma(al, F2, -3.0 * FA * be);
    const double cA = __builtin_fma(3.0 * c * be, iD, nu[0]);
    const double cn = 3.0 * c * FA * iD;
    const double cF = __builtin_fma(2.0 * c * al, iD, 3.0 * K * iR);
    out[0] = __builtin_fma(al, c * c * (1.0 / 3.0), K * __builtin_fma(4.0 * c * cE, iR, 2.0 * c));
    out[1] = cA * Ax + cn * nu[1] - cF * Fx;
    out[2] = cA * Ay + cn * nu[2] - cF * Fy;
    out[3] = cA * Az + cn * nu[3] - cF * Fz;
    if (nuF) {
        const double a = c * __builtin_fma(-F2, iD, cE * (1.0 / 3.0));
        *nuF = __builtin_fma(nu[0], FA, __builtin_fma(a, al, cn * be));
    }
}

}  // namespace
}  // namespace gearrt
