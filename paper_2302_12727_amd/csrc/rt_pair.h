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
// (eq:eddington-group) rewritten without the 0/0 of n = F/|F|:
//   with f^2 = |F|^2/(cE)^2, s = sqrt(4 - 3 f^2):
//   (3 chi - 1)/(2 f^2) = 3/(2 + s),  (1 - chi)/2 = 1/3 - f^2/(2 + s),
//   c^2 P A = c^2 E (1-chi)/2 A + 3/(2+s) (F.A) F / E.
// out[0] = F.A, out[1..3] = c^2 P A.  A state with E = 0 has no flux.
__device__ __forceinline__ void m1_flux64(double E, double Fx, double Fy, double Fz, double Ax,
                                          double Ay, double Az, double c, double c2, double ic2,
                                          double out[4]) {
    // Guarded states have E >= 0 and F = 0 when E = 0; with 1/E replaced by 0
    // there every term below vanishes, so no branch is needed.
    // g = F/E keeps every product in range: f^2 = |g|^2/c^2, (F.A) F/E = (g.A) F.
    const double FA = Fx * Ax + Fy * Ay + Fz * Az;
    const double iE = E > 0.0 ? rcp64(E) : 0.0;
    const double gx = Fx * iE, gy = Fy * iE, gz = Fz * iE;
    const double f2 = (gx * gx + gy * gy + gz * gz) * ic2;
    const double s = sqrt64(fmax(4.0 - 3.0 * f2, 0.0));
    const double id = rcp64(2.0 + s);
    const double a = c2 * E * (1.0 / 3.0 - f2 * id);
    const double b = 3.0 * id * (gx * Ax + gy * Ay + gz * Az);
    out[0] = FA;
    out[1] = a * Ax + b * Fx;
    out[2] = a * Ay + b * Fy;
    out[3] = a * Az + b * Fz;
}

__device__ __forceinline__ double minmod(double a, double b) {
    const double m = (fabs(a) <= fabs(b)) ? a : b;
    return (a * b > 0.0) ? m : 0.0;
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

template <int NP>
__device__ __forceinline__ void block_reduce_store(double (&v)[NP], double *__restrict__ out,
                                                   double *smem) {
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
        out[threadIdx.x] = s;
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
__device__ __forceinline__ void stage_lines(const double *__restrict__ src, const int64_t (&row)[8],
                                            double *sb, int lane) {
    const int piece = lane & 7, slot = lane >> 3;
    double2 v[8];
#pragma unroll
    for (int m = 0; m < 8; ++m)
        v[m] = *reinterpret_cast<const double2 *>(src + 16 * row[m] + 2 * piece);
    wave_lds_sync();
#pragma unroll
    for (int m = 0; m < 8; ++m) {
        double *d = sb + (8 * m + slot) * kStage + 2 * piece;
        d[0] = v[m].x;
        d[1] = v[m].y;
    }
    wave_lds_sync();
}


// Copy the 4-double row (row_stride doubles apart) of every lane's row index j
// into the wave's stage buffer: 2 loads, 2 lanes per row, 32 rows per load.
__device__ __forceinline__ void stage_rows4(const double *__restrict__ src, int64_t row_stride,
                                            int64_t j, double *sb, int lane) {
    const int piece = lane & 1, slot = lane >> 1;
    double2 v[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        const int64_t r = __shfl(j, 32 * m + slot, 64);
        v[m] = *reinterpret_cast<const double2 *>(src + row_stride * r + 2 * piece);
    }
    wave_lds_sync();
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        double *d = sb + (32 * m + slot) * kStage + 2 * piece;
        d[0] = v[m].x;
        d[1] = v[m].y;
    }
    wave_lds_sync();
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
// state (E, F) for cotangent nu = (nu0, nu_v) of (F.A, c^2 P A).  With
// g = F/E, f^2 = |g|^2/c^2, s = sqrt(4 - 3 f^2), id = 1/(2 + s):
//   a = c^2 E/3 - c^2 E f^2 id,  b = 3 id (g.A),  flux_v = a A + b F,
//   kappa1 = id + (3/2) id^2 f^2 / s,  kappa2 = id + 3 id^2 f^2 / s,
//   d/dF = nu0 A - 2 (nu_v.A) kappa1 g + 3 (nu_v.g)(id A + 3 id^2 (g.A) g/(s c^2)) + b nu_v
//   d/dE = (nu_v.A) c^2 (1/3 + f^2 kappa2) - 3 (nu_v.g)(g.A) kappa2
// (at E = 0, where F = 0, the one-sided limit g = 0 is used).
__device__ __forceinline__ void m1_flux64_vjp(double E, double Fx, double Fy, double Fz, double Ax,
                                              double Ay, double Az, double c2, double ic2,
                                              const double nu[4], double out[4]) {
    const double iE = E > 0.0 ? rcp64(E) : 0.0;
    const double gx = Fx * iE, gy = Fy * iE, gz = Fz * iE;
    const double f2 = (gx * gx + gy * gy + gz * gz) * ic2;
    const double s = sqrt64(fmax(4.0 - 3.0 * f2, 0.0));
    const double is = rcp64(s);
    const double id = rcp64(2.0 + s);
    const double gA = gx * Ax + gy * Ay + gz * Az;
    const double b = 3.0 * id * gA;
    const double al = nu[1] * Ax + nu[2] * Ay + nu[3] * Az;
    const double ng = nu[1] * gx + nu[2] * gy + nu[3] * gz;
    const double k1 = id + 1.5 * id * id * f2 * is;
    const double k2 = id + 3.0 * id * id * f2 * is;
    const double t = 3.0 * ng;
    const double tg = -2.0 * al * k1 + t * 3.0 * id * id * gA * is * ic2;
    out[0] = al * c2 * (1.0 / 3.0 + f2 * k2) - t * gA * k2;
    out[1] = nu[0] * Ax + tg * gx + t * id * Ax + b * nu[1];
    out[2] = nu[0] * Ay + tg * gy + t * id * Ay + b * nu[2];
    out[3] = nu[0] * Az + tg * gz + t * id * Az + b * nu[3];
}

}  // namespace
}  // namespace gearrt
