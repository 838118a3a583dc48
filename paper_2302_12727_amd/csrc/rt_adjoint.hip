// Adjoint (vector-Jacobian product) of one RT step.  The thesis has no
// adjoint; this is the exact derivative of the step the forward kernels
// compute, with the subgradient of the active branch at minmod switches and
// guards.
//
// Forward step (per particle k, group g):
//   U'   = U + dt sum_s coef_sg L_s e_E                  injection
//   D    = S^{-1} sum_j (U'_j - U'_k) w_kj s_kj           gradient
//   U''  = U'_k - dt/V_k sum_l P_kl(U'_k, D_k; U'_l, D_l) transport, P_kl = |A| Phi_kl
//   U''' = guard(U'')
// Reverse, given lam''' = dLoss/dU''':
//   A: lam''   = guard^T lam'''                             (needs U'')
//   B: mu_kl   = dt lam''_l / V_l - dt lam''_k / V_k
//      lam'_k  = lam''_k + sum_l (dP_kl/dU'_k)^T mu_kl,  lamD_k = sum_l (dP_kl/dD_k)^T mu_kl
//      (each lane differentiates its own-perspective pair flux with respect to
//      its own inputs only: the pair's other half is taken by the neighbour's
//      lane, with P_lk = -P_kl and mu_lk = -mu_kl)
//   C: rho_i   = S_i^{-1} lamD_i;
//      lam_p   = lam'_p - (sum_j w_pj s_pj) . rho_p + sum_i w(r_ip/H_i) s_ip . rho_i
//   D: dLoss/dL_s += dt sum_g coef_sg lam_E,g
#include <mutex>

#include "rt_pair.h"

using namespace gearrt;

namespace {

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// Waves per SIMD the HLL pair pass is held to.  With its own state in
// registers it spilled about 30 at 2 waves and none at 1 (in accumulation
// registers); on the 3-group 128^3 lattice the backward of 20 steps took 496
// ms at 2 and 577 ms at 1.  With the own state in LDS it fits 256 registers
// at 2 waves without spills: 410 ms.
#ifndef RT_ADJ_HLL_WAVES
#define RT_ADJ_HLL_WAVES 2
#endif
constexpr int kAdjHllWaves = RT_ADJ_HLL_WAVES;
// The HLL pair pass keeps the own state, gradients and cotangent in LDS
// rather than in registers (21 doubles per particle, 45.5 KB per block).
#ifndef RT_ADJ_HLL_OWN
#define RT_ADJ_HLL_OWN 1
#endif
// The HLL pair pass of up to 3 groups takes the tiles of the forward (the
// adjoint of the tile transport); 0 keeps it two-sided.
#ifndef RT_ADJ_TILE_HLL
#define RT_ADJ_TILE_HLL 1
#endif
// ... and with the Ivanova surfaces; 0 keeps those two-sided.
#ifndef RT_ADJ_TILE_IVA
#define RT_ADJ_TILE_IVA 1
#endif
// Waves per SIMD of the HLL tile pair pass: at 2 it spills 28 bytes outside
// its inner loop; at 1 (no spill) the 20-step backward of the 3-group 128^3
// lattice took 406 ms against 305.
#ifndef RT_ADJ_TILE_HLL_WAVES
#define RT_ADJ_TILE_HLL_WAVES 2
#endif
constexpr bool kAdjHllOwn = RT_ADJ_HLL_OWN != 0;

template <int G>
__global__ __launch_bounds__(kBlock) void k_adj_guard64(int64_t n, const double *__restrict__ Uung,
                                                        const double *__restrict__ lam_next,
                                                        double *__restrict__ lam2, double c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * G) return;
    double q[4], l[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        q[m] = Uung[4 * t + m];
        l[m] = lam_next[4 * t + m];
    }
    guard64_vjp(q, l, c);
#pragma unroll
    for (int m = 0; m < 4; ++m) lam2[4 * t + m] = l[m];
}

// Pass B.  R[k][g] = (lam'_k (4) | rho_k (4 x 3)), the layout of a gradient
// record.  As in the forward transport, a wave owns 64 particles and GW of the
// G groups.
//
// Q lanes share a particle, each taking every Q-th neighbour slot (as in the
// forward transport); the partial sums are combined by a fixed butterfly.
//
// HLL: the pair flux of the HLL solver, P = w1 F_L.A + w2 F_R.A + w3 (U_R -
// U_L) with weights from the face states' wave speeds (the table hll); its
// cotangent m = 2 nu pulls back through the two M1 fluxes, the jump term, the
// weights and, through the speeds, the table lookups (hll_weights_vjp,
// hll_speeds64_vjp).
//
// IVA: the Ivanova surfaces (eq:IvanovaAij) in the recomputed pair geometry;
// they are static, so the pull-back is otherwise the same.
template <int G, int GW, int Q = 1, bool HLL = false, bool IVA = false, bool OWNL = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(HLL ? kAdjHllWaves : 1)))
void k_adj_pair64(
    int64_t n, int64_t nb, const double *__restrict__ geo, const int32_t *__restrict__ nbr,
    const int64_t *__restrict__ wave_base, const int32_t *__restrict__ n_nbr,
    const double *__restrict__ UD, const double *__restrict__ lam2,
    const double *__restrict__ dtp, double c, double box, double *__restrict__ R,
    const double2 *__restrict__ hll = nullptr, const double *__restrict__ ivan = nullptr) {
    static_assert(G % GW == 0, "group slices must tile the groups");
    static_assert(Q == 1 || Q == 2 || Q == 4, "lanes per particle: 1, 2 or 4");
    constexpr int NS = G / GW, NQ = 4 * GW, PW = 64 / Q, PB = kBlock / Q;
    constexpr int OS = 20 * GW + 1;             // OWNL: (U, D, lam'') per group in LDS
    __shared__ double stage[kBlock / 64][64 * kStage];
    __shared__ double own[OWNL ? PB * OS : 1];
    const int64_t bg = xcd_block(nb * NS);
    if (bg >= nb * NS) return;
    const int64_t blk = bg / NS;
    const int g0 = (int)(bg - blk * NS) * GW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int sub = lane % Q;
    const int64_t i0 = blk * PB + wv * PW;      // first particle of the wave
    const int64_t i = i0 + lane / Q;
    const bool active = i < n;
    const bool owner = active && sub == 0;
    const int64_t ic = active ? i : n - 1;
    const int64_t w = i0 >> 6;                  // neighbour-table wave (PW divides 64)
    const bool wave_live = i0 < n;
    const double ibox = 1.0 / box;
    const double dt = dtp[0];
    double *sb = stage[wv];

    const double *rk = geo + (int64_t)kRec * ic;
    const double dtVk = dt / rk[R_V];
    double gk[3] = {0.0, 0.0, 0.0};   // IVA: own kernel-gradient sum
    if (IVA) {
        gk[0] = ivan[4 * ic];
        gk[1] = ivan[4 * ic + 1];
        gk[2] = ivan[4 * ic + 2];
    }
    double Ui[OWNL ? 1 : NQ], Di[OWNL ? 1 : NQ * 3], Li[OWNL ? 1 : NQ];
    double *ow = own + (OWNL ? (threadIdx.x / Q) * OS : 0);
    if constexpr (OWNL) {
        // per group: the 16 values of the gradient record, then lam''
#pragma unroll
        for (int e = sub; e < 20 * GW; e += Q) {
            const int g = e / 20, f = e - 20 * g;
            ow[e] = f < 16 ? UD[(ic * G + g0 + g) * 16 + f] : lam2[(ic * G + g0 + g) * 4 + f - 16];
        }
        wave_lds_sync();
    } else {
#pragma unroll
        for (int g = 0; g < GW; ++g) {
            const double *r = UD + (ic * G + g0 + g) * 16;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                Ui[4 * g + m] = r[m];
                Di[3 * (4 * g + m) + 0] = r[4 + 3 * m];
                Di[3 * (4 * g + m) + 1] = r[5 + 3 * m];
                Di[3 * (4 * g + m) + 2] = r[6 + 3 * m];
                Li[4 * g + m] = lam2[(ic * G + g0 + g) * 4 + m];
            }
        }
    }
    // q = 4 g + m: own state, gradient component a, cotangent
    auto ui = [&](int q) -> double {
        if constexpr (OWNL) return ow[20 * (q >> 2) + (q & 3)];
        else return Ui[q];
    };
    auto di = [&](int q, int a) -> double {
        if constexpr (OWNL) return ow[20 * (q >> 2) + 4 + 3 * (q & 3) + a];
        else return Di[3 * q + a];
    };
    auto li = [&](int q) -> double {
        if constexpr (OWNL) return ow[20 * (q >> 2) + 16 + (q & 3)];
        else return Li[q];
    };
    double aU[NQ], aD[NQ * 3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) aU[q] = aD[3 * q] = aD[3 * q + 1] = aD[3 * q + 2] = 0.0;

    if (wave_live) {
        const int64_t base = wave_base[w] + (i & 63);
        int32_t kmax = (int32_t)((wave_base[w + 1] - wave_base[w]) >> 6);
        const int32_t nn = active ? n_nbr[i] : 0;
        if (Q > 1) {                            // the longest list of this wave's particles
            kmax = nn;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
        }
        // the next iteration's neighbour index is loaded one iteration ahead
        int32_t jn = sub < nn ? nbr[base + 64 * (int64_t)sub] : (int32_t)ic;
        for (int32_t kk = 0; kk < kmax; kk += Q) {
            const int32_t k = kk + sub;
            const bool valid = k < nn;
            const int32_t j = jn;
            // (slot 0 of the wave's table exists once kmax > 0: no branch
            // around the load, whose wait would then be a full one)
            const int32_t jl = nbr[base + 64 * (int64_t)(k + Q < nn ? k + Q : 0)];
            jn = k + Q < nn ? jl : (int32_t)ic;
            int64_t row[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) row[m] = __shfl(j, 8 * m + (lane >> 3), 64);
            stage_lines(geo, row, sb, lane);
            double rl[12];
#pragma unroll
            for (int q = 0; q < 12; ++q) rl[q] = sb[lane * kStage + q];
            PairGeo pg;
            if (IVA) {
                stage_rows4(ivan, 4, j, sb, lane);
                const double gl[3] = {sb[lane * kStage], sb[lane * kStage + 1],
                                      sb[lane * kStage + 2]};
                pair_geometry_ivanova64(rk, rl, gk, gl, box, ibox, pg);
            } else {
                pair_geometry64(rk, rl, box, ibox, pg);
            }
            const bool use = valid && pg.An > 0.0;
            const double dtVl = dt / rl[R_V];
#pragma unroll
            for (int g = 0; g < GW; ++g) {
                // the record lines and the cotangent rows in one round trip
                int64_t rowg[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) rowg[m] = row[m] * G + g0 + g;
                double2 v[8], vl[2];
                load_lines(UD, rowg, lane, v);
                load_rows4(lam2 + 4 * (g0 + g), 4 * G, j, lane, vl);
                store_lines(v, sb, lane);
                double Rl[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) Rl[q] = sb[lane * kStage + q];
                store_rows4(vl, sb, lane);
                double Ll[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) Ll[m] = sb[lane * kStage + m];
                // forward recompute of this pair and group
                double qLp[4], qRp[4], qL[4], qR[4];
                bool own_slope[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int q = 4 * g + m;
                    const double dk = di(q, 0) * pg.sx + di(q, 1) * pg.sy + di(q, 2) * pg.sz;
                    const double dl = Rl[4 + 3 * m] * pg.sx + Rl[5 + 3 * m] * pg.sy + Rl[6 + 3 * m] * pg.sz;
                    const double mm = minmod(dk, dl);
                    own_slope[m] = (dk * dl > 0.0) && (fabs(dk) <= fabs(dl));
                    qLp[m] = qL[m] = ui(q) + pg.fk * mm;
                    qRp[m] = qR[m] = Rl[m] - pg.fl * mm;
                }
                guard64(qL[0], qL[1], qL[2], qL[3], c);
                guard64(qR[0], qR[1], qR[2], qR[3], c);
                // cotangent of P_kl and its pull-back to the face states
                double nu[4], tL[4], tR[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) nu[m] = 0.5 * (dtVl * Ll[m] - dtVk * li(4 * g + m));
                double S1 = 0.0, S2 = 0.0;   // HLL: m . F_L, m . F_R
                m1_flux64_vjp(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, c, nu, tL,
                              HLL ? &S1 : nullptr);
                m1_flux64_vjp(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, c, nu, tR,
                              HLL ? &S2 : nullptr);
                if constexpr (HLL) {
                    const double iAn = pg.An > 0.0 ? rcp64(pg.An) : 0.0;
                    double loL, hiL, loR, hiR, w1, w2, w3;
                    hll_speeds64(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll, loL,
                                 hiL);
                    hll_speeds64(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll, loR,
                                 hiR);
                    hll_weights(loL, hiL, loR, hiR, pg.An, w1, w2, w3);
                    double S3 = 0.0;                       // m . (U_R - U_L)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        S3 += nu[m] * (qR[m] - qL[m]);
                        tL[m] = 2.0 * (w1 * tL[m] - w3 * nu[m]);
                        tR[m] = 2.0 * (w2 * tR[m] + w3 * nu[m]);
                    }
                    double gloL, ghiL, gloR, ghiR;
                    hll_weights_vjp(loL, hiL, loR, hiR, pg.An, 2.0 * S1, 2.0 * S2, 2.0 * S3,
                                    gloL, ghiL, gloR, ghiR);
                    hll_speeds64_vjp(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll,
                                     gloL, ghiL, tL);
                    hll_speeds64_vjp(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll,
                                     gloR, ghiR, tR);
                } else {
                    const double dis = c * pg.An;   // 2 * (c/2) |A| times nu = mu/2
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        tL[m] += dis * nu[m];
                        tR[m] -= dis * nu[m];
                    }
                }
                guard64_vjp(qLp, tL, c);
                guard64_vjp(qRp, tR, c);
                if (use) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int q = 4 * g + m;
                        aU[q] += tL[m];
                        const double lm = own_slope[m] ? pg.fk * tL[m] - pg.fl * tR[m] : 0.0;
                        aD[3 * q] += lm * pg.sx;
                        aD[3 * q + 1] += lm * pg.sy;
                        aD[3 * q + 2] += lm * pg.sz;
                    }
                }
            }
        }
    }
    if (Q > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            quad_sum<Q>(aU[q]);
            quad_sum<Q>(aD[3 * q]);
            quad_sum<Q>(aD[3 * q + 1]);
            quad_sum<Q>(aD[3 * q + 2]);
        }
    }
    if (!owner) return;
    const double iV = 1.0 / rk[R_V];
    const double b00 = rk[R_B] * iV, b01 = rk[R_B + 1] * iV, b02 = rk[R_B + 2] * iV;
    const double b11 = rk[R_B + 3] * iV, b12 = rk[R_B + 4] * iV, b22 = rk[R_B + 5] * iV;
#pragma unroll
    for (int g = 0; g < GW; ++g) {
        double *o = R + (i * G + g0 + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int q = 4 * g + m;
            o[m] = li(q) + aU[q];
            o[4 + 3 * m + 0] = b00 * aD[3 * q] + b01 * aD[3 * q + 1] + b02 * aD[3 * q + 2];
            o[4 + 3 * m + 1] = b01 * aD[3 * q] + b11 * aD[3 * q + 1] + b12 * aD[3 * q + 2];
            o[4 + 3 * m + 2] = b02 * aD[3 * q] + b12 * aD[3 * q + 1] + b22 * aD[3 * q + 2];
        }
    }
}

// Pass B with the pairs inside a tile evaluated once: the adjoint of the tile
// transport (GLF or HLL, Hopkins or Ivanova surfaces).  A block owns one 64-particle tile and
// GW of the groups; its particles walk the forward's task lists (k_tasks), in
// which an in-tile pair (k, l) appears once, flagged, in one particle's list.
// That lane pulls the pair back for both particles: its own cotangents as in
// k_adj_pair64, and the partner's, added by LDS atomics to the partner's row
// of its wave's copy of the tile's accumulator.  The forward evaluates the
// pair's face states once and uses the flux with opposite signs at its two
// particles, so from l's side the face states swap, s and A change sign, and
// the pull-back gives l
//   the cotangent of its state: t_R (k's right-face cotangent),
//   that of its gradient: (f_k t_L - f_l t_R) s where l's slope was the
//     limiter's choice (|d_l| <= |d_k|, same signs),
// which is the exact adjoint of the forward's single evaluation.  After a
// block barrier each particle's sums are its own plus the 4 waves' rows in a
// fixed order, as in the forward.  HLL: the HLL solver's pull-back of
// k_adj_pair64 (its flux is antisymmetric like GLF's, so the partner's share
// is the same t_R and slope term); it keeps the particle's own state,
// gradients and cotangent in LDS (OWNL), which the HLL pull-back's registers
// need.  IVA: the Ivanova surfaces (static, so only the recomputed pair
// geometry changes), with the kernel-gradient sums from slots 13-15 of the
// geometry records, and the own values in LDS as for HLL.
template <int G, int GW, bool OFF32, bool HLL, bool IVA>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(HLL ? RT_ADJ_TILE_HLL_WAVES : 2))) void
k_adj_pair64_tile(int64_t n, int64_t nb, const double *__restrict__ geo,
                  const int32_t *__restrict__ task, const int64_t *__restrict__ wave_base,
                  const int32_t *__restrict__ n_task, const double *__restrict__ UD,
                  const double *__restrict__ lam2, const double *__restrict__ dtp, double c,
                  double box, double *__restrict__ R, const double2 *__restrict__ hll) {
    static_assert(G % GW == 0, "group slices must tile the groups");
    constexpr int NS = G / GW, NQ = 4 * GW, MS = 16 * GW + 1;   // accumulator row, padded
    static_assert(kTile == 64 && kBlock == 256, "a block of 4 waves x 16 particles per tile");
    __shared__ double stage[kBlock / 64][64 * kStage];
    __shared__ double mir[kBlock / 64][kTile * MS];
    constexpr bool OWNL = HLL || IVA;
    constexpr int OS = 5 * NQ + 1;              // own row: U (NQ), D (3 NQ), lambda (NQ), pad
    __shared__ double own[OWNL ? kTile * OS : 1];
    const int64_t bg = xcd_block(nb * NS);
    if (bg >= nb * NS) return;                  // whole block: no barrier is skipped
    const int64_t blk = bg / NS;
    const int g0 = (int)(bg - blk * NS) * GW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int sub = lane & 3;
    const int64_t t0 = blk * kTile;             // the tile's first particle
    const int pl = 16 * wv + (lane >> 2);       // the lane's particle in the tile
    const int64_t i = t0 + pl;
    const bool active = i < n;
    const bool owner = active && sub == 0;
    const int64_t ic = active ? i : n - 1;
    const bool wave_live = t0 + 16 * wv < n;    // wave-uniform
    const double ibox = 1.0 / box;
    const double dt = dtp[0];
    double *sb = stage[wv];
    double *mw = mir[wv];                       // this wave's copy of the accumulator
    for (int e = lane; e < kTile * MS; e += 64) mw[e] = 0.0;
    wave_lds_sync();

    const double *rk = geo + (int64_t)kRec * ic;
    const double dtVk = dt / rk[R_V];
    const double gk[3] = {IVA ? rk[13] : 0.0, IVA ? rk[14] : 0.0, IVA ? rk[15] : 0.0};
    double Ui[OWNL ? 1 : NQ], Di[OWNL ? 1 : NQ * 3], Li[OWNL ? 1 : NQ];
    double *orow = own + (OWNL ? pl * OS : 0);  // (OWNL) the particle's row
    if constexpr (OWNL) {
        // lane sub copies component sub of each group
#pragma unroll
        for (int g = 0; g < GW; ++g) {
            const double *r = UD + (ic * G + g0 + g) * 16;
            const int q = 4 * g + sub;
            orow[q] = r[sub];
            orow[NQ + 3 * q + 0] = r[4 + 3 * sub];
            orow[NQ + 3 * q + 1] = r[5 + 3 * sub];
            orow[NQ + 3 * q + 2] = r[6 + 3 * sub];
            orow[4 * NQ + q] = lam2[(ic * G + g0 + g) * 4 + sub];
        }
        wave_lds_sync();
    } else {
#pragma unroll
        for (int g = 0; g < GW; ++g) {
            const double *r = UD + (ic * G + g0 + g) * 16;
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                Ui[4 * g + m] = r[m];
                Di[3 * (4 * g + m) + 0] = r[4 + 3 * m];
                Di[3 * (4 * g + m) + 1] = r[5 + 3 * m];
                Di[3 * (4 * g + m) + 2] = r[6 + 3 * m];
                Li[4 * g + m] = lam2[(ic * G + g0 + g) * 4 + m];
            }
        }
    }
    auto ui = [&](int q) -> double { if constexpr (OWNL) return orow[q]; else return Ui[q]; };
    auto di = [&](int q, int a) -> double {
        if constexpr (OWNL) return orow[NQ + 3 * q + a]; else return Di[3 * q + a];
    };
    auto li = [&](int q) -> double { if constexpr (OWNL) return orow[4 * NQ + q]; else return Li[q]; };
    double aU[NQ], aD[NQ * 3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) aU[q] = aD[3 * q] = aD[3 * q + 1] = aD[3 * q + 2] = 0.0;

    if (wave_live) {
        const int64_t base = wave_base[blk] + pl;   // the particle's column in the table
        const int32_t nn = active ? n_task[i] : 0;
        int32_t kmax = nn;                          // the longest list of the wave
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
        // the next iteration's task is loaded one iteration ahead
        int32_t tn = sub < nn ? task[base + 64 * (int64_t)sub] : (int32_t)ic;
        for (int32_t kk = 0; kk < kmax; kk += 4) {
            const int32_t k = kk + sub;
            const bool valid = k < nn;
            const int32_t t = tn;
            // (slot 0 of the tile's table exists once kmax > 0: no branch
            // around the load, whose wait would then be a full one)
            const int32_t tl = task[base + 64 * (int64_t)(k + 4 < nn ? k + 4 : 0)];
            tn = k + 4 < nn ? tl : (int32_t)ic;
            const bool mirror = t < 0;
            const int32_t j = t & 0x7fffffff;
            const int mr = mirror ? (j - (int32_t)t0) * MS : 0;   // the partner's row
            // rows by 32-bit byte offsets from the tables' bases while the
            // records fit 4 GiB (OFF32), as in the tile transport
            int32_t rw[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) rw[m] = __shfl(j, 8 * m + (lane >> 3), 64);
            const RowLines<OFF32> gl(geo, rw, 1, lane), ul(UD, rw, G, lane);
            {
                double2 v[8];
                gl.load(0, v);
                store_lines(v, sb, lane);
            }
            double rl[12];
#pragma unroll
            for (int q = 0; q < 12; ++q) rl[q] = sb[lane * kStage + q];
            PairGeo pg;
            if constexpr (IVA) {
                const double gl[3] = {sb[lane * kStage + 13], sb[lane * kStage + 14],
                                      sb[lane * kStage + 15]};
                pair_geometry_ivanova64(rk, rl, gk, gl, box, ibox, pg);
            } else {
                pair_geometry64(rk, rl, box, ibox, pg);
            }
            const bool use = valid && pg.An > 0.0;
            const double dtVl = dt * rcp64(rl[R_V]);   // (about 1 ulp; no IEEE division per pair)
#pragma unroll
            for (int g = 0; g < GW; ++g) {
                // the record lines and the cotangent rows in one round trip
                double2 v[8], vl[2];
                ul.load(g0 + g, v);
                load_rows4(lam2 + 4 * (g0 + g), 4 * G, j, lane, vl);
                store_lines(v, sb, lane);
                double Rl[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) Rl[q] = sb[lane * kStage + q];
                store_rows4(vl, sb, lane);
                double Ll[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) Ll[m] = sb[lane * kStage + m];
                // forward recompute of this pair and group
                double qLp[4], qRp[4], qL[4], qR[4];
                bool slope_k[4], slope_l[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int q = 4 * g + m;
                    const double dk = di(q, 0) * pg.sx + di(q, 1) * pg.sy + di(q, 2) * pg.sz;
                    const double dl = Rl[4 + 3 * m] * pg.sx + Rl[5 + 3 * m] * pg.sy + Rl[6 + 3 * m] * pg.sz;
                    const double mm = minmod(dk, dl);
                    slope_k[m] = (dk * dl > 0.0) && (fabs(dk) <= fabs(dl));
                    slope_l[m] = (dk * dl > 0.0) && (fabs(dl) <= fabs(dk));
                    qLp[m] = qL[m] = ui(q) + pg.fk * mm;
                    qRp[m] = qR[m] = Rl[m] - pg.fl * mm;
                }
                guard64(qL[0], qL[1], qL[2], qL[3], c);
                guard64(qR[0], qR[1], qR[2], qR[3], c);
                // cotangent of P_kl and its pull-back to the face states
                double nu[4], tL[4], tR[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) nu[m] = 0.5 * (dtVl * Ll[m] - dtVk * li(4 * g + m));
                double S1 = 0.0, S2 = 0.0;   // HLL: m . F_L, m . F_R
                m1_flux64_vjp(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, c, nu, tL,
                              HLL ? &S1 : nullptr);
                m1_flux64_vjp(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, c, nu, tR,
                              HLL ? &S2 : nullptr);
                if constexpr (HLL) {
                    const double iAn = pg.An > 0.0 ? rcp64(pg.An) : 0.0;
                    double loL, hiL, loR, hiR, w1, w2, w3;
                    hll_speeds64(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll, loL,
                                 hiL);
                    hll_speeds64(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll, loR,
                                 hiR);
                    hll_weights(loL, hiL, loR, hiR, pg.An, w1, w2, w3);
                    double S3 = 0.0;                       // m . (U_R - U_L)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        S3 += nu[m] * (qR[m] - qL[m]);
                        tL[m] = 2.0 * (w1 * tL[m] - w3 * nu[m]);
                        tR[m] = 2.0 * (w2 * tR[m] + w3 * nu[m]);
                    }
                    double gloL, ghiL, gloR, ghiR;
                    hll_weights_vjp(loL, hiL, loR, hiR, pg.An, 2.0 * S1, 2.0 * S2, 2.0 * S3,
                                    gloL, ghiL, gloR, ghiR);
                    hll_speeds64_vjp(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll,
                                     gloL, ghiL, tL);
                    hll_speeds64_vjp(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll,
                                     gloR, ghiR, tR);
                } else {
                    const double dis = c * pg.An;   // 2 * (c/2) |A| times nu = mu/2
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        tL[m] += dis * nu[m];
                        tR[m] -= dis * nu[m];
                    }
                }
                guard64_vjp(qLp, tL, c);
                guard64_vjp(qRp, tR, c);
                if (use) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int q = 4 * g + m;
                        aU[q] += tL[m];
                        const double lm = slope_k[m] ? pg.fk * tL[m] - pg.fl * tR[m] : 0.0;
                        aD[3 * q] += lm * pg.sx;
                        aD[3 * q + 1] += lm * pg.sy;
                        aD[3 * q + 2] += lm * pg.sz;
                    }
                    if (mirror) {
                        double *o = mw + mr + 16 * g;
#pragma unroll
                        for (int m = 0; m < 4; ++m) {
                            const double ll = slope_l[m] ? pg.fk * tL[m] - pg.fl * tR[m] : 0.0;
                            atomicAdd(o + m, tR[m]);
                            atomicAdd(o + 4 + 3 * m, ll * pg.sx);
                            atomicAdd(o + 5 + 3 * m, ll * pg.sy);
                            atomicAdd(o + 6 + 3 * m, ll * pg.sz);
                        }
                    }
                }
            }
        }
        // the 4 lanes' partial sums, combined by a fixed butterfly
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            quad_sum<4>(aU[q]);
            quad_sum<4>(aD[3 * q]);
            quad_sum<4>(aD[3 * q + 1]);
            quad_sum<4>(aD[3 * q + 2]);
        }
    }
    // every wave's deposits are in its copy of the accumulator
    __syncthreads();
    if (!owner || !wave_live) return;
#pragma unroll
    for (int g = 0; g < GW; ++g)
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int q = 4 * g + m;
#pragma unroll
            for (int v = 0; v < kBlock / 64; ++v) {
                const double *o = mir[v] + pl * MS + 16 * g;
                aU[q] += o[m];
                aD[3 * q] += o[4 + 3 * m];
                aD[3 * q + 1] += o[5 + 3 * m];
                aD[3 * q + 2] += o[6 + 3 * m];
            }
        }
    const double iV = 1.0 / rk[R_V];
    const double b00 = rk[R_B] * iV, b01 = rk[R_B + 1] * iV, b02 = rk[R_B + 2] * iV;
    const double b11 = rk[R_B + 3] * iV, b12 = rk[R_B + 4] * iV, b22 = rk[R_B + 5] * iV;
#pragma unroll
    for (int g = 0; g < GW; ++g) {
        double *o = R + (i * G + g0 + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int q = 4 * g + m;
            o[m] = li(q) + aU[q];
            o[4 + 3 * m + 0] = b00 * aD[3 * q] + b01 * aD[3 * q + 1] + b02 * aD[3 * q + 2];
            o[4 + 3 * m + 1] = b01 * aD[3 * q] + b11 * aD[3 * q + 1] + b12 * aD[3 * q + 2];
            o[4 + 3 * m + 2] = b02 * aD[3 * q] + b12 * aD[3 * q + 1] + b22 * aD[3 * q + 2];
        }
    }
}

// Pass C: transpose of the least-squares gradient, gathered over the
// symmetric neighbour lists (i is a gather neighbour of p iff r < H_i).  All
// loads of one neighbour slot (position and 1/H, and the G records of rho)
// are issued before the first is staged, so their latencies overlap.
// Q lanes share a particle as in the pair pass.
// blist: only the listed blocks (of kBlock / Q particles).
template <int G, int Q = 1>
__global__ __launch_bounds__(kBlock) void k_adj_grad64(
    int64_t n, int64_t nb, const double *__restrict__ geo, const int32_t *__restrict__ nbr,
    const int64_t *__restrict__ wave_base, const int32_t *__restrict__ n_nbr,
    const double *__restrict__ R, double *__restrict__ lam, double box,
    const int32_t *__restrict__ blist = nullptr) {
    static_assert(Q == 1 || Q == 2 || Q == 4, "lanes per particle: 1, 2 or 4");
    constexpr int NQ = 4 * G, PW = 64 / Q, PB = kBlock / Q;
    __shared__ double stage[kBlock / 64][64 * kStage];
    const int64_t bx = xcd_block(nb);
    if (bx >= nb) return;
    const int64_t blk = blist ? (int64_t)blist[bx] : bx;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int sub = lane % Q;
    const int64_t i0 = blk * PB + wv * PW;      // first particle of the wave
    const int64_t i = i0 + lane / Q;
    const bool active = i < n;
    const bool owner = active && sub == 0;
    const int64_t ic = active ? i : n - 1;
    const int64_t w = i0 >> 6;
    const bool wave_live = i0 < n;
    const double ibox = 1.0 / box;
    double *sb = stage[wv];
    const double *rp = geo + (int64_t)kRec * ic;
    const double px = rp[0], py = rp[1], pz = rp[2], iHp = rp[R_IH];
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    double sgx = 0.0, sgy = 0.0, sgz = 0.0;
    if (wave_live) {
        const int64_t base = wave_base[w] + (i & 63);
        int32_t kmax = (int32_t)((wave_base[w + 1] - wave_base[w]) >> 6);
        const int32_t nn = active ? n_nbr[i] : 0;
        if (Q > 1) {                            // the longest list of this wave's particles
            kmax = nn;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
        }
        // the next iteration's neighbour index is loaded one iteration ahead
        int32_t jn = sub < nn ? nbr[base + 64 * (int64_t)sub] : (int32_t)ic;
        for (int32_t kk = 0; kk < kmax; kk += Q) {
            const int32_t k = kk + sub;
            const bool valid = k < nn;
            const int32_t j = jn;
            jn = k + Q < nn ? nbr[base + 64 * (int64_t)(k + Q)] : (int32_t)ic;
            int64_t row[8];
#pragma unroll
            for (int m = 0; m < 8; ++m) row[m] = __shfl(j, 8 * m + (lane >> 3), 64);
            // groups in chunks of at most GC records in flight
            constexpr int GC = G < 4 ? G : 4;
            double2 vp[2], vr[GC][8];
            load_rows4(geo, kRec, j, lane, vp);
#pragma unroll
            for (int g = 0; g < GC; ++g) {
                int64_t rowg[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) rowg[m] = row[m] * G + g;
                load_lines(R, rowg, lane, vr[g]);
            }
            store_rows4(vp, sb, lane);
            const double *rl = sb + lane * kStage;
            const double sx = min_image(rl[0] - px, box, ibox);
            const double sy = min_image(rl[1] - py, box, ibox);
            const double sz = min_image(rl[2] - pz, box, ibox);
            const double iHl = rl[R_IH];
            const double r = sqrt64(sx * sx + sy * sy + sz * sz);
            const double wpi = valid ? kern_w(r * iHp) : 0.0;
            const double wip = valid ? kern_w(r * iHl) : 0.0;
            sgx += wpi * sx;
            sgy += wpi * sy;
            sgz += wpi * sz;
#pragma unroll
            for (int c0 = 0; c0 < G; c0 += GC) {
                if (c0 > 0) {
#pragma unroll
                    for (int g = 0; g < GC; ++g) {
                        if (c0 + g >= G) break;
                        int64_t rowg[8];
#pragma unroll
                        for (int m = 0; m < 8; ++m) rowg[m] = row[m] * G + c0 + g;
                        load_lines(R, rowg, lane, vr[g]);
                    }
                }
#pragma unroll
                for (int g = 0; g < GC; ++g) {
                    if (c0 + g >= G) break;
                    store_lines(vr[g], sb, lane);
                    const double *Rl = sb + lane * kStage;
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[4 * (c0 + g) + m] -=
                            wip * (Rl[4 + 3 * m] * sx + Rl[5 + 3 * m] * sy + Rl[6 + 3 * m] * sz);
                }
            }
        }
    }
    if (Q > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) quad_sum<Q>(acc[q]);
        quad_sum<Q>(sgx);
        quad_sum<Q>(sgy);
        quad_sum<Q>(sgz);
    }
    if (!owner) return;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const double *Rp = R + (i * G + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            lam[(i * G + g) * 4 + m] =
                Rp[m] - (sgx * Rp[4 + 3 * m] + sgy * Rp[5 + 3 * m] + sgz * Rp[6 + 3 * m]) +
                acc[4 * g + m];
    }
}

// Pass C from the block's neighbour union (FP64, the symmetric lists): the
// union's positions and 1/H are staged in LDS once per block of 64 particles,
// then for each group in turn its rows of rho (the gradient cotangents of the
// records R), and every pair reads its neighbour's row from LDS by its 16-bit
// position in the union.  A lane sums the same slots in the same order with
// the same operations as k_adj_grad64 with four lanes (rows past a list are
// the own row with zero weights), so the two give identical bits; blocks whose
// union did not fit are left to it, by list.
typedef double dvec2a __attribute__((ext_vector_type(2)));
template <int G, int W>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(W, W))) void
k_adj_grad64u(int64_t n, int64_t nb, const double *__restrict__ geo,
              const int32_t *__restrict__ urow, const int64_t *__restrict__ uoff,
              const uint16_t *__restrict__ gloc, const int64_t *__restrict__ goff,
              const uint16_t *__restrict__ uown, const int32_t *__restrict__ n_nbr,
              const double *__restrict__ R, double *__restrict__ lam, double box) {
    constexpr int Q = 4, UC = adj_union_cap(W);
    static_assert(kBlock == 256 && UC <= 1024, "64 particles per block");
    __shared__ dvec2a upos[UC * 2];             // x, y | z, 1/H: the record's first line piece
    __shared__ dvec2a urho[UC * 6];             // one group's 12 gradient cotangents
    __shared__ int32_t uidx[UC];
    const int64_t blk = xcd_block(nb);
    if (blk >= nb) return;                      // whole block
    const int64_t u0 = uoff[blk];
    const int32_t rows = (int32_t)(uoff[blk + 1] - u0);
    if (rows == 0) return;                      // left to k_adj_grad64 (whole block)
    for (int e = threadIdx.x; e < rows; e += kBlock) uidx[e] = urow[u0 + e];
    __syncthreads();
    {   // positions and 1/H, all loads in flight
        constexpr int MP = (UC * 2 + kBlock - 1) / kBlock;
        const dvec2a *G2 = reinterpret_cast<const dvec2a *>(geo);
        dvec2a v[MP];
#pragma unroll
        for (int r = 0; r < MP; ++r) {
            const int e = threadIdx.x + r * kBlock;
            if (e < 2 * rows) v[r] = G2[(uint32_t)uidx[e >> 1] * (uint32_t)(kRec / 2) + (uint32_t)(e & 1)];
        }
#pragma unroll
        for (int r = 0; r < MP; ++r)
            if (threadIdx.x + r * kBlock < 2 * rows) upos[threadIdx.x + r * kBlock] = v[r];
    }
    const int lane = threadIdx.x & 63, sub = lane % Q;
    const int p = threadIdx.x / Q;              // the particle in the block
    const int64_t i = blk * (kBlock / Q) + p;
    const bool active = i < n;
    const bool owner = active && sub == 0;
    const int64_t ic = active ? i : n - 1;
    const int32_t nn = active ? n_nbr[ic] : 0;
    const int il = active ? (int)uown[ic] : 0;  // a row of the union (not used past n)
    int32_t kmax = nn;                          // the wave's longest list
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
    const double *rp = geo + (int64_t)kRec * ic;
    const double px = rp[0], py = rp[1], pz = rp[2], iHp = rp[R_IH];
    const double ibox = 1.0 / box;
    const int64_t g0 = goff[blk];
    const int ngb = (int)((goff[blk + 1] - g0) >> 10);          // the block's entry groups
    const uint64_t *gw = reinterpret_cast<const uint64_t *>(gloc + g0) + threadIdx.x;
    const int T = (kmax + Q - 1) / Q, ngq = (T + 3) / 4;        // this wave's iterations, groups
    double sgx = 0.0, sgy = 0.0, sgz = 0.0;
    const dvec2a *R2 = reinterpret_cast<const dvec2a *>(R);
#pragma unroll 1
    for (int g = 0; g < G; ++g) {
        __syncthreads();                        // the previous group's rows are read
        {   // group g's rows of rho, all loads in flight
            constexpr int MS = (UC * 6 + kBlock - 1) / kBlock;
            dvec2a v[MS];
#pragma unroll
            for (int r = 0; r < MS; ++r) {
                const int e = threadIdx.x + r * kBlock;
                if (e < 6 * rows)
                    v[r] = R2[((uint32_t)uidx[e / 6] * (uint32_t)G + (uint32_t)g) * 8u + 2u +
                              (uint32_t)(e % 6)];
            }
#pragma unroll
            for (int r = 0; r < MS; ++r)
                if (threadIdx.x + r * kBlock < 6 * rows) urho[threadIdx.x + r * kBlock] = v[r];
        }
        __syncthreads();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        if (kmax > 0) {
            auto pair = [&](int jl, bool valid) __attribute__((always_inline)) {
                const dvec2a a = upos[2 * jl], b = upos[2 * jl + 1];
                const double sx = min_image(a.x - px, box, ibox);
                const double sy = min_image(a.y - py, box, ibox);
                const double sz = min_image(b.x - pz, box, ibox);
                const double iHl = b.y;
                const double r = sqrt64(sx * sx + sy * sy + sz * sz);
                if (g == 0) {
                    const double wpi = valid ? kern_w(r * iHp) : 0.0;
                    sgx += wpi * sx;
                    sgy += wpi * sy;
                    sgz += wpi * sz;
                }
                const double wip = valid ? kern_w(r * iHl) : 0.0;
                const dvec2a *Rl = urho + 6 * jl;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    // doubles 3m .. 3m+2 of the row: pieces (3m)/2 ..
                    const double d0 = Rl[(3 * m) >> 1][(3 * m) & 1];
                    const double d1 = Rl[(3 * m + 1) >> 1][(3 * m + 1) & 1];
                    const double d2 = Rl[(3 * m + 2) >> 1][(3 * m + 2) & 1];
                    acc[m] -= wip * (d0 * sx + d1 * sy + d2 * sz);
                }
            };
            auto word = [&](int gq) __attribute__((always_inline)) {
                return gw[(int64_t)(gq < ngb ? gq : ngb - 1) * 256];
            };
            auto four = [&](uint64_t wd, int gq) __attribute__((always_inline)) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    if (4 * gq + u < T) {                        // wave-uniform
                        const int k = Q * (4 * gq + u) + sub;
                        const bool valid = k < nn;
                        pair(valid ? (int)((wd >> (16 * u)) & 0xffff) : il, valid);
                    }
                }
            };
            uint64_t ea = word(0), eb = word(1);
            for (int gq = 0; gq < ngq; gq += 2) {
                const uint64_t wa = ea;
                ea = word(gq + 2);
                four(wa, gq);
                if (gq + 1 >= ngq) break;
                const uint64_t wb = eb;
                eb = word(gq + 3);
                four(wb, gq + 1);
            }
        }
#pragma unroll
        for (int m = 0; m < 4; ++m) quad_sum<Q>(acc[m]);
        if (g == 0) {
            quad_sum<Q>(sgx);
            quad_sum<Q>(sgy);
            quad_sum<Q>(sgz);
        }
        if (owner) {
            const double *Rp = R + (i * G + g) * 16;
#pragma unroll
            for (int m = 0; m < 4; ++m)
                lam[(i * G + g) * 4 + m] =
                    Rp[m] - (sgx * Rp[4 + 3 * m] + sgy * Rp[5 + 3 * m] + sgz * Rp[6 + 3 * m]) +
                    acc[m];
        }
    }
}

// Pass D: dLoss/dL_s += dt sum_{g in s} coef_sg lam_E,g, one block per source.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_adj_inject(int32_t S, int G,
                                                       const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ gas,
                                                       const double *__restrict__ coef,
                                                       const T *__restrict__ lam,
                                                       const double *__restrict__ dtp,
                                                       double *__restrict__ dLdL) {
    __shared__ double sm[kBlock];
    const int32_t s = blockIdx.x;
    for (int grp = 0; grp < G; ++grp) {
        double v = 0.0;
        for (int32_t e = ptr[s] + threadIdx.x; e < ptr[s + 1]; e += kBlock)
            v += coef[e] * (double)lam[((int64_t)gas[e] * G + grp) * 4];
        sm[threadIdx.x] = v;
        __syncthreads();
        for (int h = kBlock / 2; h > 0; h >>= 1) {
            if (threadIdx.x < h) sm[threadIdx.x] += sm[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) dLdL[s * G + grp] += dtp[0] * sm[0];
        __syncthreads();
    }
}

// Groups per wave of the adjoint pair pass.  Its per-group state is three
// times the forward's, so one group per wave wins here (G = 3: 239 VGPRs and
// 2 waves per SIMD, against occupancy 1 with all groups; the pass is 1.5x
// faster).
#ifndef RT_ADJ_GW
#define RT_ADJ_GW 1
#endif
// Lanes per particle of the adjoint pair pass and of the transposed gradient
// (1, 2 or 4).  On the 128^3 adjoint workload 4 lanes took the transposed
// gradient from 4.2 to about 2 ms per step (backward 337 -> 292 ms); the pair
// pass gains little (one group per wave already keeps its records in cache).
#ifndef RT_ADJ_Q
#define RT_ADJ_Q 4
#endif
#ifndef RT_ADJ_GRAD_Q
#define RT_ADJ_GRAD_Q 4
#endif
constexpr int kAQ = RT_ADJ_Q, kAGQ = RT_ADJ_GRAD_Q;

template <int G>
void launch_adjoint64(rt_ctx *ctx, const double *UD, const double *Uung, const double *lam_next,
                      double *lam2, double *R, double *lam, const double *dt) {
    const int64_t n = ctx->p.n, nb = (n + kBlock - 1) / kBlock;
    hipStream_t st = ctx->stream;
    k_adj_guard64<G><<<nblk(n * G), kBlock, 0, st>>>(n, Uung, lam_next, lam2, ctx->p.c_red);
    constexpr int GW = (RT_ADJ_GW == 0 || G % RT_ADJ_GW != 0) ? G : RT_ADJ_GW;
    const int64_t np = (n + kBlock / kAQ - 1) / (kBlock / kAQ);
    const double2 *tab = (const double2 *)ctx->hll_table;
    const bool iva = ctx->surfaces == RT_IVANOVA;
    const bool hll_tile = RT_ADJ_TILE_HLL != 0 && ctx->solver == RT_HLL && G <= 3;
    const bool iva_tile = RT_ADJ_TILE_IVA != 0 && iva && G <= 3;
    if ((ctx->solver == RT_GLF || hll_tile) && (!iva || iva_tile) && ctx->task) {
        // the adjoint of the tile transport (in-tile pairs once)
        const int64_t nt = (n + kTile - 1) / kTile;
        const bool off32 = (uint64_t)n * 128u * G < (uint64_t(1) << 32);
#define RT_ADJ_TILE_LAUNCH(OFF32_, HLL_, IVA_)                                                  \
    k_adj_pair64_tile<G, GW, OFF32_, HLL_, IVA_>                                                \
        <<<(unsigned)xcd_grid(nt * (G / GW)), kBlock, 0, st>>>(                                 \
            n, nt, ctx->geo, ctx->task, ctx->wave_base, ctx->n_task, UD, lam2, dt,              \
            ctx->p.c_red, ctx->p.box, R, tab)
#define RT_ADJ_TILE_LAUNCH_S(HLL_, IVA_)                                                        \
    do {                                                                                        \
        if (off32) RT_ADJ_TILE_LAUNCH(true, HLL_, IVA_);                                        \
        else RT_ADJ_TILE_LAUNCH(false, HLL_, IVA_);                                             \
    } while (0)
        if (hll_tile || iva_tile) {
            if constexpr (G <= 3) {
                if (hll_tile && iva_tile) RT_ADJ_TILE_LAUNCH_S(true, true);
                else if (hll_tile) RT_ADJ_TILE_LAUNCH_S(true, false);
                else RT_ADJ_TILE_LAUNCH_S(false, true);
            }
        } else {
            RT_ADJ_TILE_LAUNCH_S(false, false);
        }
#undef RT_ADJ_TILE_LAUNCH_S
#undef RT_ADJ_TILE_LAUNCH
    } else {
#define RT_ADJ_PAIR_LAUNCH(HLL_, IVA_)                                                          \
    k_adj_pair64<G, GW, kAQ, HLL_, IVA_, (HLL_ && kAdjHllOwn)><<<(unsigned)xcd_grid(np * (G / GW)), kBlock, 0, st>>>( \
        n, np, ctx->geo, ctx->nbr, ctx->wave_base, ctx->n_nbr, UD, lam2, dt, ctx->p.c_red,      \
        ctx->p.box, R, tab, ctx->ivan)
    if (ctx->solver == RT_HLL) {
        if (iva) RT_ADJ_PAIR_LAUNCH(true, true);
        else RT_ADJ_PAIR_LAUNCH(true, false);
    } else {
        if (iva) RT_ADJ_PAIR_LAUNCH(false, true);
        else RT_ADJ_PAIR_LAUNCH(false, false);
    }
#undef RT_ADJ_PAIR_LAUNCH
    }
    if constexpr (G <= 4 && kAGQ == 4) {
        if (ctx->aoff) {
            // blocks whose union fits: from LDS; the others: by list
            const int64_t nw = ctx->nwaves;
            if (ctx->adj_union_waves == 3)
                k_adj_grad64u<G, 3><<<(unsigned)xcd_grid(nw), kBlock, 0, st>>>(
                    n, nw, ctx->geo, ctx->arow, ctx->aoff, ctx->agloc, ctx->goff, ctx->aown,
                    ctx->n_nbr, R, lam, ctx->p.box);
            else
                k_adj_grad64u<G, 2><<<(unsigned)xcd_grid(nw), kBlock, 0, st>>>(
                    n, nw, ctx->geo, ctx->arow, ctx->aoff, ctx->agloc, ctx->goff, ctx->aown,
                    ctx->n_nbr, R, lam, ctx->p.box);
            if (ctx->n_ablk > 0)
                k_adj_grad64<G, 4><<<(unsigned)xcd_grid(ctx->n_ablk), kBlock, 0, st>>>(
                    n, ctx->n_ablk, ctx->geo, ctx->nbr, ctx->wave_base, ctx->n_nbr, R, lam,
                    ctx->p.box, ctx->ablk);
            return;
        }
    }
    const int64_t ng = (n + kBlock / kAGQ - 1) / (kBlock / kAGQ);
    k_adj_grad64<G, kAGQ><<<(unsigned)xcd_grid(ng), kBlock, 0, st>>>(
        n, ng, ctx->geo, ctx->nbr, ctx->wave_base, ctx->n_nbr, R, lam, ctx->p.box);
}

}  // namespace

// Scratch of the adjoint: [lam''  | R | recomputed U' | UD | U'' | U_out]
static rt_status adj_scratch(rt_ctx *ctx, size_t es, char **base) {
    const size_t nu = (size_t)ctx->p.n * 4 * ctx->p.groups * es;
    const size_t need = nu * (1 + 4 + 1 + 4 + 1 + 1) + 6 * 256;
    if (!ctx->adj_buf || ctx->adj_bytes < need) {
        rt_free(ctx, ctx->adj_buf);
        ctx->adj_buf = nullptr;
        rt_status rs = rt_alloc(ctx, &ctx->adj_buf, need);
        if (rs != RT_OK) return rs;
        ctx->adj_bytes = need;
    }
    *base = (char *)ctx->adj_buf;
    return RT_OK;
}

// Passes A-D of one adjoint step on the gradient record UD and unguarded
// state U_ung of the forward, with lam'' and R in caller-provided scratch.
static void adjoint_passes(rt_ctx *ctx, const double *L, const double *dt, const void *UD,
                           const void *U_ung, const void *lam_next, void *lam2, void *Rb,
                           void *lam, double *dL_dL) {
    (void)L;
    if (ctx->p.precision == RT_FP32C) {
        rt_adjoint32(ctx, (const float *)UD, (const float *)U_ung, (const float *)lam_next,
                     (float *)lam2, (float *)Rb, (float *)lam, dt);
    } else {
#define RT_ADJ64(G_)                                                                          \
    case G_:                                                                                  \
        launch_adjoint64<G_>(ctx, (const double *)UD, (const double *)U_ung,                  \
                             (const double *)lam_next, (double *)lam2, (double *)Rb,          \
                             (double *)lam, dt);                                              \
        break;
        switch (ctx->p.groups) {
            RT_ADJ64(1) RT_ADJ64(2) RT_ADJ64(3) RT_ADJ64(4)
            RT_ADJ64(5) RT_ADJ64(6) RT_ADJ64(7) RT_ADJ64(8)
            default: break;
        }
#undef RT_ADJ64
    }
    if (ctx->S > 0 && dL_dL) {
        if (ctx->p.precision == RT_FP64)
            k_adj_inject<double><<<ctx->S, kBlock, 0, ctx->stream>>>(
                ctx->S, ctx->p.groups, ctx->src_ptr, ctx->src_gas, ctx->src_coef,
                (const double *)lam, dt, dL_dL);
        else
            k_adj_inject<float><<<ctx->S, kBlock, 0, ctx->stream>>>(
                ctx->S, ctx->p.groups, ctx->src_ptr, ctx->src_gas, ctx->src_coef,
                (const float *)lam, dt, dL_dL);
    }
}

rt_status rt_adjoint_impl(rt_ctx *ctx, const void *U_pre, const double *L, const double *dt,
                          const void *UD, const void *U_ung, const void *lam_next, void *lam,
                          double *dL_dL) {
    const size_t es = ctx->p.precision == RT_FP64 ? 8 : 4;
    const size_t nu = (size_t)ctx->p.n * 4 * ctx->p.groups * es;
    char *b;
    rt_status rs = adj_scratch(ctx, es, &b);
    if (rs != RT_OK) return rs;
    auto carve = [&](size_t bytes) {
        char *p = b;
        b += (bytes + 255) & ~size_t(255);
        return (void *)p;
    };
    void *lam2 = carve(nu);
    void *Rb = carve(4 * nu);
    void *Ut = carve(nu);
    void *UDs = carve(4 * nu);
    void *Uu = carve(nu);
    void *Uo = carve(nu);
    rt_timer_begin(ctx, "adjoint");
    if (!UD) {
        if (!U_pre) return rt_fail(ctx, RT_EINVAL, "U_pre is required when UD is NULL");
        RT_HIP(hipMemcpyAsync(Ut, U_pre, nu, hipMemcpyDeviceToDevice, ctx->stream));
        if ((rs = rt_inject_impl(ctx, Ut, L, dt)) != RT_OK) return rs;
        if ((rs = rt_gradient_impl(ctx, Ut, UDs)) != RT_OK) return rs;
        UD = UDs;
    }
    if (!U_ung) {
        if ((rs = rt_transport_impl(ctx, UD, dt, Uo, nullptr, nullptr, nullptr, Uu)) != RT_OK)
            return rs;
        U_ung = Uu;
    }
    adjoint_passes(ctx, L, dt, UD, U_ung, lam_next, lam2, Rb, lam, dL_dL);
    rt_timer_end(ctx, "adjoint");
    RT_HIP(hipGetLastError());
    return RT_OK;
}

// ---------------------------------------------------------------------------
// The adjoint for callers that cannot allocate device memory.  Its scratch,
// lam'' (one state-sized array) and the pair-pass records R (four), lives in
// the fixed array `scratch` instead of the context's lazily allocated buffer.
// Each device holds its own copy of the array at its own address: host code
// never names `scratch` where it needs the memory, it uses the address
// rt_adjoint_static_init looked up for the device (g_scratch).  Every pass
// writes the scratch it later reads, so nothing needs clearing between calls;
// calls that overlap on one device share the array and race.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch[kMaxDevices];
static hipError_t g_scratch_err[kMaxDevices];
static bool g_scratch_done[kMaxDevices];

// Look up the device address of `scratch` once per device, with the context's
// device current (called by rt_create).
void rt_adjoint_static_init(rt_ctx *ctx) {
    const int d = ctx->device;
    if (d < 0 || d >= kMaxDevices) return;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_done[d]) return;
    g_scratch_done[d] = true;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        g_scratch_err[d] = e;
        return;
    }
    g_scratch[d] = p;
}

size_t rt_adjoint_static_bytes(const rt_ctx *ctx) {
    const size_t es = ctx->p.precision == RT_FP64 ? 8 : 4;
    const size_t nu = (size_t)ctx->p.n * 4 * ctx->p.groups * es;
    return ((nu + 255) & ~size_t(255)) + ((4 * nu + 255) & ~size_t(255));
}

rt_status rt_adjoint_static_impl(rt_ctx *ctx, const double *L, const double *dt, const void *UD,
                                 const void *U_ung, const void *lam_next, void *lam,
                                 double *dL_dL) {
    const size_t need = rt_adjoint_static_bytes(ctx);
    if (need > kStaticScratchBytes)
        return rt_fail(ctx, RT_EINVAL,
                       "rt_adjoint_static: n x groups needs " + std::to_string(need) +
                           " bytes of scratch, more than its fixed " +
                           std::to_string(kStaticScratchBytes) + " (use rt_adjoint)");
    int cur = -1;
    RT_HIP(hipGetDevice(&cur));
    if (cur != ctx->device)
        return rt_fail(ctx, RT_EINVAL, "rt_adjoint_static: the context's device is not current");
    void *base = nullptr;
    hipError_t err = hipSuccess;
    if (cur >= 0 && cur < kMaxDevices) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        base = g_scratch[cur];
        err = g_scratch_err[cur];
    }
    if (!base)
        return rt_fail(ctx, RT_EHIP, std::string("rt_adjoint_static: no scratch on this device") +
                                         (err != hipSuccess ? std::string(": ") +
                                                                  hipGetErrorString(err)
                                                            : std::string()));
    const size_t es = ctx->p.precision == RT_FP64 ? 8 : 4;
    const size_t nu = (size_t)ctx->p.n * 4 * ctx->p.groups * es;
    char *b = (char *)base;
    void *lam2 = b;
    void *Rb = b + ((nu + 255) & ~size_t(255));
    adjoint_passes(ctx, L, dt, UD, U_ung, lam_next, lam2, Rb, lam, dL_dL);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
