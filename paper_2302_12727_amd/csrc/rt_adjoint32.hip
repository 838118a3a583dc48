// Compensated-FP32 adjoint of one RT step: the passes of the FP64 adjoint
// (guard VJP, own-side pair VJPs, transpose of the gradient) with FP32 pair
// arithmetic; the state cotangent of every particle is summed with Kahan
// compensation.
#include "rt_pair32.h"

using namespace gearrt;

namespace {

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

template <int G>
__global__ __launch_bounds__(kBlock) void k_adj_guard32(int64_t n, const float *__restrict__ Uung,
                                                        const float *__restrict__ lam_next,
                                                        float *__restrict__ lam2, float c) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * G) return;
    float q[4], l[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        q[m] = Uung[4 * t + m];
        l[m] = lam_next[4 * t + m];
    }
    guard32_vjp(q, l, c);
#pragma unroll
    for (int m = 0; m < 4; ++m) lam2[4 * t + m] = l[m];
}

// A wave owns 64 particles and GW of the G groups (G/GW waves per 64
// particles), as in the FP64 pair pass.  HLL and IVA as in the FP64 pair
// pass (the FP32 table, the FP32 Ivanova surfaces of the FP32C transport).
template <int G, int GW, bool HLL = false, bool IVA = false>
__global__ __launch_bounds__(kBlock) void k_adj_pair32(
    int64_t n, int64_t nb, const float *__restrict__ geo32, const double *__restrict__ geo,
    const int32_t *__restrict__ nbr, const int64_t *__restrict__ wave_base,
    const int32_t *__restrict__ n_nbr, const float *__restrict__ UD,
    const float *__restrict__ lam2, const double *__restrict__ dtp, double c, double box,
    float *__restrict__ R, const float2 *__restrict__ hll = nullptr,
    const double *__restrict__ ivan = nullptr) {
    static_assert(G % GW == 0, "group slices must tile the groups");
    constexpr int NS = G / GW, NQ = 4 * GW;
    __shared__ float stage[kBlock / 64][64 * kStage32];
    const int64_t bg = xcd_block(nb * NS);
    if (bg >= nb * NS) return;
    const int64_t blk = bg / NS;
    const int g0 = (int)(bg - blk * NS) * GW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t i = blk * kBlock + threadIdx.x;
    const bool active = i < n;
    const int64_t ic = active ? i : n - 1;
    const int64_t w = i >> 6;
    const bool wave_live = (w << 6) < n;
    const double ibox = 1.0 / box;
    const float cf = (float)c, c2 = (float)(c * c), ic2 = (float)(1.0 / (c * c));
    const float dtf = (float)dtp[0];
    float *sb = stage[wv];

    const float *rk = geo32 + (int64_t)F_REC * ic;
    const double *xk = reinterpret_cast<const double *>(rk);
    const double pkx = xk[0], pky = xk[1], pkz = xk[2];
    const float iHk = rk[F_IH], hk = rk[F_H];
    float gk[3] = {0.0f, 0.0f, 0.0f};   // IVA: own kernel-gradient sum
    if (IVA) {
        gk[0] = (float)ivan[4 * ic];
        gk[1] = (float)ivan[4 * ic + 1];
        gk[2] = (float)ivan[4 * ic + 2];
    }
    float Bk[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) Bk[a] = rk[F_B + a];
    const float dtVk = (float)(dtp[0] / geo[(int64_t)kRec * ic + R_V]);
    float Ui[NQ], Di[NQ * 3], Li[NQ];
#pragma unroll
    for (int g = 0; g < GW; ++g) {
        const float *r = UD + (ic * G + g0 + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            Ui[4 * g + m] = r[m];
            Di[3 * (4 * g + m) + 0] = r[4 + 3 * m];
            Di[3 * (4 * g + m) + 1] = r[5 + 3 * m];
            Di[3 * (4 * g + m) + 2] = r[6 + 3 * m];
            Li[4 * g + m] = lam2[(ic * G + g0 + g) * 4 + m];
        }
    }
    Kahan aU[NQ];
    float aD[NQ * 3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        aU[q].s = aU[q].c = 0.0f;
        aD[3 * q] = aD[3 * q + 1] = aD[3 * q + 2] = 0.0f;
    }
    if (wave_live) {
        const int64_t base = wave_base[w] + lane;
        const int32_t kmax = (int32_t)((wave_base[w + 1] - wave_base[w]) >> 6);
        const int32_t nn = active ? n_nbr[i] : 0;
        // the next iteration's neighbour index is loaded one iteration ahead
        int32_t jn = 0 < nn ? nbr[base] : (int32_t)ic;
        for (int32_t k = 0; k < kmax; ++k) {
            const bool valid = k < nn;
            const int32_t j = jn;
            jn = k + 1 < nn ? nbr[base + 64 * (int64_t)(k + 1)] : (int32_t)ic;
            int64_t row[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) row[m] = __shfl(j, 16 * m + (lane >> 2), 64);
            stage_rows32(geo32, row, sb, lane);
            PairGeo32 pg;
            pair_geometry32(pkx, pky, pkz, iHk, hk, Bk, sb + lane * kStage32, box, ibox, pg);
            if (IVA) {                          // the same pair with the Ivanova surface
                const float *rl = sb + lane * kStage32;
                const double *gd = ivan + 4 * (int64_t)j;
                const float gl[3] = {(float)gd[0], (float)gd[1], (float)gd[2]};
                const float r = sqrt32(pg.sx * pg.sx + pg.sy * pg.sy + pg.sz * pg.sz);
                ivanova_surface32(pg.sx, pg.sy, pg.sz, r, iHk, rk[F_V], gk, rl[F_IH], rl[F_V], gl,
                                  pg.Ax, pg.Ay, pg.Az);
                pg.An = sqrt32(pg.Ax * pg.Ax + pg.Ay * pg.Ay + pg.Az * pg.Az);
            }
            const float dtVl = dtf * rcp32(sb[lane * kStage32 + F_V]);
            const bool use = valid && pg.An > 0.0f;
#pragma unroll
            for (int g = 0; g < GW; ++g) {
                int64_t rowg[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) rowg[m] = row[m] * G + g0 + g;
                stage_rows32(UD, rowg, sb, lane);
                float Rl[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) Rl[q] = sb[lane * kStage32 + q];
                const float4 Ll =
                    *reinterpret_cast<const float4 *>(lam2 + ((int64_t)j * G + g0 + g) * 4);
                float qLp[4], qRp[4], qL[4], qR[4];
                bool own_slope[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int q = 4 * g + m;
                    const float dk = Di[3 * q] * pg.sx + Di[3 * q + 1] * pg.sy + Di[3 * q + 2] * pg.sz;
                    const float dl = Rl[4 + 3 * m] * pg.sx + Rl[5 + 3 * m] * pg.sy + Rl[6 + 3 * m] * pg.sz;
                    const float mm = minmod32(dk, dl);
                    own_slope[m] = (dk * dl > 0.0f) && (fabsf(dk) <= fabsf(dl));
                    qLp[m] = qL[m] = Ui[q] + pg.fk * mm;
                    qRp[m] = qR[m] = Rl[m] - pg.fl * mm;
                }
                guard32(qL[0], qL[1], qL[2], qL[3], cf);
                guard32(qR[0], qR[1], qR[2], qR[3], cf);
                const float Llm[4] = {Ll.x, Ll.y, Ll.z, Ll.w};
                float nu[4], tL[4], tR[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) nu[m] = 0.5f * (dtVl * Llm[m] - dtVk * Li[4 * g + m]);
                m1_flux32_vjp(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, c2, ic2, nu, tL);
                m1_flux32_vjp(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, c2, ic2, nu, tR);
                if constexpr (HLL) {
                    const float iAn = pg.An > 0.0f ? rcp32(pg.An) : 0.0f;
                    float loL, hiL, loR, hiR, w1, w2, w3;
                    hll_speeds32(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, iAn, cf, ic2, hll,
                                 loL, hiL);
                    hll_speeds32(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, iAn, cf, ic2, hll,
                                 loR, hiR);
                    hll_weights32(loL, hiL, loR, hiR, pg.An, w1, w2, w3);
                    float FL[4], FR[4];
                    m1_flux32(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, c2, ic2, FL);
                    m1_flux32(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, c2, ic2, FR);
                    float S1 = 0.0f, S2 = 0.0f, S3 = 0.0f;   // m . (F_L, F_R, U_R - U_L)
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        S1 += nu[m] * FL[m];
                        S2 += nu[m] * FR[m];
                        S3 += nu[m] * (qR[m] - qL[m]);
                        tL[m] = 2.0f * (w1 * tL[m] - w3 * nu[m]);
                        tR[m] = 2.0f * (w2 * tR[m] + w3 * nu[m]);
                    }
                    float gloL, ghiL, gloR, ghiR;
                    hll_weights32_vjp(loL, hiL, loR, hiR, pg.An, 2.0f * S1, 2.0f * S2, 2.0f * S3,
                                      gloL, ghiL, gloR, ghiR);
                    hll_speeds32_vjp(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, iAn, cf, ic2,
                                     hll, gloL, ghiL, tL);
                    hll_speeds32_vjp(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, iAn, cf, ic2,
                                     hll, gloR, ghiR, tR);
                } else {
                    const float dis = cf * pg.An;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        tL[m] += dis * nu[m];
                        tR[m] -= dis * nu[m];
                    }
                }
                guard32_vjp(qLp, tL, cf);
                guard32_vjp(qRp, tR, cf);
                if (use) {
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int q = 4 * g + m;
                        aU[q].add(tL[m]);
                        const float lm = own_slope[m] ? pg.fk * tL[m] - pg.fl * tR[m] : 0.0f;
                        aD[3 * q] += lm * pg.sx;
                        aD[3 * q + 1] += lm * pg.sy;
                        aD[3 * q + 2] += lm * pg.sz;
                    }
                }
            }
        }
    }
    if (!active) return;
    const float iV = rcp32(rk[F_V]);
    const float b00 = Bk[0] * iV, b01 = Bk[1] * iV, b02 = Bk[2] * iV;
    const float b11 = Bk[3] * iV, b12 = Bk[4] * iV, b22 = Bk[5] * iV;
#pragma unroll
    for (int g = 0; g < GW; ++g) {
        float *o = R + (i * G + g0 + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int q = 4 * g + m;
            o[m] = (float)((double)Li[q] + aU[q].value());
            o[4 + 3 * m + 0] = b00 * aD[3 * q] + b01 * aD[3 * q + 1] + b02 * aD[3 * q + 2];
            o[4 + 3 * m + 1] = b01 * aD[3 * q] + b11 * aD[3 * q + 1] + b12 * aD[3 * q + 2];
            o[4 + 3 * m + 2] = b02 * aD[3 * q] + b12 * aD[3 * q + 1] + b22 * aD[3 * q + 2];
        }
    }
}

// Q lanes share a particle, each taking every Q-th neighbour slot; the
// per-lane compensated sums are combined in FP64 by a fixed butterfly.
template <int G, int Q = 1>
__global__ __launch_bounds__(kBlock) void k_adj_grad32(
    int64_t n, int64_t nb, const float *__restrict__ geo32, const int32_t *__restrict__ nbr,
    const int64_t *__restrict__ wave_base, const int32_t *__restrict__ n_nbr,
    const float *__restrict__ R, float *__restrict__ lam, double box) {
    static_assert(Q == 1 || Q == 2 || Q == 4, "lanes per particle: 1, 2 or 4");
    constexpr int NQ = 4 * G, PW = 64 / Q, PB = kBlock / Q;
    __shared__ float stage[kBlock / 64][64 * kStage32];
    const int64_t blk = xcd_block(nb);
    if (blk >= nb) return;
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
    float *sb = stage[wv];
    const float *rp = geo32 + (int64_t)F_REC * ic;
    const double *xp = reinterpret_cast<const double *>(rp);
    const double px = xp[0], py = xp[1], pz = xp[2];
    const float iHp = rp[F_IH];
    Kahan acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q].s = acc[q].c = 0.0f;
    float sgx = 0.0f, sgy = 0.0f, sgz = 0.0f;
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
            int64_t row[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) row[m] = __shfl(j, 16 * m + (lane >> 2), 64);
            // all rows of this slot in flight before the first is staged
            constexpr int GC = G < 6 ? G : 6;
            float4 vp[4], vr[GC][4];
            load_rows32(geo32, row, lane, vp);
#pragma unroll
            for (int g = 0; g < GC; ++g) {
                int64_t rowg[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) rowg[m] = row[m] * G + g;
                load_rows32(R, rowg, lane, vr[g]);
            }
            store_rows32(vp, sb, lane);
            const float *rl = sb + lane * kStage32;
            double xl[3];
            {
                union { float f[2]; double d; } u;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u.f[0] = rl[2 * a];
                    u.f[1] = rl[2 * a + 1];
                    xl[a] = u.d;
                }
            }
            const float sx = (float)min_image(xl[0] - px, box, ibox);
            const float sy = (float)min_image(xl[1] - py, box, ibox);
            const float sz = (float)min_image(xl[2] - pz, box, ibox);
            const float r = sqrt32(sx * sx + sy * sy + sz * sz);
            const float wpi = valid ? kern_wf(r * iHp) : 0.0f;
            const float wip = valid ? kern_wf(r * rl[F_IH]) : 0.0f;
            sgx += wpi * sx;
            sgy += wpi * sy;
            sgz += wpi * sz;
#pragma unroll
            for (int c0 = 0; c0 < G; c0 += GC) {
                if (c0 > 0) {
#pragma unroll
                    for (int g = 0; g < GC; ++g) {
                        if (c0 + g >= G) break;
                        int64_t rowg[4];
#pragma unroll
                        for (int m = 0; m < 4; ++m) rowg[m] = row[m] * G + c0 + g;
                        load_rows32(R, rowg, lane, vr[g]);
                    }
                }
#pragma unroll
                for (int g = 0; g < GC; ++g) {
                    if (c0 + g >= G) break;
                    store_rows32(vr[g], sb, lane);
                    const float *Rl = sb + lane * kStage32;
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[4 * (c0 + g) + m].add(
                            -wip * (Rl[4 + 3 * m] * sx + Rl[5 + 3 * m] * sy + Rl[6 + 3 * m] * sz));
                }
            }
        }
    }
    double av[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) av[q] = acc[q].value();
    if (Q > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) quad_sum<Q>(av[q]);
        quad_sum<Q>(sgx);
        quad_sum<Q>(sgy);
        quad_sum<Q>(sgz);
    }
    if (!owner) return;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const float *Rp = R + (i * G + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            lam[(i * G + g) * 4 + m] = (float)(
                (double)Rp[m] - (double)(sgx * Rp[4 + 3 * m] + sgy * Rp[5 + 3 * m] + sgz * Rp[6 + 3 * m]) +
                av[4 * g + m]);
    }
}

// Groups per wave of the pair pass (0: all G); one group per wave keeps the
// pass at 135 VGPRs and 3 waves per SIMD for any G (all four groups of a
// G = 4 set in one wave need 276 registers: 1 wave per SIMD).
#ifndef RT_ADJ32_GW
#define RT_ADJ32_GW 1
#endif
// Lanes per particle of the FP32 transposed gradient (1, 2 or 4); 4 took the
// FP32C backward of the 128^3 adjoint workload from 188 to 166 ms.
#ifndef RT_ADJ32_GRAD_Q
#define RT_ADJ32_GRAD_Q 4
#endif
constexpr int kAGQ32 = RT_ADJ32_GRAD_Q;

template <int G>
void launch(rt_ctx *ctx, const float *UD, const float *Uung, const float *lam_next, float *lam2,
            float *R, float *lam, const double *dt) {
    const int64_t n = ctx->p.n, nb = (n + kBlock - 1) / kBlock;
    hipStream_t st = ctx->stream;
    constexpr int GW = (RT_ADJ32_GW == 0 || G % RT_ADJ32_GW != 0) ? G : RT_ADJ32_GW;
    k_adj_guard32<G><<<nblk(n * G), kBlock, 0, st>>>(n, Uung, lam_next, lam2, (float)ctx->p.c_red);
    const float2 *tab = (const float2 *)ctx->hll_table32;
    const bool iva = ctx->surfaces == RT_IVANOVA;
#define RT_ADJ32_PAIR_LAUNCH(HLL_, IVA_)                                                       \
    k_adj_pair32<G, GW, HLL_, IVA_><<<(unsigned)xcd_grid(nb * (G / GW)), kBlock, 0, st>>>(    \
        n, nb, ctx->geo32, ctx->geo, ctx->nbr, ctx->wave_base, ctx->n_nbr, UD, lam2, dt,       \
        ctx->p.c_red, ctx->p.box, R, tab, ctx->ivan)
    if (ctx->solver == RT_HLL) {
        if (iva) RT_ADJ32_PAIR_LAUNCH(true, true);
        else RT_ADJ32_PAIR_LAUNCH(true, false);
    } else {
        if (iva) RT_ADJ32_PAIR_LAUNCH(false, true);
        else RT_ADJ32_PAIR_LAUNCH(false, false);
    }
#undef RT_ADJ32_PAIR_LAUNCH
    const int64_t ng = (n + kBlock / kAGQ32 - 1) / (kBlock / kAGQ32);
    k_adj_grad32<G, kAGQ32><<<(unsigned)xcd_grid(ng), kBlock, 0, st>>>(
        n, ng, ctx->geo32, ctx->nbr, ctx->wave_base, ctx->n_nbr, R, lam, ctx->p.box);
}

}  // namespace

void rt_adjoint32(rt_ctx *ctx, const float *UD, const float *Uung, const float *lam_next,
                  float *lam2, float *R, float *lam, const double *dt) {
    switch (ctx->p.groups) {
        case 1: launch<1>(ctx, UD, Uung, lam_next, lam2, R, lam, dt); break;
        case 2: launch<2>(ctx, UD, Uung, lam_next, lam2, R, lam, dt); break;
        case 3: launch<3>(ctx, UD, Uung, lam_next, lam2, R, lam, dt); break;
        case 4: launch<4>(ctx, UD, Uung, lam_next, lam2, R, lam, dt); break;
        case 5: launch<5>(ctx, UD, Uung, lam_next, lam2, R, lam, dt); break;
        case 6: launch<6>(ctx, UD, Uung, lam_next, lam2, R, lam, dt); break;
        case 7: launch<7>(ctx, UD, Uung, lam_next, lam2, R, lam, dt); break;
        case 8: launch<8>(ctx, UD, Uung, lam_next, lam2, R, lam, dt); break;
        default: break;
    }
}
