// FP32 device functions of one neighbour pair (compensated-FP32 path), shared
// by the FP32 transport kernel and its adjoint.
#pragma once

#include "rt_internal.h"

namespace gearrt {
namespace {

constexpr int kStage32 = 17;   // floats per staged 16-float row (bank padding)

// Hardware FP32 reciprocal and square root (about one ulp).  FP32 denormals are
// flushed on this path: the square root of a product that underflowed is 0
// (never 0 * inf), which the callers treat as "no surface" / "no flux".
__device__ __forceinline__ float rcp32(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float sqrt32(float x) { return __builtin_amdgcn_sqrtf(fmaxf(x, 0.0f)); }

__device__ __forceinline__ void wave_lds_sync32() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Kahan-compensated running sum.
struct Kahan {
    float s, c;
    __device__ __forceinline__ void add(float x) {
        const float y = x - c;
        const float t = s + y;
        c = (t - s) - y;
        s = t;
    }
    __device__ __forceinline__ double value() const { return (double)s - (double)c; }
};

// Transport in FP32 with compensated accumulation.  Same scheme as the FP64
// kernel (guards, M1 closure rewritten without n = F/|F|, GLF, minmod).
__device__ __forceinline__ int guard32(float &E, float &Fx, float &Fy, float &Fz, float c) {
    int fired = 0;
    if (E < 0.0f) {
        E = 0.0f;
        fired = 1;
    }
    if (E == 0.0f) {
        Fx = Fy = Fz = 0.0f;
        return fired;
    }
    const float F2 = Fx * Fx + Fy * Fy + Fz * Fz;
    const float lim = c * E;
    if (F2 > lim * lim) {
        // |F| below 1e-19 (|F|^2 not a normal float) is scaled to the limit 0
        const float Fn = sqrt32(F2);
        const float sc = Fn > 0.0f ? lim * rcp32(Fn) : 0.0f;
        Fx *= sc;
        Fy *= sc;
        Fz *= sc;
        fired |= 2;
    }
    return fired;
}

// With g = F/E (|g| <= c after the guard) the closure needs no product that
// can leave the FP32 range: f^2 = |g|^2/c^2 and (F.A) F / E = (g.A) F.  Energy
// densities below 1e-30 carry no anisotropic term (their flux is below
// 1e-30 |A| c^2 / 3).
__device__ __forceinline__ void m1_flux32(float E, float Fx, float Fy, float Fz, float Ax,
                                          float Ay, float Az, float c2, float ic2, float out[4]) {
    const float FA = Fx * Ax + Fy * Ay + Fz * Az;
    const float iE = E > 1e-30f ? rcp32(E) : 0.0f;
    const float gx = Fx * iE, gy = Fy * iE, gz = Fz * iE;
    const float f2 = (gx * gx + gy * gy + gz * gz) * ic2;
    const float s = sqrt32(fmaxf(4.0f - 3.0f * f2, 0.0f));
    const float id = rcp32(2.0f + s);
    const float a = c2 * E * (1.0f / 3.0f - f2 * id);
    const float b = 3.0f * id * (gx * Ax + gy * Ay + gz * Az);
    out[0] = FA;
    out[1] = a * Ax + b * Fx;
    out[2] = a * Ay + b * Fy;
    out[3] = a * Az + b * Fz;
}

// HLL wave speeds of one face state in FP32 (eq:riemann-HLL; see
// hll_speeds64): bilinear in tab[RT_HLL_NF][RT_HLL_NMU] = (l_min, l_max)/c over
// f = |F|/(cE), clamped to 1, and mu = F.A/(|F||A|), clamped to [-1, 1], both
// formed from g = F/E as the FP32 closure is; a state with E <= 1e-30 or
// F = 0 is looked up at f = 0.  Every index stays in the table.
__device__ __forceinline__ void hll_speeds32(float E, float Fx, float Fy, float Fz, float Ax,
                                             float Ay, float Az, float iAn, float c, float ic2,
                                             const float2 *__restrict__ tab, float &lo,
                                             float &hi) {
    const float iE = E > 1e-30f ? rcp32(E) : 0.0f;
    const float gx = Fx * iE, gy = Fy * iE, gz = Fz * iE;
    const float g2 = gx * gx + gy * gy + gz * gz;
    float f = 0.0f, mu = 0.0f;
    if (g2 > 0.0f) {
        const float ig = __builtin_amdgcn_rsqf(g2);
        f = fminf(sqrt32(g2 * ic2), 1.0f);
        mu = fminf(fmaxf((gx * Ax + gy * Ay + gz * Az) * ig * iAn, -1.0f), 1.0f);
    }
    const float x = f * (RT_HLL_NF - 1), y = (mu + 1.0f) * (0.5f * (RT_HLL_NMU - 1));
    const int i = max(min((int)x, RT_HLL_NF - 2), 0);
    const int j = max(min((int)y, RT_HLL_NMU - 2), 0);
    const float tx = x - i, ty = y - j;
    const float2 *t = tab + i * RT_HLL_NMU + j;
    const float2 v00 = t[0], v01 = t[1], v10 = t[RT_HLL_NMU], v11 = t[RT_HLL_NMU + 1];
    const float ux = 1.0f - tx, uy = 1.0f - ty;
    lo = c * (ux * (uy * v00.x + ty * v01.x) + tx * (uy * v10.x + ty * v11.x));
    hi = c * (ux * (uy * v00.y + ty * v01.y) + tx * (uy * v10.y + ty * v11.y));
}

// HLL weights of Phi.A = w1 F_L.A + w2 F_R.A + w3 (U_R - U_L) (see hll_weights).
__device__ __forceinline__ void hll_weights32(float loL, float hiL, float loR, float hiR,
                                              float An, float &w1, float &w2, float &w3) {
    const float lp = fmaxf(fmaxf(hiL, hiR), 0.0f), lm = fminf(fminf(loL, loR), 0.0f);
    const float den = lp - lm;
    if (den > 0.0f) {
        const float id = rcp32(den);
        w1 = lp * id;
        w2 = -lm * id;
        w3 = lp * lm * An * id;
    } else {
        w1 = w2 = 0.5f;
        w3 = 0.0f;
    }
}

__device__ __forceinline__ float minmod32(float a, float b) {
    const float m = (fabsf(a) <= fabsf(b)) ? a : b;
    return (a * b > 0.0f) ? m : 0.0f;
}

// Copy one 16-float (64-byte) row per lane's neighbour into the wave's stage
// buffer: 4 loads, 4 lanes per row, 16 rows per load.  Load and store halves
// are separate so that several rows can be in flight before the first store.
__device__ __forceinline__ void load_rows32(const float *__restrict__ src, const int64_t (&row)[4],
                                            int lane, float4 (&v)[4]) {
    const int piece = lane & 3;
#pragma unroll
    for (int m = 0; m < 4; ++m)
        v[m] = *reinterpret_cast<const float4 *>(src + 16 * row[m] + 4 * piece);
}
__device__ __forceinline__ void store_rows32(const float4 (&v)[4], float *sb, int lane) {
    const int piece = lane & 3, slot = lane >> 2;
    wave_lds_sync32();
#pragma unroll
    for (int m = 0; m < 4; ++m) {
        float *d = sb + (16 * m + slot) * kStage32 + 4 * piece;
        d[0] = v[m].x;
        d[1] = v[m].y;
        d[2] = v[m].z;
        d[3] = v[m].w;
    }
    wave_lds_sync32();
}
__device__ __forceinline__ void stage_rows32(const float *__restrict__ src,
                                             const int64_t (&row)[4], float *sb, int lane) {
    float4 v[4];
    load_rows32(src, row, lane, v);
    store_rows32(v, sb, lane);
}

// VJP of guard32 at its input state q (see guard64_vjp).
__device__ __forceinline__ void guard32_vjp(const float q[4], float lam[4], float c) {
    const float E = q[0];
    if (E < 0.0f) {
        lam[0] = lam[1] = lam[2] = lam[3] = 0.0f;
        return;
    }
    if (E == 0.0f) {
        lam[1] = lam[2] = lam[3] = 0.0f;
        return;
    }
    const float F2 = q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    const float lim = c * E;
    if (F2 > lim * lim) {
        const float Fn = sqrt32(F2);
        if (!(Fn > 0.0f)) {          // forward set F = 0
            lam[1] = lam[2] = lam[3] = 0.0f;
            return;
        }
        const float iF = rcp32(Fn);
        const float nx = q[1] * iF, ny = q[2] * iF, nz = q[3] * iF;
        const float nl = nx * lam[1] + ny * lam[2] + nz * lam[3];
        const float sc = lim * iF;
        lam[0] += c * nl;
        lam[1] = sc * (lam[1] - nx * nl);
        lam[2] = sc * (lam[2] - ny * nl);
        lam[3] = sc * (lam[3] - nz * nl);
    }
}

// VJPs of the FP32 HLL weights and speeds (see hll_weights_vjp and
// hll_speeds64_vjp): the branch the forward takes at every kink; here f and mu
// come from g = F/E, so a state with E <= 1e-30 or g = 0 passes nothing.
__device__ __forceinline__ void hll_weights32_vjp(float loL, float hiL, float loR, float hiR,
                                                  float An, float S1, float S2, float S3,
                                                  float &gloL, float &ghiL, float &gloR,
                                                  float &ghiR) {
    gloL = ghiL = gloR = ghiR = 0.0f;
    const float mx = hiL >= hiR ? hiL : hiR, mn = loL <= loR ? loL : loR;
    const float lp = mx > 0.0f ? mx : 0.0f, lm = mn < 0.0f ? mn : 0.0f;
    const float den = lp - lm;
    if (!(den > 0.0f)) return;
    const float id = rcp32(den), id2 = id * id;
    const float glp = (-lm * S1 + lm * S2 - An * lm * lm * S3) * id2;
    const float glm = (lp * S1 - lp * S2 + An * lp * lp * S3) * id2;
    if (mx > 0.0f) (hiL >= hiR ? ghiL : ghiR) = glp;
    if (mn < 0.0f) (loL <= loR ? gloL : gloR) = glm;
}
__device__ __forceinline__ void hll_speeds32_vjp(float E, float Fx, float Fy, float Fz, float Ax,
                                                 float Ay, float Az, float iAn, float c,
                                                 float ic2, const float2 *__restrict__ tab,
                                                 float glo, float ghi, float (&t)[4]) {
    const float iE = E > 1e-30f ? rcp32(E) : 0.0f;
    const float gx = Fx * iE, gy = Fy * iE, gz = Fz * iE;
    const float g2 = gx * gx + gy * gy + gz * gz;
    if (!(g2 > 0.0f)) return;
    const float ig = __builtin_amdgcn_rsqf(g2);
    const float fr = sqrt32(g2 * ic2);
    const float mr = (gx * Ax + gy * Ay + gz * Az) * ig * iAn;
    const float f = fminf(fr, 1.0f), mu = fminf(fmaxf(mr, -1.0f), 1.0f);
    const float x = f * (RT_HLL_NF - 1), y = (mu + 1.0f) * (0.5f * (RT_HLL_NMU - 1));
    const int i = max(min((int)x, RT_HLL_NF - 2), 0);
    const int j = max(min((int)y, RT_HLL_NMU - 2), 0);
    const float tx = x - i, ty = y - j;
    const float2 *tb = tab + i * RT_HLL_NMU + j;
    const float2 v00 = tb[0], v01 = tb[1], v10 = tb[RT_HLL_NMU], v11 = tb[RT_HLL_NMU + 1];
    const float ux = 1.0f - tx, uy = 1.0f - ty;
    const float gxx = glo * (uy * (v10.x - v00.x) + ty * (v11.x - v01.x)) +
                      ghi * (uy * (v10.y - v00.y) + ty * (v11.y - v01.y));
    const float gyy = glo * (ux * (v01.x - v00.x) + tx * (v11.x - v10.x)) +
                      ghi * (ux * (v01.y - v00.y) + tx * (v11.y - v10.y));
    const float gf = c * gxx * (RT_HLL_NF - 1), gm = c * gyy * (0.5f * (RT_HLL_NMU - 1));
    if (fr <= 1.0f) {            // f = |g|/c: df/dE = -f/E, df/dF = g/(|g| c E)
        const float k = gf * ig * iE * (c * ic2);   // (1/c) g/|g| / E
        t[0] -= gf * fr * iE;
        t[1] += k * gx;
        t[2] += k * gy;
        t[3] += k * gz;
    }
    if (mr >= -1.0f && mr <= 1.0f) {   // dmu/dF = (A/|A| - mu g/|g|) / |F|
        const float a = gm * ig * iE * iAn, b = gm * mr * ig * ig * iE;
        t[1] += a * Ax - b * gx;
        t[2] += a * Ay - b * gy;
        t[3] += a * Az - b * gz;
    }
}
// Ivanova surface (eq:IvanovaAij) in FP32 for the pair k, l: separation s,
// distance r, the particles' 1/H, V and kernel-gradient sums g.
__device__ __forceinline__ void ivanova_surface32(float sx, float sy, float sz, float r, float iHk,
                                                  float Vk, const float (&gk)[3], float iHl,
                                                  float Vl, const float (&gl)[3], float &Ax,
                                                  float &Ay, float &Az) {
    const float qk = r * iHk, ql = r * iHl;
    const float sk = (float)kSigma3 * Vk * Vk * iHk * iHk * iHk;
    const float sl = (float)kSigma3 * Vl * Vl * iHl * iHl * iHl;
    const float ir = r > 0.0f ? rcp32(r) : 0.0f;
    const float a = -(sk * iHk * kern_dwf(qk) + sl * iHl * kern_dwf(ql)) * ir;
    const float bk = sk * Vk * kern_wf(qk), bl = sl * Vl * kern_wf(ql);
    Ax = a * sx - bk * gk[0] + bl * gl[0];
    Ay = a * sy - bk * gk[1] + bl * gl[1];
    Az = a * sz - bk * gk[2] + bl * gl[2];
}

// VJP of m1_flux32 (see m1_flux64_vjp for the formulas).
__device__ __forceinline__ void m1_flux32_vjp(float E, float Fx, float Fy, float Fz, float Ax,
                                              float Ay, float Az, float c2, float ic2,
                                              const float nu[4], float out[4]) {
    const float iE = E > 1e-30f ? rcp32(E) : 0.0f;
    const float gx = Fx * iE, gy = Fy * iE, gz = Fz * iE;
    const float f2 = (gx * gx + gy * gy + gz * gz) * ic2;
    const float s = sqrt32(fmaxf(4.0f - 3.0f * f2, 0.0f));
    const float is = rcp32(s);
    const float id = rcp32(2.0f + s);
    const float gA = gx * Ax + gy * Ay + gz * Az;
    const float b = 3.0f * id * gA;
    const float al = nu[1] * Ax + nu[2] * Ay + nu[3] * Az;
    const float ng = nu[1] * gx + nu[2] * gy + nu[3] * gz;
    const float k1 = id + 1.5f * id * id * f2 * is;
    const float k2 = id + 3.0f * id * id * f2 * is;
    const float t = 3.0f * ng;
    const float tg = -2.0f * al * k1 + t * 3.0f * id * id * gA * is * ic2;
    out[0] = al * c2 * (1.0f / 3.0f + f2 * k2) - t * gA * k2;
    out[1] = nu[0] * Ax + tg * gx + t * id * Ax + b * nu[1];
    out[2] = nu[0] * Ay + tg * gy + t * id * Ay + b * nu[2];
    out[3] = nu[0] * Az + tg * gz + t * id * Az + b * nu[3];
}

// Geometry of one pair from the staged FP32 record rl of the neighbour and the
// own FP64 position / FP32 record fields.
struct PairGeo32 {
    float sx, sy, sz, Ax, Ay, Az, An, fk, fl;
};

__device__ __forceinline__ void pair_geometry32(double pkx, double pky, double pkz, float iHk,
                                                float hk, const float (&Bk)[6],
                                                const float *__restrict__ rl, double box,
                                                double ibox, PairGeo32 &pg) {
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
    pg.sx = (float)min_image(xl[0] - pkx, box, ibox);
    pg.sy = (float)min_image(xl[1] - pky, box, ibox);
    pg.sz = (float)min_image(xl[2] - pkz, box, ibox);
    const float r = sqrt32(pg.sx * pg.sx + pg.sy * pg.sy + pg.sz * pg.sz);
    const float wk = kern_wf(r * iHk);
    const float wl = kern_wf(r * rl[F_IH]);
    const float m00 = wk * Bk[0] + wl * rl[F_B + 0];
    const float m01 = wk * Bk[1] + wl * rl[F_B + 1];
    const float m02 = wk * Bk[2] + wl * rl[F_B + 2];
    const float m11 = wk * Bk[3] + wl * rl[F_B + 3];
    const float m12 = wk * Bk[4] + wl * rl[F_B + 4];
    const float m22 = wk * Bk[5] + wl * rl[F_B + 5];
    pg.Ax = m00 * pg.sx + m01 * pg.sy + m02 * pg.sz;
    pg.Ay = m01 * pg.sx + m11 * pg.sy + m12 * pg.sz;
    pg.Az = m02 * pg.sx + m12 * pg.sy + m22 * pg.sz;
    pg.An = sqrt32(pg.Ax * pg.Ax + pg.Ay * pg.Ay + pg.Az * pg.Az);
    const float hl = rl[F_H];
    const float ih = rcp32(hk + hl);
    pg.fk = hk * ih;
    pg.fl = hl * ih;
}

}  // namespace
}  // namespace gearrt
