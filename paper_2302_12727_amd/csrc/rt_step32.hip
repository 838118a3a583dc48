// Compensated-FP32 variants of the gradient and transport kernels.
//
// State, gradient records and all pair arithmetic are FP32; each particle sums
// its pair fluxes with Kahan compensation (sum, comp) in FP32, and the final
// update combines sum and compensation once in FP64 before rounding the new
// state to FP32.  FP64 stays in the geometry (separations from FP64 positions,
// the FP64 inversion of S_i in the build) and in the photon budget.
#include "rt_pair32.h"

using namespace gearrt;

// Waves per SIMD of the GLF FP32C transport up to 3 groups.
#ifndef RT_TRANSPORT32_WAVES
#define RT_TRANSPORT32_WAVES 3
#endif
// 1: the FP32C transport with Hopkins surfaces evaluates in-tile pairs
// once (k_transport32_tile); 0: always two-sided.
#ifndef RT_TRANSPORT32_TILE
#define RT_TRANSPORT32_TILE 1
#endif
// The HLL solver takes the FP32C tiles too; 0 keeps it two-sided.
#ifndef RT_TRANSPORT32_TILE_HLL
#define RT_TRANSPORT32_TILE_HLL 1
#endif
// The time-bin ticks too; 0 keeps them two-sided.
#ifndef RT_TICK32_TILE
#define RT_TICK32_TILE 1
#endif
// ... with their gradients from the neighbour unions; 0: staged.
#ifndef RT_TICK_UNION32
#define RT_TICK_UNION32 1
#endif
// The Ivanova surfaces too; 0 keeps them two-sided.
#ifndef RT_TRANSPORT32_TILE_IVA
#define RT_TRANSPORT32_TILE_IVA 1
#endif

namespace {

// ---------------------------------------------------------------------------
// Gradient (eq:gradient) in FP32, S_i^{-1} sum_j (q_j - q_i) w(r_ij/H_i) s_ij.
// Q lanes share a particle as in the FP64 gradient.  BIN: only the particles
// that end a step in tick `tick` (time bin in slot F_BIN) recompute theirs.
template <int G, int Q = 1, bool BIN = false>
__global__ __launch_bounds__(kBlock) void k_gradient32(
    int64_t n, int64_t nb, const float *__restrict__ geo32, const double *__restrict__ xs,
    const int32_t *__restrict__ nbr, const int64_t *__restrict__ wave_base,
    const int32_t *__restrict__ n_gath, const float *__restrict__ U, float *__restrict__ UD,
    int32_t *__restrict__ status, double box, int64_t tick = 0,
    const int32_t *__restrict__ blist = nullptr, int64_t n_list = 0) {
    static_assert(Q == 1 || Q == 2 || Q == 4, "lanes per particle: 1, 2 or 4");
    const int64_t bx = xcd_block(nb);
    if (bx >= nb) return;
    const int sub = (threadIdx.x & 63) % Q;
    int64_t i = bx * (kBlock / Q) + threadIdx.x / Q;
    if (blist) {                                // only the listed 64-particle blocks, 4 / Q a block
        const int64_t e = bx * (4 / Q) + (threadIdx.x / Q) / 64;
        if (e >= n_list) return;
        i = (int64_t)blist[e] * 64 + (threadIdx.x / Q) % 64;
    }
    if (i >= n) return;                         // a particle's Q lanes leave together
    if (BIN && ((tick + 1) & ((int64_t(1) << (int32_t)geo32[(int64_t)F_REC * i + F_BIN]) - 1)) != 0)
        return;
    constexpr int NQ = 4 * G;
    const double ibox = 1.0 / box;
    const float *rec = geo32 + (int64_t)F_REC * i;
    const double px = xs[3 * i], py = xs[3 * i + 1], pz = xs[3 * i + 2];
    const float iH = rec[F_IH], iV = 1.0f / rec[F_V];
    float Ui[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) Ui[q] = U[i * NQ + q];
    float acc[NQ][3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0f;
    const int64_t base = wave_base[i >> 6] + (i & 63);
    const int32_t ng = n_gath[i];
    // the next neighbour index is loaded one iteration ahead
    int64_t jn = sub < ng ? nbr[base + 64 * (int64_t)sub] : 0;
    for (int32_t k = sub; k < ng; k += Q) {
        const int64_t j = jn;
        if (k + Q < ng) jn = nbr[base + 64 * (int64_t)(k + Q)];
        const float sx = (float)min_image(xs[3 * j] - px, box, ibox);
        const float sy = (float)min_image(xs[3 * j + 1] - py, box, ibox);
        const float sz = (float)min_image(xs[3 * j + 2] - pz, box, ibox);
        const float w = kern_wf(sqrt32(sx * sx + sy * sy + sz * sz) * iH);
        const float wx = w * sx, wy = w * sy, wz = w * sz;
        const float *Uj = U + j * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const float d = Uj[q] - Ui[q];
            acc[q][0] += d * wx;
            acc[q][1] += d * wy;
            acc[q][2] += d * wz;
        }
    }
    if (Q > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                quad_sum<Q>(acc[q][a]);
        if (sub != 0) return;
    }
    const float b00 = rec[F_B] * iV, b01 = rec[F_B + 1] * iV, b02 = rec[F_B + 2] * iV;
    const float b11 = rec[F_B + 3] * iV, b12 = rec[F_B + 4] * iV, b22 = rec[F_B + 5] * iV;
    // chk stays 0 unless a value written is NaN or infinite
    float chk = 0.0f;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        float *o = UD + (i * G + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const int q = 4 * g + m;
            const float d0 = b00 * acc[q][0] + b01 * acc[q][1] + b02 * acc[q][2];
            const float d1 = b01 * acc[q][0] + b11 * acc[q][1] + b12 * acc[q][2];
            const float d2 = b02 * acc[q][0] + b12 * acc[q][1] + b22 * acc[q][2];
            o[m] = Ui[q];
            o[4 + 3 * m + 0] = d0;
            o[4 + 3 * m + 1] = d1;
            o[4 + 3 * m + 2] = d2;
            chk = __builtin_fmaf(Ui[q], 0.0f, chk);
            chk = __builtin_fmaf(d0, 0.0f, chk);
            chk = __builtin_fmaf(d1, 0.0f, chk);
            chk = __builtin_fmaf(d2, 0.0f, chk);
        }
    }
    if (chk != chk) atomicOr(status, ST_NONFINITE);
}

// four floats as one 16-byte access (a native vector: copies stay in registers)
typedef float fvec4 __attribute__((ext_vector_type(4)));

// quad broadcast: every lane of a quad takes lane L's value (DPP quad_perm)
template <int L>
__device__ __forceinline__ float quad_bcast(float v) {
    return __builtin_bit_cast(
        float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), L * 0x55, 0xf, 0xf, false));
}
template <int L>
__device__ __forceinline__ int quad_bcast(int v) {
    return __builtin_amdgcn_mov_dpp(v, L * 0x55, 0xf, 0xf, false);
}

// Gradient from the block's neighbour union in FP32 (compensated mode, up to
// 4 groups; see k_gradient64u): the union's FP32 states (16G bytes a row) and
// FP64 positions are staged in LDS once per block of 64 particles, and every
// pair reads its neighbour's row from LDS by its 16-bit position in the union.
// Three blocks per CU, 3 waves per SIMD.
//
// A particle's four lanes form a quad.  Each lane forms the pair geometry
// w(r/H_i) s of every fourth neighbour, the quad shares the four by DPP
// broadcasts, and lane m then accumulates component m (E, F_x, F_y, F_z) of
// every group over all neighbours in list order: every sum is formed in the
// same order and with the same operations as one lane per particle
// (k_gradient32 with Q = 1), so the two give identical bits (see
// RT_GRADIENT32_Q for why that order is kept).  Padding past a list is the
// own row, which adds an exact zero.  Blocks whose union did not fit are
// left to k_gradient32 with one lane per particle.  BIN: only the particles
// that end a step in tick `tick` recompute their record; a block none of
// whose particles does so stages nothing.
template <int G, bool BIN = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3, 3))) void
k_gradient32u(int64_t n, int64_t nb, const float *__restrict__ geo32, const double *__restrict__ xs,
              const int32_t *__restrict__ urow, const int64_t *__restrict__ uoff,
              const uint16_t *__restrict__ gloc, const int64_t *__restrict__ goff,
              const uint16_t *__restrict__ uown, const int32_t *__restrict__ n_gath,
              const float *__restrict__ U, float *__restrict__ UD, int32_t *__restrict__ status,
              double box, int64_t tick = 0) {
    constexpr int Q = 4, UC = union_cap32(G);
    static_assert(kBlock == 256 && UC > 0 && UC <= kUnionSort, "64 particles per block");
    __shared__ fvec4 ust[UC * G];              // G pieces of 16 bytes a row
    __shared__ double upos[UC * 3];
    __shared__ int32_t uidx[UC];
    const int64_t blk = xcd_block(nb);
    if (blk >= nb) return;                      // whole block
    const int64_t u0 = uoff[blk];
    const int32_t rows = (int32_t)(uoff[blk + 1] - u0);
    if (rows == 0) return;                      // left to k_gradient32 (whole block)
    if constexpr (BIN) {
        const int64_t ib = blk * (kBlock / Q) + threadIdx.x / Q;
        const bool e = ib < n && ((tick + 1) & ((int64_t(1) << (int32_t)geo32[(int64_t)F_REC * ib + F_BIN]) - 1)) == 0;
        if (!__syncthreads_or(e)) return;       // whole block: no particle ends a step
    }
    for (int e = threadIdx.x; e < rows; e += kBlock) uidx[e] = urow[u0 + e];
    __syncthreads();
    const fvec4 *U4 = reinterpret_cast<const fvec4 *>(U);
    const int ts = rows * G, tp = rows * 3;
    {   // positions, then states (one set of loads in flight at a time)
        constexpr int MP = (UC * 3 + kBlock - 1) / kBlock;
        double x[MP];
#pragma unroll
        for (int r = 0; r < MP; ++r) {
            const int e = threadIdx.x + r * kBlock;
            if (e < tp) x[r] = xs[(uint32_t)uidx[e / 3] * 3u + (uint32_t)(e % 3)];
        }
#pragma unroll
        for (int r = 0; r < MP; ++r)
            if (threadIdx.x + r * kBlock < tp) upos[threadIdx.x + r * kBlock] = x[r];
    }
    {
        constexpr int MS = (UC * G + kBlock - 1) / kBlock;
        fvec4 v[MS];
#pragma unroll
        for (int r = 0; r < MS; ++r) {
            const int e = threadIdx.x + r * kBlock;
            if (e < ts) v[r] = U4[(uint32_t)uidx[e / G] * (uint32_t)G + (uint32_t)(e % G)];
        }
#pragma unroll
        for (int r = 0; r < MS; ++r)
            if (threadIdx.x + r * kBlock < ts) ust[threadIdx.x + r * kBlock] = v[r];
    }
    __syncthreads();
    const int sub = threadIdx.x % Q;            // the component this lane sums
    const int p = threadIdx.x / Q;              // the particle in the block
    const int64_t i = blk * (kBlock / Q) + p;
    const bool active =
        i < n && (!BIN || ((tick + 1) & ((int64_t(1) << (int32_t)geo32[(int64_t)F_REC * i + F_BIN]) - 1)) == 0);
    const int64_t ic = active ? i : n - 1;
    const int32_t ng = active ? n_gath[ic] : 0;
    const int il = active ? (int)uown[ic] : 0;  // a row of the union (not used past n)
    int32_t kmax = ng;                          // the wave's longest list
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
    const float *rec = geo32 + (int64_t)F_REC * ic;
    const double ibox = 1.0 / box;
    const float iH = rec[F_IH];
    const float *ustf = reinterpret_cast<const float *>(ust) + sub;
    float Ui[G];                                // component sub of every group
#pragma unroll
    for (int t = 0; t < G; ++t) Ui[t] = ustf[(il * G + t) * 4];
    const double px = upos[3 * il], py = upos[3 * il + 1], pz = upos[3 * il + 2];
    float acc[G][3];
#pragma unroll
    for (int t = 0; t < G; ++t) acc[t][0] = acc[t][1] = acc[t][2] = 0.0f;
    if (kmax > 0) {
        // the four neighbours 4 it + 0..3: this lane's geometry for 4 it + sub,
        // then every lane adds all four to its component
        auto four_pairs = [&](int jl) __attribute__((always_inline)) {
            const float sx = (float)min_image(upos[3 * jl] - px, box, ibox);
            const float sy = (float)min_image(upos[3 * jl + 1] - py, box, ibox);
            const float sz = (float)min_image(upos[3 * jl + 2] - pz, box, ibox);
            const float w = kern_wf(sqrt32(sx * sx + sy * sy + sz * sz) * iH);
            const float wx = w * sx, wy = w * sy, wz = w * sz;
            auto one = [&](int jq, float qx, float qy, float qz) __attribute__((always_inline)) {
#pragma unroll
                for (int t = 0; t < G; ++t) {
                    const float d = ustf[(jq * G + t) * 4] - Ui[t];
                    acc[t][0] += d * qx;
                    acc[t][1] += d * qy;
                    acc[t][2] += d * qz;
                }
            };
            one(quad_bcast<0>(jl), quad_bcast<0>(wx), quad_bcast<0>(wy), quad_bcast<0>(wz));
            one(quad_bcast<1>(jl), quad_bcast<1>(wx), quad_bcast<1>(wy), quad_bcast<1>(wz));
            one(quad_bcast<2>(jl), quad_bcast<2>(wx), quad_bcast<2>(wy), quad_bcast<2>(wz));
            one(quad_bcast<3>(jl), quad_bcast<3>(wx), quad_bcast<3>(wy), quad_bcast<3>(wz));
        };
        // packed table entries, as in k_gradient64u
        const int64_t g0 = goff[blk];
        const int ngb = (int)((goff[blk + 1] - g0) >> 10);      // the block's groups
        const uint64_t *gw = reinterpret_cast<const uint64_t *>(gloc + g0) + threadIdx.x;
        auto word = [&](int gq) __attribute__((always_inline)) {
            return gw[(int64_t)(gq < ngb ? gq : ngb - 1) * 256];
        };
        const int T = (kmax + Q - 1) / Q, ngq = (T + 3) / 4;    // this wave's iterations, groups
        auto four = [&](uint64_t wd, int gq) __attribute__((always_inline)) {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (4 * gq + u < T) {                            // wave-uniform
                    const int k = Q * (4 * gq + u) + sub;
                    four_pairs(k < ng ? (int)((wd >> (16 * u)) & 0xffff) : il);
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
    if (!active) return;
    // the record, as k_gradient32 forms it: lane m writes state m and the
    // gradient of component m of every group
    const float iV = 1.0f / rec[F_V];
    const float b00 = rec[F_B] * iV, b01 = rec[F_B + 1] * iV, b02 = rec[F_B + 2] * iV;
    const float b11 = rec[F_B + 3] * iV, b12 = rec[F_B + 4] * iV, b22 = rec[F_B + 5] * iV;
    float chk = 0.0f;
#pragma unroll
    for (int t = 0; t < G; ++t) {
        const float d0 = b00 * acc[t][0] + b01 * acc[t][1] + b02 * acc[t][2];
        const float d1 = b01 * acc[t][0] + b11 * acc[t][1] + b12 * acc[t][2];
        const float d2 = b02 * acc[t][0] + b12 * acc[t][1] + b22 * acc[t][2];
        float *o = UD + (ic * G + t) * 16;
        o[sub] = Ui[t];
        o[4 + 3 * sub + 0] = d0;
        o[4 + 3 * sub + 1] = d1;
        o[4 + 3 * sub + 2] = d2;
        chk = __builtin_fmaf(Ui[t], 0.0f, chk);
        chk = __builtin_fmaf(d0, 0.0f, chk);
        chk = __builtin_fmaf(d1, 0.0f, chk);
        chk = __builtin_fmaf(d2, 0.0f, chk);
    }
    if (chk != chk) atomicOr(status, ST_NONFINITE);
}

// HLL: the HLL solver (eq:riemann-HLL) with the FP32 copy of the wave-speed
// table in place of GLF.  Up to 3 groups the HLL instantiation is held to 3
// waves per SIMD (168 registers, 2 spilled), measured 10% faster than the 2
// its 184 registers would give.
//
// Q lanes share a particle, each taking every Q-th neighbour slot (see the
// FP64 transport); the per-lane compensated sums are combined in FP64 by a
// fixed butterfly.
//
// IVA: the Ivanova surfaces (eq:IvanovaAij) in FP32 from the records' V and
// 1/H and the kernel-gradient sums ivan (FP64, rounded to FP32 on load), the
// separation from the FP64 positions as for the Hopkins surfaces.
//
// BIN: one tick of the individual-time-step scheme, as in the FP64 transport
// (bins from the FP64 records' slot 12, the neighbourhoods' smallest from
// binm, and the FP32 records' F_BIN;
// each due pair's exchange weighted by dt 2^min(b_k, b_l) in the compensated
// sums; pending sums accm in FP64).
template <int G, bool HLL = false, int Q = 1, bool IVA = false, bool BIN = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    G <= 3 ? (HLL ? 3 : RT_TRANSPORT32_WAVES) : 1))) void k_transport32(
    int64_t n, int64_t nb, const float *__restrict__ geo32, const double *__restrict__ geo,
    const int32_t *__restrict__ nbr, const int64_t *__restrict__ wave_base,
    const int32_t *__restrict__ n_nbr, const float *__restrict__ UD,
    const double *__restrict__ dtp, double c, double box, float *__restrict__ Uout,
    double *__restrict__ partials, unsigned long long *__restrict__ counts,
    float *__restrict__ Uung, int32_t *__restrict__ status,
    const float2 *__restrict__ hll = nullptr, const double *__restrict__ ivan = nullptr,
    int64_t tick = 0, double *__restrict__ accm = nullptr,
    const uint8_t *__restrict__ binm = nullptr) {
    static_assert(Q == 1 || Q == 2 || Q == 4, "lanes per particle: 1, 2 or 4");
    // PIPE: the next stage's rows in flight during each evaluation (GLF; the
    // HLL instantiation has no registers left for them)
    constexpr bool PIPE = !HLL;
    constexpr int NQ = 4 * G, PW = 64 / Q, PB = kBlock / Q;
    __shared__ float stage[kBlock / 64][64 * kStage32];
    __shared__ double smem[(kBlock / 64) * 2 * G];
    __shared__ unsigned long long scnt[4];
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
    const float cf = (float)c, c2 = (float)(c * c), ic2 = (float)(1.0 / (c * c)), hc = 0.5f * cf;
    if (threadIdx.x < 4) scnt[threadIdx.x] = 0;
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
    float Ui[NQ], Di[NQ * 3];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const float *r = UD + (ic * G + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            Ui[4 * g + m] = r[m];
            Di[3 * (4 * g + m) + 0] = r[4 + 3 * m];
            Di[3 * (4 * g + m) + 1] = r[5 + 3 * m];
            Di[3 * (4 * g + m) + 2] = r[6 + 3 * m];
        }
    }
    Kahan acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q].s = acc[q].c = 0.0f;
    int cE = 0, cF = 0;
    // time bins: this particle ends a step in this tick (ends), or some pair of
    // its neighbourhood does (touched)
    const int64_t t1 = tick + 1;
    const int32_t bk = BIN ? (int32_t)geo[(int64_t)kRec * ic + 12] : 0;
    const bool ends = !BIN || (t1 & ((int64_t(1) << bk) - 1)) == 0;
    const int32_t bm = (BIN && binm) ? (int32_t)binm[ic] : 0;
    const bool touched = !BIN || (t1 & ((int64_t(1) << bm) - 1)) == 0;

    if (wave_live) {
        const int64_t base = wave_base[w] + (i & 63);
        int32_t kmax = (int32_t)((wave_base[w + 1] - wave_base[w]) >> 6);
        const int32_t nn = (active && touched) ? n_nbr[i] : 0;
        if (Q > 1) {                            // the longest list of this wave's particles
            kmax = nn;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
        }
        if (BIN && __ballot(nn > 0) == 0) kmax = 0;   // no due pair in this wave
        // Rows in flight: v holds the loads of the next stage (the geometry
        // rows, then each group's record rows) while the current stage is
        // evaluated from the stage buffer.  The next iteration's neighbour
        // index is loaded one iteration ahead.
        int32_t jc = sub < nn ? nbr[base + 64 * (int64_t)sub] : (int32_t)ic;
        int64_t row[4];
        float4 v[4];
        if constexpr (PIPE) {
#pragma unroll
            for (int m = 0; m < 4; ++m) row[m] = __shfl(jc, 16 * m + (lane >> 2), 64);
            load_rows32(geo32, row, lane, v);
        }
        for (int32_t kk = 0; kk < kmax; kk += Q) {
            const int32_t k = kk + sub;
            const bool valid = k < nn;
            const int32_t j = jc;
            // (slot 0 of the wave's table exists once kmax > 0: no branch
            // around the load, whose wait would then be a full one)
            const int32_t jl = nbr[base + 64 * (int64_t)(k + Q < nn ? k + Q : 0)];
            const int32_t jn = k + Q < nn ? jl : (int32_t)ic;
            if constexpr (!PIPE) {
#pragma unroll
                for (int m = 0; m < 4; ++m) row[m] = __shfl(j, 16 * m + (lane >> 2), 64);
                load_rows32(geo32, row, lane, v);
            }
            store_rows32(v, sb, lane);          // the geometry rows
            if constexpr (PIPE) {
                int64_t rowg[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) rowg[m] = row[m] * G;
                load_rows32(UD, rowg, lane, v);
            }
            const float *rl = sb + lane * kStage32;
            // separation in FP64 from FP64 positions, rounded once
            double xl[3];
            {
                // the staged row holds the three doubles as six floats
                union { float f[2]; double d; } u;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    u.f[0] = rl[2 * a];
                    u.f[1] = rl[2 * a + 1];
                    xl[a] = u.d;
                }
            }
            const float sx = (float)min_image(xl[0] - pkx, box, ibox);
            const float sy = (float)min_image(xl[1] - pky, box, ibox);
            const float sz = (float)min_image(xl[2] - pkz, box, ibox);
            const float r = sqrt32(sx * sx + sy * sy + sz * sz);
            float Ax, Ay, Az;
            if (IVA) {
                const double *gd = ivan + 4 * (int64_t)j;
                const float gl[3] = {(float)gd[0], (float)gd[1], (float)gd[2]};
                ivanova_surface32(sx, sy, sz, r, iHk, rk[F_V], gk, rl[F_IH], rl[F_V], gl, Ax, Ay,
                                  Az);
            } else {
                const float wk = kern_wf(r * iHk);
                const float wl = kern_wf(r * rl[F_IH]);
                const float m00 = wk * Bk[0] + wl * rl[F_B + 0];
                const float m01 = wk * Bk[1] + wl * rl[F_B + 1];
                const float m02 = wk * Bk[2] + wl * rl[F_B + 2];
                const float m11 = wk * Bk[3] + wl * rl[F_B + 3];
                const float m12 = wk * Bk[4] + wl * rl[F_B + 4];
                const float m22 = wk * Bk[5] + wl * rl[F_B + 5];
                Ax = m00 * sx + m01 * sy + m02 * sz;
                Ay = m01 * sx + m11 * sy + m12 * sz;
                Az = m02 * sx + m12 * sy + m22 * sz;
            }
            const float An = sqrt32(Ax * Ax + Ay * Ay + Az * Az);
            const float hl = rl[F_H];
            const float ih = rcp32(hk + hl);
            const float fk = hk * ih, fl = hl * ih;
            bool use = valid && An > 0.0f;
            float wkl = 1.0f;                   // time integration of this exchange
            if (BIN) {
                const int32_t bl = (int32_t)rl[F_BIN];
                const int32_t bmin = bk < bl ? bk : bl;
                use = use && (t1 & ((int64_t(1) << bmin) - 1)) == 0;
                wkl = (float)ldexp(dtp[0], bmin);
            }
            const float iAn = (HLL && An > 0.0f) ? rcp32(An) : 0.0f;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                // the stages in program order: each one's loads stay in
                // flight across the evaluation of the previous one
                if constexpr (PIPE) {
                    __builtin_amdgcn_sched_barrier(0);
                } else {
                    int64_t rowg[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) rowg[m] = row[m] * G + g;
                    load_rows32(UD, rowg, lane, v);
                }
                store_rows32(v, sb, lane);      // group g's record rows
                if constexpr (PIPE) {
                    if (g + 1 < G) {
                        int64_t rowg[4];
#pragma unroll
                        for (int m = 0; m < 4; ++m) rowg[m] = row[m] * G + g + 1;
                        load_rows32(UD, rowg, lane, v);
                    } else {                    // the next iteration's geometry rows
#pragma unroll
                        for (int m = 0; m < 4; ++m) row[m] = __shfl(jn, 16 * m + (lane >> 2), 64);
                        load_rows32(geo32, row, lane, v);
                    }
                }
                const float *Rl = sb + lane * kStage32;
                float qL[4], qR[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int q = 4 * g + m;
                    const float dk = Di[3 * q] * sx + Di[3 * q + 1] * sy + Di[3 * q + 2] * sz;
                    const float dl = Rl[4 + 3 * m] * sx + Rl[5 + 3 * m] * sy + Rl[6 + 3 * m] * sz;
                    const float mm = minmod32(dk, dl);
                    qL[m] = Ui[q] + fk * mm;
                    qR[m] = Rl[m] - fl * mm;
                }
                const int f1 = guard32(qL[0], qL[1], qL[2], qL[3], cf);
                const int f2 = guard32(qR[0], qR[1], qR[2], qR[3], cf);
                float w1 = 0.5f, w2 = 0.5f, w3 = -hc * An;   // GLF
                if (HLL) {
                    float loL, hiL, loR, hiR;
                    hll_speeds32(qL[0], qL[1], qL[2], qL[3], Ax, Ay, Az, iAn, cf, ic2, hll, loL,
                                 hiL);
                    hll_speeds32(qR[0], qR[1], qR[2], qR[3], Ax, Ay, Az, iAn, cf, ic2, hll, loR,
                                 hiR);
                    hll_weights32(loL, hiL, loR, hiR, An, w1, w2, w3);
                }
                float FL[4], FR[4];
                m1_flux32(qL[0], qL[1], qL[2], qL[3], Ax, Ay, Az, c2, ic2, FL);
                m1_flux32(qR[0], qR[1], qR[2], qR[3], Ax, Ay, Az, c2, ic2, FR);
                if (use) {
                    cE += (f1 & 1) + (f2 & 1);
                    cF += (f1 >> 1) + (f2 >> 1);
#pragma unroll
                    for (int m = 0; m < 4; ++m)
                        acc[4 * g + m].add(wkl * (w1 * FL[m] + w2 * FR[m] + w3 * (qR[m] - qL[m])));
                }
            }
            jc = jn;
            if constexpr (PIPE) __builtin_amdgcn_sched_barrier(0);
        }
    }
    double av[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) av[q] = acc[q].value();
    if (Q > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
            quad_sum<Q>(av[q]);
    }
    double red[2 * G];
    int gE = 0, gF = 0;
    float chk = 0.0f;   // NaN iff an updated state is NaN or infinite
    if (BIN && owner && !ends) {
        // no update in this tick: keep the pending sums, count the current state
        const double V = geo[(int64_t)kRec * i + R_V];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (touched) {
                double *a = accm + (i * G + g) * 4;
#pragma unroll
                for (int m = 0; m < 4; ++m) a[m] += av[4 * g + m];
            }
            red[g] = V * (double)Ui[4 * g];
            red[G + g] = 0.0;
        }
    } else if (owner) {
        const double V = geo[(int64_t)kRec * i + R_V];
        // the update: U - dt/V sum (global step), or U - (pending + this tick)/V
        const double dtV = BIN ? 1.0 / V : dtp[0] / V;
        if (BIN) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double *a = accm + (i * G + g) * 4;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    av[4 * g + m] += a[m];
                    a[m] = 0.0;
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double q0 = (double)Ui[4 * g + 0] - dtV * av[4 * g + 0];
            double q1 = (double)Ui[4 * g + 1] - dtV * av[4 * g + 1];
            double q2 = (double)Ui[4 * g + 2] - dtV * av[4 * g + 2];
            double q3 = (double)Ui[4 * g + 3] - dtV * av[4 * g + 3];
            const double Epre = q0;
            if (Uung) {
                float *u = Uung + i * NQ + 4 * g;
                u[0] = (float)q0;
                u[1] = (float)q1;
                u[2] = (float)q2;
                u[3] = (float)q3;
            }
            int f = 0;
            if (q0 < 0.0) {
                q0 = q1 = q2 = q3 = 0.0;
                f = 1;
            } else if (q0 == 0.0) {
                q1 = q2 = q3 = 0.0;
            } else {
                const double F2 = q1 * q1 + q2 * q2 + q3 * q3, lim = c * q0;
                if (F2 > lim * lim) {
                    const double sc = lim * rsq64(F2);
                    q1 *= sc;
                    q2 *= sc;
                    q3 *= sc;
                    f = 2;
                }
            }
            gE += f & 1;
            gF += f >> 1;
            float *o = Uout + i * NQ + 4 * g;
            const float o0 = (float)q0, o1 = (float)q1, o2 = (float)q2, o3 = (float)q3;
            o[0] = o0;
            o[1] = o1;
            o[2] = o2;
            o[3] = o3;
            // the unguarded state in its stored precision (NaN stays NaN
            // through the guard; a state beyond the FP32 range rounds to inf)
            chk = __builtin_fmaf((float)Epre, 0.0f, chk);
            chk = __builtin_fmaf(o1, 0.0f, chk);
            chk = __builtin_fmaf(o2, 0.0f, chk);
            chk = __builtin_fmaf(o3, 0.0f, chk);
            red[g] = V * (double)o0;
            red[G + g] = (f & 1) ? -Epre * V : 0.0;
        }
    } else {
#pragma unroll
        for (int p = 0; p < 2 * G; ++p) red[p] = 0.0;
    }
    if (chk != chk) atomicOr(status, ST_NONFINITE);
    if (partials) {
        const int ln = threadIdx.x & 63;
#pragma unroll
        for (int p = 0; p < 2 * G; ++p) {
            double x = wave_sum(red[p]);
            if (ln == 0) smem[wv * 2 * G + p] = x;
        }
        __syncthreads();
        if (threadIdx.x < 2 * G) {
            double s = 0.0;
            for (int u = 0; u < kBlock / 64; ++u) s += smem[u * 2 * G + threadIdx.x];
            partials[blk * 2 * G + threadIdx.x] = s;
        }
    }
    if (counts) {
        int64_t v0 = wave_sum_i64(cE), v1 = wave_sum_i64(cF), v2 = wave_sum_i64(gE),
                v3 = wave_sum_i64(gF);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&scnt[0], (unsigned long long)v0);
            atomicAdd(&scnt[1], (unsigned long long)v1);
            atomicAdd(&scnt[2], (unsigned long long)v2);
            atomicAdd(&scnt[3], (unsigned long long)v3);
        }
        __syncthreads();
        if (threadIdx.x < 4 && scnt[threadIdx.x]) atomicAdd(&counts[threadIdx.x], scnt[threadIdx.x]);
    }
}

// FP32C transport with the pairs inside a tile evaluated once (GLF or HLL,
// Hopkins surfaces, one global step, up to 3 groups): the tile scheme of the FP64
// transport (k_transport64_tile, the same task lists) with the FP32 pair
// arithmetic of k_transport32.  The lane that evaluates an in-tile pair adds
// Phi_kl to its own compensated sums and -Phi_kl, in FP64 by an LDS atomic
// add, to the partner's row of its wave's copy of the tile accumulator; after
// a block barrier each particle's FP64 sum is its own (compensated, combined
// by the butterfly) plus the 4 waves' rows in a fixed order.  Each stage's
// rows are in flight across the previous stage's evaluation, as in the
// two-sided kernel.
// BIN: one tick of the individual-time-step scheme on the tiles, as in the
// FP64 tile kernel (due pairs weighted by dt 2^min(b_k, b_l) in the
// compensated sums, pending sums accm in FP64).  IVA: the Ivanova surfaces
// as in k_transport32, each neighbour's kernel-gradient sum read from ivan.
template <int G, bool HLL, bool BIN, bool IVA>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(RT_TRANSPORT32_WAVES))) void
k_transport32_tile(int64_t n, int64_t nb, const float *__restrict__ geo32,
                   const double *__restrict__ geo, const int32_t *__restrict__ task,
                   const int64_t *__restrict__ wave_base, const int32_t *__restrict__ n_task,
                   const float *__restrict__ UD, const double *__restrict__ dtp, double c,
                   double box, float *__restrict__ Uout, double *__restrict__ partials,
                   unsigned long long *__restrict__ counts, float *__restrict__ Uung,
                   int32_t *__restrict__ status, const float2 *__restrict__ hll,
                   int64_t tick = 0, double *__restrict__ accm = nullptr,
                   const uint8_t *__restrict__ binm = nullptr,
                   const double *__restrict__ ivan = nullptr) {
    constexpr int NQ = 4 * G, MS = NQ + 1;      // accumulator row, padded against bank conflicts
    static_assert(kTile == 64 && kBlock == 256, "a block of 4 waves x 16 particles per tile");
    __shared__ float stage[kBlock / 64][64 * kStage32];
    __shared__ double mir[kBlock / 64][kTile * MS];
    constexpr int DS = 3 * NQ + 1;              // own-gradient row, padded
    __shared__ float dsh[kBlock / 64][16 * DS];
    __shared__ double smem[(kBlock / 64) * 2 * G];
    __shared__ unsigned long long scnt[4];
    const int64_t blk = xcd_block(nb);
    if (blk >= nb) return;                      // whole block: no barrier is skipped
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
    const float cf = (float)c, c2 = (float)(c * c), ic2 = (float)(1.0 / (c * c)), hc = 0.5f * cf;
    if (threadIdx.x < 4) scnt[threadIdx.x] = 0;
    float *sb = stage[wv];
    double *mw = mir[wv];                       // this wave's copy of the accumulator
    for (int e = lane; e < kTile * MS; e += 64) mw[e] = 0.0;
    wave_lds_sync32();

    const float *rk = geo32 + (int64_t)F_REC * ic;
    const double *xk = reinterpret_cast<const double *>(rk);
    const double pkx = xk[0], pky = xk[1], pkz = xk[2];
    const float iHk = rk[F_IH], hk = rk[F_H];
    float gk[3] = {0.0f, 0.0f, 0.0f};   // IVA: own kernel-gradient sum
    if constexpr (IVA) {
        gk[0] = (float)ivan[4 * ic];
        gk[1] = (float)ivan[4 * ic + 1];
        gk[2] = (float)ivan[4 * ic + 2];
    }
    float Bk[6];
#pragma unroll
    for (int a = 0; a < 6; ++a) Bk[a] = rk[F_B + a];
    float Ui[NQ];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const float *r = UD + (ic * G + g) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m) Ui[4 * g + m] = r[m];
    }
    // the own gradients live in LDS (the 4 lanes of a particle read one
    // address; in registers they left 36 bytes a lane spilled); lane sub
    // copies component sub's
    float *Dsh = dsh[wv] + (lane >> 2) * DS;
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            Dsh[3 * (4 * g + sub) + a] = UD[(ic * G + g) * 16 + 4 + 3 * sub + a];
    wave_lds_sync32();
    Kahan acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q].s = acc[q].c = 0.0f;
    int cE = 0, cF = 0;
    // BIN: this particle ends a step in this tick (ends), or some pair of its
    // neighbourhood is due (touched)
    const int64_t t1 = tick + 1;
    int32_t bk = 0;
    bool ends = true, touched = true;
    if constexpr (BIN) {
        bk = (int32_t)geo[(int64_t)kRec * ic + 12];
        const int32_t bm = binm ? (int32_t)binm[ic] : 0;
        ends = (t1 & ((int64_t(1) << bk) - 1)) == 0;
        touched = (t1 & ((int64_t(1) << bm) - 1)) == 0;
    }
    if (wave_live) {
        const int64_t base = wave_base[blk] + pl;   // the particle's column in the table
        const int32_t nn = (active && touched) ? n_task[i] : 0;
        int32_t kmax = nn;                          // the longest list of the wave
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
        // rows in flight as in k_transport32; the task of the next iteration
        // is loaded one iteration ahead
        int32_t tc = sub < nn ? task[base + 64 * (int64_t)sub] : (int32_t)ic;
        int64_t row[4];
        float4 v[4];
        {
            const int32_t j = tc & 0x7fffffff;
#pragma unroll
            for (int m = 0; m < 4; ++m) row[m] = __shfl(j, 16 * m + (lane >> 2), 64);
            load_rows32(geo32, row, lane, v);
        }
        for (int32_t kk = 0; kk < kmax; kk += 4) {
            const int32_t k = kk + sub;
            const bool valid = k < nn;
            const int32_t t = tc;
            // (slot 0 of the tile's table exists once kmax > 0: no branch
            // around the load, whose wait would then be a full one)
            const int32_t tl = task[base + 64 * (int64_t)(k + 4 < nn ? k + 4 : 0)];
            const int32_t tn = k + 4 < nn ? tl : (int32_t)ic;
            const bool mirror = t < 0;
            const int32_t j = t & 0x7fffffff;
            const int mr = mirror ? (j - (int32_t)t0) * MS : 0;   // the partner's row
            store_rows32(v, sb, lane);          // the geometry rows
            {
                int64_t rowg[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) rowg[m] = row[m] * G;
                load_rows32(UD, rowg, lane, v);
            }
            const float *rl = sb + lane * kStage32;
            // separation in FP64 from FP64 positions, rounded once
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
            const float sx = (float)min_image(xl[0] - pkx, box, ibox);
            const float sy = (float)min_image(xl[1] - pky, box, ibox);
            const float sz = (float)min_image(xl[2] - pkz, box, ibox);
            const float r = sqrt32(sx * sx + sy * sy + sz * sz);
            float Ax, Ay, Az;
            if constexpr (IVA) {
                const double *gd = ivan + 4 * (int64_t)j;
                const float gl[3] = {(float)gd[0], (float)gd[1], (float)gd[2]};
                ivanova_surface32(sx, sy, sz, r, iHk, rk[F_V], gk, rl[F_IH], rl[F_V], gl, Ax, Ay,
                                  Az);
            } else {
                const float wk = kern_wf(r * iHk);
                const float wl = kern_wf(r * rl[F_IH]);
                const float m00 = wk * Bk[0] + wl * rl[F_B + 0];
                const float m01 = wk * Bk[1] + wl * rl[F_B + 1];
                const float m02 = wk * Bk[2] + wl * rl[F_B + 2];
                const float m11 = wk * Bk[3] + wl * rl[F_B + 3];
                const float m12 = wk * Bk[4] + wl * rl[F_B + 4];
                const float m22 = wk * Bk[5] + wl * rl[F_B + 5];
                Ax = m00 * sx + m01 * sy + m02 * sz;
                Ay = m01 * sx + m11 * sy + m12 * sz;
                Az = m02 * sx + m12 * sy + m22 * sz;
            }
            const float An = sqrt32(Ax * Ax + Ay * Ay + Az * Az);
            const float hl = rl[F_H];
            const float ih = rcp32(hk + hl);
            const float fk = hk * ih, fl = hl * ih;
            bool use = valid && An > 0.0f;
            float wkl = 1.0f;                       // BIN: time integration of the exchange
            if constexpr (BIN) {
                const int32_t bl = (int32_t)rl[F_BIN];
                const int32_t bmin = bk < bl ? bk : bl;
                use = use && (t1 & ((int64_t(1) << bmin) - 1)) == 0;
                wkl = (float)ldexp(dtp[0], bmin);
            }
            const float iAn = (HLL && An > 0.0f) ? rcp32(An) : 0.0f;
            const int cnt2 = mirror ? 2 : 1;
#pragma unroll
            for (int g = 0; g < G; ++g) {
                // the stages in program order: each one's loads stay in
                // flight across the evaluation of the previous one
                __builtin_amdgcn_sched_barrier(0);
                store_rows32(v, sb, lane);      // group g's record rows
                if (g + 1 < G) {
                    int64_t rowg[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) rowg[m] = row[m] * G + g + 1;
                    load_rows32(UD, rowg, lane, v);
                } else {                        // the next iteration's geometry rows
                    const int32_t jn = tn & 0x7fffffff;
#pragma unroll
                    for (int m = 0; m < 4; ++m) row[m] = __shfl(jn, 16 * m + (lane >> 2), 64);
                    load_rows32(geo32, row, lane, v);
                }
                const float *Rl = sb + lane * kStage32;
                float qL[4], qR[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int q = 4 * g + m;
                    const float dk = Dsh[3 * q] * sx + Dsh[3 * q + 1] * sy + Dsh[3 * q + 2] * sz;
                    const float dl = Rl[4 + 3 * m] * sx + Rl[5 + 3 * m] * sy + Rl[6 + 3 * m] * sz;
                    const float mm = minmod32(dk, dl);
                    qL[m] = Ui[q] + fk * mm;
                    qR[m] = Rl[m] - fl * mm;
                }
                const int f1 = guard32(qL[0], qL[1], qL[2], qL[3], cf);
                const int f2 = guard32(qR[0], qR[1], qR[2], qR[3], cf);
                float w1 = 0.5f, w2 = 0.5f, w3 = -hc * An;   // GLF
                if constexpr (HLL) {
                    float loL, hiL, loR, hiR;
                    hll_speeds32(qL[0], qL[1], qL[2], qL[3], Ax, Ay, Az, iAn, cf, ic2, hll, loL,
                                 hiL);
                    hll_speeds32(qR[0], qR[1], qR[2], qR[3], Ax, Ay, Az, iAn, cf, ic2, hll, loR,
                                 hiR);
                    hll_weights32(loL, hiL, loR, hiR, An, w1, w2, w3);
                }
                float FL[4], FR[4];
                m1_flux32(qL[0], qL[1], qL[2], qL[3], Ax, Ay, Az, c2, ic2, FL);
                m1_flux32(qR[0], qR[1], qR[2], qR[3], Ax, Ay, Az, c2, ic2, FR);
                if (use) {
                    cE += cnt2 * ((f1 & 1) + (f2 & 1));
                    cF += cnt2 * ((f1 >> 1) + (f2 >> 1));
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const float phi = BIN ? wkl * (w1 * FL[m] + w2 * FR[m] + w3 * (qR[m] - qL[m]))
                                              : w1 * FL[m] + w2 * FR[m] + w3 * (qR[m] - qL[m]);
                        acc[4 * g + m].add(phi);
                        if (mirror) atomicAdd(mw + mr + 4 * g + m, -(double)phi);
                    }
                }
            }
            tc = tn;
            __builtin_amdgcn_sched_barrier(0);
        }
    }
    double av[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        av[q] = acc[q].value();
        quad_sum<4>(av[q]);
    }
    // every wave's deposits are in its copy of the accumulator
    __syncthreads();
    double red[2 * G];
    int gE = 0, gF = 0;
    float chk = 0.0f;   // NaN iff an updated state is NaN or infinite
    if (BIN && owner && !ends) {
        // no update in this tick: keep the pending sums, count the current state
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int v = 0; v < kBlock / 64; ++v) av[q] += mir[v][pl * MS + q];
        const double V = geo[(int64_t)kRec * i + R_V];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (touched) {
                double *a = accm + (i * G + g) * 4;
#pragma unroll
                for (int m = 0; m < 4; ++m) a[m] += av[4 * g + m];
            }
            red[g] = V * (double)Ui[4 * g];
            red[G + g] = 0.0;
        }
    } else if (owner) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int v = 0; v < kBlock / 64; ++v) av[q] += mir[v][pl * MS + q];
        const double V = geo[(int64_t)kRec * i + R_V];
        // the update: U - dt/V sum (global step), or U - (pending + this tick)/V
        const double dtV = BIN ? 1.0 / V : dtp[0] / V;
        if constexpr (BIN) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double *a = accm + (i * G + g) * 4;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    av[4 * g + m] += a[m];
                    a[m] = 0.0;
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double q0 = (double)Ui[4 * g + 0] - dtV * av[4 * g + 0];
            double q1 = (double)Ui[4 * g + 1] - dtV * av[4 * g + 1];
            double q2 = (double)Ui[4 * g + 2] - dtV * av[4 * g + 2];
            double q3 = (double)Ui[4 * g + 3] - dtV * av[4 * g + 3];
            const double Epre = q0;
            if (Uung) {
                float *u = Uung + i * NQ + 4 * g;
                u[0] = (float)q0;
                u[1] = (float)q1;
                u[2] = (float)q2;
                u[3] = (float)q3;
            }
            int f = 0;
            if (q0 < 0.0) {
                q0 = q1 = q2 = q3 = 0.0;
                f = 1;
            } else if (q0 == 0.0) {
                q1 = q2 = q3 = 0.0;
            } else {
                const double F2 = q1 * q1 + q2 * q2 + q3 * q3, lim = c * q0;
                if (F2 > lim * lim) {
                    const double sc = lim * rsq64(F2);
                    q1 *= sc;
                    q2 *= sc;
                    q3 *= sc;
                    f = 2;
                }
            }
            gE += f & 1;
            gF += f >> 1;
            float *o = Uout + i * NQ + 4 * g;
            const float o0 = (float)q0, o1 = (float)q1, o2 = (float)q2, o3 = (float)q3;
            o[0] = o0;
            o[1] = o1;
            o[2] = o2;
            o[3] = o3;
            chk = __builtin_fmaf((float)Epre, 0.0f, chk);
            chk = __builtin_fmaf(o1, 0.0f, chk);
            chk = __builtin_fmaf(o2, 0.0f, chk);
            chk = __builtin_fmaf(o3, 0.0f, chk);
            red[g] = V * (double)o0;
            red[G + g] = (f & 1) ? -Epre * V : 0.0;
        }
    } else {
#pragma unroll
        for (int p = 0; p < 2 * G; ++p) red[p] = 0.0;
    }
    if (chk != chk) atomicOr(status, ST_NONFINITE);
    if (partials) {
        const int ln = threadIdx.x & 63;
#pragma unroll
        for (int p = 0; p < 2 * G; ++p) {
            double x = wave_sum(red[p]);
            if (ln == 0) smem[wv * 2 * G + p] = x;
        }
        __syncthreads();
        if (threadIdx.x < 2 * G) {
            double s = 0.0;
            for (int u = 0; u < kBlock / 64; ++u) s += smem[u * 2 * G + threadIdx.x];
            partials[blk * 2 * G + threadIdx.x] = s;
        }
    }
    if (counts) {
        int64_t v0 = wave_sum_i64(cE), v1 = wave_sum_i64(cF), v2 = wave_sum_i64(gE),
                v3 = wave_sum_i64(gF);
        __syncthreads();
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&scnt[0], (unsigned long long)v0);
            atomicAdd(&scnt[1], (unsigned long long)v1);
            atomicAdd(&scnt[2], (unsigned long long)v2);
            atomicAdd(&scnt[3], (unsigned long long)v3);
        }
        __syncthreads();
        if (threadIdx.x < 4 && scnt[threadIdx.x]) atomicAdd(&counts[threadIdx.x], scnt[threadIdx.x]);
    }
}

// Lanes per particle of the FP32 gradient (1, 2 or 4).  With 4 the
// compensated-FP32 adjoint of the 1000-particle adjoint case moved away from
// the FP64 one (luminosity gradients 1.4e-5 apart instead of 3e-8): the
// four-lane order of the FP32 sums decides a minmod tie of the next transport
// (one pair whose two slopes agree to 2.5e-7 in FP64) the other way, and the
// adjoint differentiates through the branch taken.  Either order is as
// accurate as the other; the one-lane order is kept since it leaves that case
// on the FP64 branch.
#ifndef RT_GRADIENT32_Q
#define RT_GRADIENT32_Q 1
#endif
constexpr int kGQ32 = RT_GRADIENT32_Q;

template <int G>
void launch_gradient32(rt_ctx *ctx, const float *U, float *UD) {
    if constexpr (union_cap32(G) > 0 && kGQ32 == 1) {   // the union sums in one lane's order
        if (ctx->uoff) {
            // blocks whose union fits: from LDS; the others: one lane per
            // particle (the same order), by list
            const int64_t nw = ctx->nwaves;
            k_gradient32u<G><<<(unsigned)xcd_grid(nw), kBlock, 0, ctx->stream>>>(
                ctx->p.n, nw, ctx->geo32, ctx->xs, ctx->urow, ctx->uoff, ctx->gloc, ctx->goff,
                ctx->uown, ctx->n_gath, U, UD, ctx->status, ctx->p.box);
            if (ctx->n_ublk > 0) {
                const int64_t nl = (ctx->n_ublk + 3) / 4;
                k_gradient32<G, 1><<<(unsigned)xcd_grid(nl), kBlock, 0, ctx->stream>>>(
                    ctx->p.n, nl, ctx->geo32, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath, U,
                    UD, ctx->status, ctx->p.box, 0, ctx->ublk, ctx->n_ublk);
            }
            return;
        }
    }
    const int64_t n = ctx->p.n, nb = (n + kBlock / kGQ32 - 1) / (kBlock / kGQ32);
    k_gradient32<G, kGQ32><<<(unsigned)xcd_grid(nb), kBlock, 0, ctx->stream>>>(
        n, nb, ctx->geo32, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath, U, UD, ctx->status,
        ctx->p.box);
}

// Lanes per particle of the FP32C transport (1, 2 or 4).  On the 3-group
// 128^3 lattice Q = 4 ran GLF 6% and HLL 5% faster than Q = 1.
#ifndef RT_TRANSPORT32_Q
#define RT_TRANSPORT32_Q 4
#endif
constexpr int kQ32 = RT_TRANSPORT32_Q;

template <int G>
void launch_transport32(rt_ctx *ctx, const float *UD, const double *dt, float *Uout,
                        double *partials, int64_t *counts, float *Uung) {
    const int64_t n = ctx->p.n, nb = rt_transport32_rows(n);
    const float2 *tab = (const float2 *)ctx->hll_table32;
    const bool iva = ctx->surfaces == RT_IVANOVA;
    if constexpr (G <= 3) {
        const bool hll = ctx->solver == RT_HLL;
        if (RT_TRANSPORT32_TILE != 0 && (ctx->solver == RT_GLF || (RT_TRANSPORT32_TILE_HLL != 0 && hll)) &&
            (!iva || RT_TRANSPORT32_TILE_IVA != 0) && ctx->task) {
            // pair-once tiles: one block of 64 particles per tile, as many
            // blocks (and rows of partials) as the two-sided kernel
            static_assert(kBlock / kQ32 == kTile, "a tile per two-sided block");
#define RT_TILE32_LAUNCH(HLL_, IVA_)                                                            \
    k_transport32_tile<G, HLL_, false, IVA_><<<(unsigned)xcd_grid(nb), kBlock, 0, ctx->stream>>>( \
        n, nb, ctx->geo32, ctx->geo, ctx->task, ctx->wave_base, ctx->n_task, UD, dt,            \
        ctx->p.c_red, ctx->p.box, Uout, partials, (unsigned long long *)counts, Uung,           \
        ctx->status, tab, 0, nullptr, nullptr, ctx->ivan)
            if (hll) {
                if (iva) RT_TILE32_LAUNCH(true, true);
                else RT_TILE32_LAUNCH(true, false);
            } else {
                if (iva) RT_TILE32_LAUNCH(false, true);
                else RT_TILE32_LAUNCH(false, false);
            }
#undef RT_TILE32_LAUNCH
            return;
        }
    }
#define RT_TRANSPORT32_LAUNCH(HLL_, IVA_)                                                     \
    k_transport32<G, HLL_, kQ32, IVA_><<<(unsigned)xcd_grid(nb), kBlock, 0, ctx->stream>>>(   \
        n, nb, ctx->geo32, ctx->geo, ctx->nbr, ctx->wave_base, ctx->n_nbr, UD, dt,            \
        ctx->p.c_red, ctx->p.box, Uout, partials, (unsigned long long *)counts, Uung,         \
        ctx->status, tab, ctx->ivan)
    if (ctx->solver == RT_HLL) {
        if (iva) RT_TRANSPORT32_LAUNCH(true, true);
        else RT_TRANSPORT32_LAUNCH(true, false);
    } else {
        if (iva) RT_TRANSPORT32_LAUNCH(false, true);
        else RT_TRANSPORT32_LAUNCH(false, false);
    }
#undef RT_TRANSPORT32_LAUNCH
}

template <int G>
void launch_tick32(rt_ctx *ctx, float *U, float *UD, const double *dt, double *partials,
                   int64_t *counts, int64_t tick, double *accm) {
    const int64_t n = ctx->p.n;
    const int64_t ng = (n + kBlock / kGQ32 - 1) / (kBlock / kGQ32);
    bool grad_done = false;
    if constexpr (union_cap32(G) > 0 && kGQ32 == 1) {
        if (RT_TICK_UNION32 != 0 && ctx->uoff) {
            // the neighbour unions in their time-bin mode; the blocks whose
            // union does not fit: one lane per particle, by list
            const int64_t nw = ctx->nwaves;
            k_gradient32u<G, true><<<(unsigned)xcd_grid(nw), kBlock, 0, ctx->stream>>>(
                n, nw, ctx->geo32, ctx->xs, ctx->urow, ctx->uoff, ctx->gloc, ctx->goff,
                ctx->uown, ctx->n_gath, U, UD, ctx->status, ctx->p.box, tick);
            if (ctx->n_ublk > 0) {
                const int64_t nl = (ctx->n_ublk + 3) / 4;
                k_gradient32<G, 1, true><<<(unsigned)xcd_grid(nl), kBlock, 0, ctx->stream>>>(
                    n, nl, ctx->geo32, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath, U, UD,
                    ctx->status, ctx->p.box, tick, ctx->ublk, ctx->n_ublk);
            }
            grad_done = true;
        }
    }
    if (!grad_done)
        k_gradient32<G, kGQ32, true><<<(unsigned)xcd_grid(ng), kBlock, 0, ctx->stream>>>(
            n, ng, ctx->geo32, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath, U, UD, ctx->status,
            ctx->p.box, tick);
    const int64_t nb = rt_transport32_rows(n);
    const float2 *tab = (const float2 *)ctx->hll_table32;
    const bool iva = ctx->surfaces == RT_IVANOVA;
    const uint8_t *binm = ctx->bin8 ? ctx->bin8 + n : nullptr;
    if constexpr (G <= 3) {
        const bool hll = ctx->solver == RT_HLL;
        if (RT_TICK32_TILE != 0 && RT_TRANSPORT32_TILE != 0 &&
            (ctx->solver == RT_GLF || (RT_TRANSPORT32_TILE_HLL != 0 && hll)) &&
            (!iva || RT_TRANSPORT32_TILE_IVA != 0) && ctx->task) {
            // the tiles in their time-bin mode (one row of partials per tile)
            static_assert(kBlock / kQ32 == kTile, "a tile per two-sided block");
#define RT_TICK32_TILE_LAUNCH(HLL_, IVA_)                                                       \
    k_transport32_tile<G, HLL_, true, IVA_><<<(unsigned)xcd_grid(nb), kBlock, 0, ctx->stream>>>( \
        n, nb, ctx->geo32, ctx->geo, ctx->task, ctx->wave_base, ctx->n_task, UD, dt,            \
        ctx->p.c_red, ctx->p.box, U, partials, (unsigned long long *)counts, nullptr,           \
        ctx->status, tab, tick, accm, binm, ctx->ivan)
            if (hll) {
                if (iva) RT_TICK32_TILE_LAUNCH(true, true);
                else RT_TICK32_TILE_LAUNCH(true, false);
            } else {
                if (iva) RT_TICK32_TILE_LAUNCH(false, true);
                else RT_TICK32_TILE_LAUNCH(false, false);
            }
#undef RT_TICK32_TILE_LAUNCH
            return;
        }
    }
#define RT_TICK32_LAUNCH(HLL_, IVA_)                                                           \
    k_transport32<G, HLL_, kQ32, IVA_, true><<<(unsigned)xcd_grid(nb), kBlock, 0, ctx->stream>>>( \
        n, nb, ctx->geo32, ctx->geo, ctx->nbr, ctx->wave_base, ctx->n_nbr, UD, dt,             \
        ctx->p.c_red, ctx->p.box, U, partials, (unsigned long long *)counts, nullptr,          \
        ctx->status, tab, ctx->ivan, tick, accm, binm)
    if (ctx->solver == RT_HLL) {
        if (iva) RT_TICK32_LAUNCH(true, true);
        else RT_TICK32_LAUNCH(true, false);
    } else {
        if (iva) RT_TICK32_LAUNCH(false, true);
        else RT_TICK32_LAUNCH(false, false);
    }
#undef RT_TICK32_LAUNCH
}

}  // namespace

void rt_gradient32(rt_ctx *ctx, const float *U, float *UD) {
    switch (ctx->p.groups) {
        case 1: launch_gradient32<1>(ctx, U, UD); break;
        case 2: launch_gradient32<2>(ctx, U, UD); break;
        case 3: launch_gradient32<3>(ctx, U, UD); break;
        case 4: launch_gradient32<4>(ctx, U, UD); break;
        case 5: launch_gradient32<5>(ctx, U, UD); break;
        case 6: launch_gradient32<6>(ctx, U, UD); break;
        case 7: launch_gradient32<7>(ctx, U, UD); break;
        case 8: launch_gradient32<8>(ctx, U, UD); break;
        default: break;
    }
}

int64_t rt_transport32_rows(int64_t n) { return (n + kBlock / kQ32 - 1) / (kBlock / kQ32); }

void rt_transport32(rt_ctx *ctx, const float *UD, const double *dt, float *Uout,
                    double *partials, int64_t *counts, float *Uung) {
    switch (ctx->p.groups) {
        case 1: launch_transport32<1>(ctx, UD, dt, Uout, partials, counts, Uung); break;
        case 2: launch_transport32<2>(ctx, UD, dt, Uout, partials, counts, Uung); break;
        case 3: launch_transport32<3>(ctx, UD, dt, Uout, partials, counts, Uung); break;
        case 4: launch_transport32<4>(ctx, UD, dt, Uout, partials, counts, Uung); break;
        case 5: launch_transport32<5>(ctx, UD, dt, Uout, partials, counts, Uung); break;
        case 6: launch_transport32<6>(ctx, UD, dt, Uout, partials, counts, Uung); break;
        case 7: launch_transport32<7>(ctx, UD, dt, Uout, partials, counts, Uung); break;
        case 8: launch_transport32<8>(ctx, UD, dt, Uout, partials, counts, Uung); break;
        default: break;
    }
}

rt_status rt_tick_step32_impl(rt_ctx *ctx, float *U, float *UD, const double *dt, int64_t tick,
                              double *accm, double *Q, int64_t *counts, double *ledger) {
    const int64_t nb = rt_transport32_rows(ctx->p.n);
    double *part = (Q || ledger) ? ctx->partials : nullptr;
    rt_timer_begin(ctx, "tick");
    switch (ctx->p.groups) {
        case 1: launch_tick32<1>(ctx, U, UD, dt, part, counts, tick, accm); break;
        case 2: launch_tick32<2>(ctx, U, UD, dt, part, counts, tick, accm); break;
        case 3: launch_tick32<3>(ctx, U, UD, dt, part, counts, tick, accm); break;
        case 4: launch_tick32<4>(ctx, U, UD, dt, part, counts, tick, accm); break;
        case 5: launch_tick32<5>(ctx, U, UD, dt, part, counts, tick, accm); break;
        case 6: launch_tick32<6>(ctx, U, UD, dt, part, counts, tick, accm); break;
        case 7: launch_tick32<7>(ctx, U, UD, dt, part, counts, tick, accm); break;
        case 8: launch_tick32<8>(ctx, U, UD, dt, part, counts, tick, accm); break;
        default: break;
    }
    rt_timer_end(ctx, "tick");
    RT_HIP(hipGetLastError());
    if (part) rt_finalize_partials(ctx, nb, Q, ledger);
    return RT_OK;
}
