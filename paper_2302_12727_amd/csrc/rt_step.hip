// Per-step kernels of the photon transport (Part III "One RT time step"):
// injection, least-squares gradients, the pair transport loop with its fused
// update, and the photon budget.
//
// Every kernel is a gather over the wave-sliced neighbour table: lane i owns
// particle i (Morton order), reads slot j of its list at
// wave_base[i/64] + 64 j + i%64 (coalesced), and accumulates in registers, so
// results are deterministic and no atomics touch floating-point state.
#include "rt_pair.h"

using namespace gearrt;

namespace {

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

// FP64 transport with the GLF solver: the particle's own state and gradients
// in LDS instead of registers (OWN), which frees the registers to hold the
// next stage's neighbour lines in flight while the current stage is computed
// (PIPE).  The HLL instantiations keep both off: they run 3 waves per SIMD
// at 168 registers, which the in-flight lines would not fit.
#ifndef RT_TRANSPORT_OWN_LDS
#define RT_TRANSPORT_OWN_LDS 1
#endif
#ifndef RT_TRANSPORT_PIPE
#define RT_TRANSPORT_PIPE 1
#endif
constexpr bool kOwnL = RT_TRANSPORT_OWN_LDS != 0;
constexpr bool kPipe = RT_TRANSPORT_PIPE != 0;
// GLF with the Hopkins surfaces keeps its own state and gradients in
// registers and loads each stage just before it (256 VGPRs, 5 spilled): since
// the inner loop was trimmed to 731 VALU instructions per slot, this form
// saves the 24 KB of LDS reads of the own state per wave-iteration and ran
// 4% faster than the LDS-resident pipelined one (4.10 against 4.27-4.29 ms
// on the 3-group 128^3 lattice, same box).  The Ivanova and HLL forms keep
// the LDS-resident own state (their register forms spill more).
#ifndef RT_TRANSPORT_GLF_REGS
#define RT_TRANSPORT_GLF_REGS 1
#endif
constexpr bool own_lds(bool hll, bool iva, int w) {
    return (hll || iva) ? (kOwnL && (!hll || w > 1)) : (kOwnL && RT_TRANSPORT_GLF_REGS == 0);
}
constexpr bool pipe_on(bool hll, bool iva, int w) {
    return (hll || iva) ? (kPipe && (!hll || w > 1)) : (kPipe && RT_TRANSPORT_GLF_REGS == 0);
}

// ---------------------------------------------------------------------------
// Injection: E_g += dt sum_s xi_sg L_s / V_g, one thread per receiving particle.
template <typename T>
__global__ void k_inject(int32_t ngas, int G, const int32_t *__restrict__ gptr,
                         const int32_t *__restrict__ gas, const int32_t *__restrict__ src,
                         const double *__restrict__ coef, const double *__restrict__ L,
                         const double *__restrict__ dtp, T *__restrict__ U) {
    int32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ngas) return;
    const int64_t g = gas[t];
    const double dt = dtp[0];
    for (int grp = 0; grp < G; ++grp) {
        double s = 0.0;
        for (int32_t e = gptr[t]; e < gptr[t + 1]; ++e) s += coef[e] * L[(int64_t)src[e] * G + grp];
        T *E = U + (g * G + grp) * 4;
        E[0] = (T)((double)E[0] + dt * s);
    }
}

// two doubles as one 16-byte access (a native vector: copies stay in registers)
typedef double dvec2 __attribute__((ext_vector_type(2)));

// Gradient record of particle i from its Q lanes' sums (every lane holds the
// combined sums acc = sum_j (q_j - q_i) w_ij s_ij and the own state Ui): the
// gradients are B_i/V_i acc; the Q lanes write consecutive 16-byte pieces of
// the record.  chk stays 0 unless a value written is NaN or infinite (0 x v is
// 0 for finite v and NaN otherwise).
template <int G, int Q>
__device__ __forceinline__ void gradient_record(double (&acc)[4 * G][3], const double (&Ui)[4 * G],
                                                const double *__restrict__ rec, double *o, int sub,
                                                int32_t *__restrict__ status) {
    constexpr int NQ = 4 * G;
    const double iV = 1.0 / rec[R_V];
    const double b00 = rec[R_B] * iV, b01 = rec[R_B + 1] * iV, b02 = rec[R_B + 2] * iV;
    const double b11 = rec[R_B + 3] * iV, b12 = rec[R_B + 4] * iV, b22 = rec[R_B + 5] * iV;
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const double d0 = b00 * acc[q][0] + b01 * acc[q][1] + b02 * acc[q][2];
        const double d1 = b01 * acc[q][0] + b11 * acc[q][1] + b12 * acc[q][2];
        const double d2 = b02 * acc[q][0] + b12 * acc[q][1] + b22 * acc[q][2];
        acc[q][0] = d0;
        acc[q][1] = d1;
        acc[q][2] = d2;
    }
    // group-major record: per group the state then its gradients (one line);
    // double d of the record, d = 16 g + s
    auto value = [&](int d) {
        const int g = d / 16, s = d % 16;
        return s < 4 ? Ui[4 * g + s] : acc[4 * g + (s - 4) / 3][(s - 4) % 3];
    };
    double chk = 0.0;
#pragma unroll
    for (int t = 0; t < 8 * G / Q; ++t) {
        double2 val = make_double2(value(2 * Q * t), value(2 * Q * t + 1));
#pragma unroll
        for (int s = 1; s < Q; ++s)
            if (sub == s) val = make_double2(value(2 * (Q * t + s)), value(2 * (Q * t + s) + 1));
        chk = __builtin_fma(val.x, 0.0, chk);
        chk = __builtin_fma(val.y, 0.0, chk);
        *reinterpret_cast<double2 *>(o + 2 * (Q * t + sub)) = val;
    }
    if (chk != chk) atomicOr(status, ST_NONFINITE);
}

// Reduce-scatter of a particle's four lanes' partial sums (4 lanes a
// particle, DPP): afterwards lane sub holds in s[g] the full sums of
// component sub of every group g, formed with the same additions in the same
// order as quad_sum, so with the same bits, while no lane holds all 12 G sums
// (the record then needs a quarter of the registers).  After the first step
// slot k of a lane with bit 0 = b0 holds q = 2k + b0, after the second slot g
// of lane sub holds q = 4g + sub.
template <int G>
__device__ __forceinline__ void quad_scatter(const double (&acc)[4 * G][3], int sub,
                                             double (&s)[G][3]) {
    const bool b0 = (sub & 1) != 0, b1 = (sub & 2) != 0;
    double t[2 * G][3];
#pragma unroll
    for (int k = 0; k < 2 * G; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double mine = b0 ? acc[2 * k + 1][a] : acc[2 * k][a];
            const double other = b0 ? acc[2 * k][a] : acc[2 * k + 1][a];
            t[k][a] = mine + quad_xor<1>(other);
        }
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double mine = b1 ? t[2 * g + 1][a] : t[2 * g][a];
            const double other = b1 ? t[2 * g][a] : t[2 * g + 1][a];
            s[g][a] = mine + quad_xor<2>(other);
        }
}

// The record from the scattered sums (gradient_record's arithmetic): lane sub
// writes component sub of every group, its state u[g] and its gradient.
template <int G>
__device__ __forceinline__ void gradient_record_part(const double (&s)[G][3], const double (&u)[G],
                                                     const double *__restrict__ rec, double *o,
                                                     int sub, int32_t *__restrict__ status) {
    const double iV = 1.0 / rec[R_V];
    const double b00 = rec[R_B] * iV, b01 = rec[R_B + 1] * iV, b02 = rec[R_B + 2] * iV;
    const double b11 = rec[R_B + 3] * iV, b12 = rec[R_B + 4] * iV, b22 = rec[R_B + 5] * iV;
    double chk = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const double d0 = b00 * s[g][0] + b01 * s[g][1] + b02 * s[g][2];
        const double d1 = b01 * s[g][0] + b11 * s[g][1] + b12 * s[g][2];
        const double d2 = b02 * s[g][0] + b12 * s[g][1] + b22 * s[g][2];
        double *og = o + 16 * g;
        og[sub] = u[g];
        og[4 + 3 * sub] = d0;
        og[5 + 3 * sub] = d1;
        og[6 + 3 * sub] = d2;
        chk = __builtin_fma(u[g], 0.0, chk);
        chk = __builtin_fma(d0, 0.0, chk);
        chk = __builtin_fma(d1, 0.0, chk);
        chk = __builtin_fma(d2, 0.0, chk);
    }
    if (chk != chk) atomicOr(status, ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// Gradient (eq:gradient):  grad q_i = sum_j (q_j - q_i) psi~_j(x_i)
//   = S_i^{-1} sum_j (q_j - q_i) w(r_ij / H_i) s_ij   (the kernel normalisation
// and V_i cancel against B_i, see the geometry record).
// BIN: only the particles that end a step in tick `tick` (time bin in slot 12
// of the geometry record) recompute their gradient record.
//
// Q lanes share a particle, each summing every Q-th gather neighbour; the
// partial sums are combined by a fixed butterfly (the same bits on every lane
// of the particle), and the Q lanes write the particle's record together.
//
// Neighbour rows are staged through LDS.  Gathered lane by lane, each of the
// 8 loads of a neighbour's state and position touches 64 different cache
// lines (1.31 ms on the 3-group 128^3 lattice, the L1 doing about one tag
// lookup a cycle).  Here the wave moves the 64 rows of an iteration with
// consecutive lanes taking consecutive pieces: 2G loads of 16 bytes for the
// neighbours' states (64 / 2G rows a load) and 3 of 8 bytes for their
// positions (x, y, z from the packed position array, 21 rows a load; the
// heads of the 128-byte geometry records would take a cache line per
// neighbour and raised the L1 misses by 60%).  The lane that stores a piece
// subtracts the same piece of the row's own particle (the wave's own rows sit
// in LDS in the same layout), so a lane reads U_j - U_i and x_j - x_i from its
// row and holds neither its own state nor its position, which keeps the
// kernel at 3 waves per SIMD without spills.  State rows lie 2G + 1 pieces of
// 16 bytes apart in LDS, an odd number, and positions are packed 3 doubles a
// row in an array of their own, so that the stores and reads of both are
// free of bank conflicts (8-byte halves of the state pieces, or positions
// inside the state rows, conflicted 2-way).  Past
// the end of its list a lane's row is its own particle's, whose differences
// are zero: the sums need no branch.  The table entry of an iteration is
// loaded two iterations ahead and its rows one.  1.20 ms on the lattice: the
// texture data path stays busy 95% of the time, half of it waiting for L1
// misses (a wave's 16 particles reach about 400 distinct neighbours, more
// than the L1 holds).  Two iterations of rows in flight at 2 waves per SIMD
// ran 1.25 ms, blocks of 8 and 12 waves 1.41 and 1.31 ms.
#ifndef RT_GRADIENT_WAVES
#define RT_GRADIENT_WAVES 3
#endif
#ifndef RT_GRADIENT_BLOCK
#define RT_GRADIENT_BLOCK 4
#endif
constexpr int gradient_waves(int G) { return G <= 3 ? RT_GRADIENT_WAVES : G == 4 ? 2 : 1; }
static_assert(RT_GRADIENT_BLOCK >= 1 && RT_GRADIENT_BLOCK <= 16, "1 to 16 waves per block");
// threads per block of the FP64 gradient: at most the waves of one CU and
// the LDS of one CU (80 staged rows of 2G + 1 pieces and 3 doubles per wave at
// 4 lanes per particle)
constexpr int grad_lds_wave(int G) { return 80 * ((2 * G + 1) * 16 + 24); }
constexpr int grad_block(int G) {
    const int by_lds = 163840 / grad_lds_wave(G);
    int w = RT_GRADIENT_BLOCK;
    if (w > 4 * gradient_waves(G)) w = 4 * gradient_waves(G);
    if (w > by_lds) w = by_lds;
    return 64 * w;
}

template <int G, bool BIN = false, int Q = 1>
__global__ __launch_bounds__(grad_block(G)) __attribute__((amdgpu_waves_per_eu(
    gradient_waves(G), gradient_waves(G)))) void k_gradient64(
    int64_t n, int64_t nb, const double *__restrict__ geo, const double *__restrict__ xs,
    const int32_t *__restrict__ nbr, const int64_t *__restrict__ wave_base,
    const int32_t *__restrict__ n_gath, const double *__restrict__ U, double *__restrict__ UD,
    int32_t *__restrict__ status, double box, int64_t tick = 0,
    const int32_t *__restrict__ blist = nullptr) {
    static_assert(Q == 1 || Q == 2 || Q == 4, "lanes per particle: 1, 2 or 4");
    constexpr int NQ = 4 * G;
    constexpr int PU = 2 * G;           // 16-byte pieces of a state
    constexpr int S = PU + 1;           // LDS row stride in pieces (odd)
    constexpr int NP = 64 / Q;          // particles of a wave
    constexpr int W = grad_block(G) / 64;
    static_assert(Q != 4 || grad_lds_wave(G) * W <= 163840, "LDS of one CU");
    __shared__ dvec2 stage[W][64 * S];
    __shared__ dvec2 own[W][NP * S];
    __shared__ double spos[W][64 * 3];
    __shared__ double opos[W][NP * 3];
    const int64_t bx = xcd_block(nb);
    if (bx >= nb) return;                       // whole block
    const int64_t blk = blist ? (int64_t)blist[bx] : bx;   // only the listed blocks
    const int lane = threadIdx.x & 63;
    const int sub = lane % Q;
    // the wave's first particle; the wave stays whole (its loads are shared)
    const int64_t i0 = blk * (grad_block(G) / Q) + (threadIdx.x >> 6) * NP;
    if (i0 >= n) return;                        // whole wave
    const int64_t i = i0 + lane / Q;
    const int64_t ic = i < n ? i : n - 1;
    const double *rec = geo + (int64_t)kRec * ic;
    const bool active =
        i < n && (!BIN || ((tick + 1) & ((int64_t(1) << (int32_t)rec[12]) - 1)) == 0);
    const int32_t ng = active ? n_gath[ic] : 0;
    int32_t kmax = ng;                          // the wave's longest list
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
    const double ibox = 1.0 / box;
    const double iH = rec[R_IH];
    double acc[NQ][3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
    dvec2 *sb = stage[threadIdx.x >> 6], *ob = own[threadIdx.x >> 6];
    double *sd = spos[threadIdx.x >> 6], *od = opos[threadIdx.x >> 6];
    const dvec2 *U2 = reinterpret_cast<const dvec2 *>(U);
    // the wave's own rows (the last particle repeated past n)
#pragma unroll
    for (int c = 0; c < (NP * PU + 63) / 64; ++c) {
        const int e = 64 * c + lane;
        if (NP * PU % 64 == 0 || e < NP * PU) {
            const uint32_t jo = (uint32_t)min(i0 + e / PU, n - 1);
            ob[(e / PU) * S + e % PU] = U2[jo * (uint32_t)PU + (uint32_t)(e % PU)];
        }
    }
#pragma unroll
    for (int c = 0; c < (NP * 3 + 63) / 64; ++c) {
        const int e = 64 * c + lane;
        if (NP * 3 % 64 == 0 || e < NP * 3) {
            const uint32_t jo = (uint32_t)min(i0 + e / 3, n - 1);
            od[e] = xs[jo * 3u + (uint32_t)(e % 3)];
        }
    }
    if (kmax > 0) {
        // Slot k of the particle's column, or slot 0 past the end of its list
        // (present: some column of this table block holds an entry); an index
        // past the end is replaced by the particle's own.
        const int32_t *col = nbr + wave_base[ic >> 6] + (ic & 63);
        auto entry = [&](int32_t k) __attribute__((always_inline)) {
            return col[64 * (k < ng ? k : 0)];
        };
        auto index = [&](int32_t k, int32_t e) __attribute__((always_inline)) {
            return k < ng ? e : (int32_t)ic;
        };
        // the rows of lane j's: state piece c of every lane is e = 64 c + lane,
        // row e / PU; position double c is e = 64 c + lane, row e / 3
        struct Rows { dvec2 u[PU]; double x[3]; };
        auto load = [&](Rows &v, int32_t j) __attribute__((always_inline)) {
#pragma unroll
            for (int c = 0; c < PU; ++c) {
                const int e = 64 * c + lane;
                const uint32_t jr = (uint32_t)__shfl(j, e / PU, 64);
                v.u[c] = U2[jr * (uint32_t)PU + (uint32_t)(e % PU)];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int e = 64 * c + lane;
                const uint32_t jr = (uint32_t)__shfl(j, e / 3, 64);
                v.x[c] = xs[jr * 3u + (uint32_t)(e % 3)];
            }
        };
        // store the pieces less the own particle's, for the lanes to read
        auto put = [&](const Rows &v) __attribute__((always_inline)) {
            wave_lds_sync();
#pragma unroll
            for (int c = 0; c < PU; ++c) {
                const int e = 64 * c + lane, r = e / PU, p = e % PU;
                sb[r * S + p] = v.u[c] - ob[(r / Q) * S + p];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const int e = 64 * c + lane;
                sd[e] = v.x[c] - od[(e / (3 * Q)) * 3 + e % 3];
            }
            wave_lds_sync();
        };
        auto gather = [&]() __attribute__((always_inline)) {
            const dvec2 *row = sb + lane * S;
            const double sx = min_image(sd[3 * lane], box, ibox);
            const double sy = min_image(sd[3 * lane + 1], box, ibox);
            const double sz = min_image(sd[3 * lane + 2], box, ibox);
            const double w = kern_w(sqrt64(sx * sx + sy * sy + sz * sz) * iH);
            const double wx = w * sx, wy = w * sy, wz = w * sz;
#pragma unroll
            for (int t = 0; t < PU; ++t) {
                const dvec2 d = row[t];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int q = 2 * t + h;
                    acc[q][0] += d[h] * wx;
                    acc[q][1] += d[h] * wy;
                    acc[q][2] += d[h] * wz;
                }
            }
        };
        // Each table entry is loaded before the rows of the iteration ahead of
        // it, so waiting for the entry never waits for rows still in flight;
        // no step is skipped near the end (rows past every list are the own
        // rows), so that every path through the loop body is alike.
        Rows v;
        const int32_t e0 = entry(sub);
        int32_t e1 = entry(Q + sub);
        load(v, index(sub, e0));
        for (int32_t kk = 0; kk < kmax; kk += Q) {
            put(v);
            const int32_t e2 = entry(kk + 2 * Q + sub);
            load(v, index(kk + Q + sub, e1));
            e1 = e2;
            gather();
        }
    }
    if constexpr (Q == 4) {
        double sg[G][3];
        quad_scatter<G>(acc, sub, sg);
        if (!active) return;
        // the own state, as loaded, from the wave's own row: component sub
        wave_lds_sync();
        double u[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const dvec2 x = ob[(lane / Q) * S + 2 * g + (sub >> 1)];
            u[g] = (sub & 1) ? x.y : x.x;
        }
        gradient_record_part<G>(sg, u, rec, UD + ic * (16 * G), sub, status);
        return;
    }
    if (Q > 1) {
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                quad_sum<Q>(acc[q][a]);
    }
    if (!active) return;
    // the own state, as loaded, from the wave's own row
    wave_lds_sync();
    double Ui[NQ];
#pragma unroll
    for (int t = 0; t < PU; ++t) {
        const dvec2 x = ob[(lane / Q) * S + t];
        Ui[2 * t] = x.x;
        Ui[2 * t + 1] = x.y;
    }
    gradient_record<G, Q>(acc, Ui, rec, UD + ic * (16 * G), sub, status);
}

// Gradient from the block's neighbour union (FP64, up to 4 groups, the global
// step).  The 64 particles of a block (a column block of the neighbour table)
// gather from about 360 (lattice) to 580 (Plummer set) distinct particles,
// each 6-8 times.  The build lists them (k_union); this kernel stages their
// states and positions in LDS once, with coalesced loads, and every pair then
// reads its neighbour's row from LDS by its 16-bit position in the union
// (gloc): the pair loop's only global loads are the table's entries, 8 bytes
// per 4 iterations.
// Blocks whose union did not fit the LDS are left to k_gradient64 (a second
// launch over their list).  Sums in the same order as k_gradient64 (lane sub
// takes the slots sub, sub + Q, ...; rows past a list are the own row, whose
// differences are zero), so the two give the same bits.
// BIN: only the particles that end a step in tick `tick` recompute their
// record, as in k_gradient64; a block none of whose particles does so stages
// nothing.
template <int G, int Q, int W, bool BIN = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(W, W))) void
k_gradient64u(int64_t n, int64_t nb, const double *__restrict__ geo, const double *__restrict__ xs,
              const int32_t *__restrict__ urow, const int64_t *__restrict__ uoff,
              const uint16_t *__restrict__ gloc, const int64_t *__restrict__ goff,
              const uint16_t *__restrict__ uown, const int32_t *__restrict__ n_gath,
              const double *__restrict__ U, double *__restrict__ UD, int32_t *__restrict__ status,
              double box, int64_t tick = 0) {
    static_assert(Q == 4 && kBlock == 256, "one block of 64 particles per table column block");
    constexpr int NQ = 4 * G, PU = 2 * G, UC = W == 3 ? union_cap3(G) : union_cap(G);
    static_assert(UC > 0 && UC <= kUnionSort, "union capacity");
    __shared__ dvec2 ust[UC * PU];
    __shared__ double upos[UC * 3];
    __shared__ int32_t uidx[UC];
    const int64_t blk = xcd_block(nb);
    if (blk >= nb) return;                      // whole block
    const int64_t u0 = uoff[blk];
    const int32_t rows = (int32_t)(uoff[blk + 1] - u0);
    if (rows == 0) return;                      // left to the staged gradient (whole block)
    if constexpr (BIN) {
        const int64_t ib = blk * (kBlock / Q) + threadIdx.x / Q;
        const bool e = ib < n &&
                       ((tick + 1) & ((int64_t(1) << (int32_t)geo[(int64_t)kRec * ib + 12]) - 1)) == 0;
        if (!__syncthreads_or(e)) return;       // whole block: no particle ends a step
    }
    // stage the union: its indices first, then every thread's pieces of the
    // states (16 bytes) and positions (doubles) in flight at once (a chain of
    // dependent loads per piece left the blocks waiting: 1.38 ms)
    for (int e = threadIdx.x; e < rows; e += kBlock) uidx[e] = urow[u0 + e];
    __syncthreads();
    const dvec2 *U2 = reinterpret_cast<const dvec2 *>(U);
    const int ts = rows * PU, tp = rows * 3;
    {
        constexpr int MS = (UC * PU + kBlock - 1) / kBlock, MP = (UC * 3 + kBlock - 1) / kBlock;
        dvec2 v[MS];
        double x[MP];
#pragma unroll
        for (int r = 0; r < MS; ++r) {
            const int e = threadIdx.x + r * kBlock;
            if (e < ts) v[r] = U2[(uint32_t)uidx[e / PU] * (uint32_t)PU + (uint32_t)(e % PU)];
        }
#pragma unroll
        for (int r = 0; r < MP; ++r) {
            const int e = threadIdx.x + r * kBlock;
            if (e < tp) x[r] = xs[(uint32_t)uidx[e / 3] * 3u + (uint32_t)(e % 3)];
        }
#pragma unroll
        for (int r = 0; r < MS; ++r)
            if (threadIdx.x + r * kBlock < ts) ust[threadIdx.x + r * kBlock] = v[r];
#pragma unroll
        for (int r = 0; r < MP; ++r)
            if (threadIdx.x + r * kBlock < tp) upos[threadIdx.x + r * kBlock] = x[r];
    }
    __syncthreads();
    const int lane = threadIdx.x & 63, sub = lane % Q;
    const int p = threadIdx.x / Q;              // the particle in the block
    const int64_t i = blk * (kBlock / Q) + p;
    const bool active =
        i < n && (!BIN || ((tick + 1) & ((int64_t(1) << (int32_t)geo[(int64_t)kRec * i + 12]) - 1)) == 0);
    const int64_t ic = active ? i : n - 1;
    const int32_t ng = active ? n_gath[ic] : 0;
    const int il = active ? (int)uown[ic] : 0;  // a row of the union (not used past n)
    int32_t kmax = ng;                          // the wave's longest list
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
    const double *rec = geo + (int64_t)kRec * ic;
    const double ibox = 1.0 / box, iH = rec[R_IH];
    double Ui[NQ];
#pragma unroll
    for (int t = 0; t < PU; ++t) {
        const dvec2 x = ust[il * PU + t];
        Ui[2 * t] = x.x;
        Ui[2 * t + 1] = x.y;
    }
    const double px = upos[3 * il], py = upos[3 * il + 1], pz = upos[3 * il + 2];
    double acc[NQ][3];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
    if (kmax > 0) {
        auto pair = [&](int jl) __attribute__((always_inline)) {
            const dvec2 *row = ust + jl * PU;
            const double sx = min_image(upos[3 * jl] - px, box, ibox);
            const double sy = min_image(upos[3 * jl + 1] - py, box, ibox);
            const double sz = min_image(upos[3 * jl + 2] - pz, box, ibox);
            const double w = kern_w(sqrt64(sx * sx + sy * sy + sz * sz) * iH);
            const double wx = w * sx, wy = w * sy, wz = w * sz;
#pragma unroll
            for (int t = 0; t < PU; ++t) {
                const dvec2 uj = row[t];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int q = 2 * t + h;
                    const double d = uj[h] - Ui[q];
                    acc[q][0] += d * wx;
                    acc[q][1] += d * wy;
                    acc[q][2] += d * wz;
                }
            }
        };
        // The lane's table entries come packed 4 iterations to an 8-byte word
        // (group gq of the block's words at gw + 256 gq), each word loaded a
        // group pair ahead into the register its own use has just freed.  Past
        // a list the row is the own one.  (One 2-byte load per iteration,
        // even two iterations ahead, left 0.11 ms of the kernel waiting.)
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
                    pair(k < ng ? (int)((wd >> (16 * u)) & 0xffff) : il);
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
    double sg[G][3];
    quad_scatter<G>(acc, sub, sg);
    if (!active) return;
    // the own state component sub of every group, from the union's row
    double u[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const dvec2 x = ust[il * PU + 2 * g + (sub >> 1)];
        u[g] = (sub & 1) ? x.y : x.x;
    }
    gradient_record_part<G>(sg, u, rec, UD + ic * (16 * G), sub, status);
}

// Transport (eq:transport-update-explicit with the GLF flux eq:riemann-GLF).
// A wave owns 64 particles and GW of the G photon groups (G/GW waves share
// the same particles): fewer groups per wave keep less state in registers
// and so more waves resident, at the price of recomputing the pair geometry
// once per group slice.
// The compiler is held to the 256 registers of 2 waves per SIMD (at 1 wave
// per SIMD the kernel runs 1.6x slower).
//
// OWNL: the particle's own state and gradients (48 doubles at 3 groups) are
// read from the block's LDS instead of being held in registers.  PIPE: with
// the registers this frees, each stage's neighbour lines are loaded one stage
// ahead (the next group's lines while a group is computed; the next
// iteration's geometry and first group lines while the last group is), so no
// stage waits for its own loads.  Measured on the 3-group 128^3 lattice: 2%
// faster with the Hopkins surfaces, 9% with the Ivanova ones (whose
// register-held form spilled).
//
// HLL: the HLL solver (eq:riemann-HLL) with the wave-speed table hll in
// place of GLF.
//
// BIN: one tick of the individual-time-step scheme (time bins in slot 12 of
// the geometry records, the smallest bin of each particle's neighbourhood in
// binm): only pairs whose smaller bin ends a step in this tick contribute,
// each with dt 2^min(b_k, b_l); the sums go to the pending flux sums accm, and
// the particles that end a step apply and clear theirs (Part III
// eq:transport-update-explicit with min{dt_k, dt_l}).
// With one group per wave the HLL instantiation fits 3 waves per SIMD (168
// registers), measured 4% faster than 2 (the GLF one is slower there).
template <int G, int GW, bool BIN = false, bool HLL = false, bool IVA = false, int Q = 1,
          bool OWNL = false, bool PIPE = false>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    (HLL && GW == 1 && !OWNL) ? 3 : 2, (HLL && GW == 1 && !OWNL) ? 3 : 2))) void k_transport64(
    int64_t n, int64_t nb, const double *__restrict__ geo, const int32_t *__restrict__ nbr,
    const int64_t *__restrict__ wave_base, const int32_t *__restrict__ n_nbr,
    const double *__restrict__ UD, const double *__restrict__ dtp, double c, double box,
    double *__restrict__ Uout, double *__restrict__ partials,
    unsigned long long *__restrict__ counts, double *__restrict__ Uung,
    int32_t *__restrict__ status, int64_t tick = 0, double *__restrict__ accm = nullptr,
    const double2 *__restrict__ hll = nullptr, const uint8_t *__restrict__ binm = nullptr) {
    static_assert(G % GW == 0, "group slices must tile the groups");
    static_assert(Q == 1 || Q == 2 || Q == 4, "lanes per particle: 1, 2 or 4");
    constexpr int NS = G / GW, NQ = 4 * G;
    constexpr int PW = 64 / Q, PB = kBlock / Q;   // particles per wave, per block
    constexpr int OS = 16 * GW + 1;               // own record in LDS (padded, doubles)
    __shared__ double stage[kBlock / 64][64 * kStage];
    __shared__ double own[OWNL ? PB * OS : 1];
    __shared__ double smem[(kBlock / 64) * 2 * GW];
    __shared__ unsigned long long scnt[4];
    const int64_t bg = xcd_block(nb * NS);
    if (bg >= nb * NS) return;                  // whole block: no barrier is skipped
    const int64_t blk = bg / NS;
    const int g0 = (int)(bg - blk * NS) * GW;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // Q lanes share a particle, each taking every Q-th of its neighbour slots
    const int sub = lane % Q;
    const int64_t i0 = blk * PB + wv * PW;      // first particle of the wave
    const int64_t i = i0 + lane / Q;
    const bool active = i < n;
    const bool owner = active && sub == 0;      // writes the particle's results
    const int64_t ic = active ? i : n - 1;      // in-range index for inactive lanes
    const int64_t w = i0 >> 6;                  // neighbour-table wave (PW divides 64)
    const bool wave_live = i0 < n;              // wave-uniform
    const double ibox = 1.0 / box, hc = 0.5 * c, c3 = 3.0 * c;
    if (threadIdx.x < 4) scnt[threadIdx.x] = 0;
    double *sb = stage[wv];

    // own particle: geometry record, state and gradients (registers, or with
    // OWNL the wave's LDS, each lane of the particle copying every Q-th value)
    const double *rk = geo + (int64_t)kRec * ic;
    double Ui[OWNL ? 1 : 4 * GW], Di[OWNL ? 1 : 12 * GW];
    double *ow = own + (OWNL ? (threadIdx.x / Q) * OS : 0);
    if constexpr (OWNL) {
#pragma unroll
        for (int e = sub; e < 16 * GW; e += Q) ow[e] = UD[(ic * G + g0 + (e >> 4)) * 16 + (e & 15)];
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
            }
        }
    }
    // q = 4 g + m: the state value, and its gradient component a
    auto ui = [&](int q) -> double {
        if constexpr (OWNL) return ow[16 * (q >> 2) + (q & 3)];
        else return Ui[q];
    };
    auto di = [&](int q, int a) -> double {
        if constexpr (OWNL) return ow[16 * (q >> 2) + 4 + 3 * (q & 3) + a];
        else return Di[3 * q + a];
    };
    double acc[4 * GW];
#pragma unroll
    for (int q = 0; q < 4 * GW; ++q) acc[q] = 0.0;
    int cE = 0, cF = 0;
    double gk[3] = {0.0, 0.0, 0.0};   // IVA: own kernel-gradient sum (record slots 13-15)
    if (IVA) {
        gk[0] = rk[13];
        gk[1] = rk[14];
        gk[2] = rk[15];
    }
    // time bins: this particle ends a step in this tick (ends), or some pair of
    // its neighbourhood does (touched); binm: the smallest bin of each
    // neighbourhood (none before rt_time_bins: every bin is 0)
    const int64_t t1 = tick + 1;
    const int32_t bk = BIN ? (int32_t)rk[12] : 0;
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
        // the neighbour index of the next iteration is loaded one iteration
        // ahead, so its latency overlaps this iteration's record loads
        int32_t jn = sub < nn ? nbr[base + 64 * (int64_t)sub] : (int32_t)ic;
        // PIPE: while a stage computes, the lines of the next group (pb), or
        // of the next iteration's geometry (pa) and first group (pb), are in
        // flight in registers
        double2 pa[PIPE ? 8 : 1], pb[PIPE ? 8 : 1];
        // pointers to this lane's pieces of the gradient-record lines of the 8
        // neighbour rows it helps to move (PIPE: the rows of the stage in
        // flight, replaced when the next iteration's are loaded)
        const double *udp[8];
        if constexpr (PIPE) {
            if (kmax > 0) {
                int32_t rn[8];
                const double *gp[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) rn[m] = __shfl(jn, 8 * m + (lane >> 3), 64);
                row_ptrs(geo, rn, 1, 0, lane, gp);
                row_ptrs(UD, rn, G, g0, lane, udp);
                load_at(gp, 0, *reinterpret_cast<double2(*)[8]>(pa));
                load_at(udp, 0, *reinterpret_cast<double2(*)[8]>(pb));
            }
        }
        for (int32_t kk = 0; kk < kmax; kk += Q) {
            const int32_t k = kk + sub;
            const bool valid = k < nn;
            const int32_t j = jn;
            jn = k + Q < nn ? nbr[base + 64 * (int64_t)(k + Q)] : (int32_t)ic;
            // pair geometry from the staged geometry records
            if constexpr (PIPE) {
                store_lines(*reinterpret_cast<double2(*)[8]>(pa), sb, lane);
            } else {
                int32_t rw[8];
                const double *gp[8];
#pragma unroll
                for (int m = 0; m < 8; ++m) rw[m] = __shfl(j, 8 * m + (lane >> 3), 64);
                row_ptrs(geo, rw, 1, 0, lane, gp);
                row_ptrs(UD, rw, G, g0, lane, udp);
                double2 v[8];
                load_at(gp, 0, v);
                store_lines(v, sb, lane);
            }
            double rl[12];
#pragma unroll
            for (int q = 0; q < 12; ++q) rl[q] = sb[lane * kStage + q];
            // the neighbour's time bin (slot 12 of its record)
            const int32_t bl = BIN ? (int32_t)sb[lane * kStage + 12] : 0;
            PairGeo pg;
            if (IVA) {
                // its kernel-gradient sum: slots 13-15 of the same record
                const double gl[3] = {sb[lane * kStage + 13], sb[lane * kStage + 14],
                                      sb[lane * kStage + 15]};
                pair_geometry_ivanova64(rk, rl, gk, gl, box, ibox, pg);
            } else {
                pair_geometry64(rk, rl, box, ibox, pg);
            }
            bool use = valid && pg.An > 0.0;
            double wkl = 1.0;                   // time integration of this exchange
            if (BIN) {
                const int32_t bmin = bk < bl ? bk : bl;
                use = use && (t1 & ((int64_t(1) << bmin) - 1)) == 0;
                wkl = ldexp(dtp[0], bmin);
            }
            const double iAn = (HLL && pg.An > 0.0) ? rcp64(pg.An) : 0.0;
#pragma unroll
            for (int g = 0; g < GW; ++g) {
                if constexpr (PIPE) {
                    double2(&vb)[8] = *reinterpret_cast<double2(*)[8]>(pb);
                    store_lines(vb, sb, lane);
                    if (g + 1 < GW) {
                        load_at(udp, g + 1, vb);
                    } else if (kk + Q < kmax) {
                        int32_t rn[8];
                        const double *gp[8];
#pragma unroll
                        for (int m = 0; m < 8; ++m) rn[m] = __shfl(jn, 8 * m + (lane >> 3), 64);
                        row_ptrs(geo, rn, 1, 0, lane, gp);
                        row_ptrs(UD, rn, G, g0, lane, udp);
                        load_at(gp, 0, *reinterpret_cast<double2(*)[8]>(pa));
                        load_at(udp, 0, vb);
                    }
                } else {
                    double2 v[8];
                    load_at(udp, g, v);
                    store_lines(v, sb, lane);
                }
                const double *Rl = sb + lane * kStage;
                double qL[4], qR[4];
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const int q = 4 * g + m;
                    const double dk = di(q, 0) * pg.sx + di(q, 1) * pg.sy + di(q, 2) * pg.sz;
                    const double dl = Rl[4 + 3 * m] * pg.sx + Rl[5 + 3 * m] * pg.sy + Rl[6 + 3 * m] * pg.sz;
                    const double mm = minmod_med(dk, dl);
                    qL[m] = ui(q) + pg.fk * mm;
                    qR[m] = Rl[m] - pg.fl * mm;
                }
                // face guards and M1 fluxes: F_X.A = (FA_X, a_X A + b_X F_X)
                double FAL, aL, bL, FAR, aR, bR;
                const int f1 = face_m164(qL, pg.Ax, pg.Ay, pg.Az, c, c3, FAL, aL, bL);
                const int f2 = face_m164(qR, pg.Ax, pg.Ay, pg.Az, c, c3, FAR, aR, bR);
                double w1 = 0.5, w2 = 0.5, w3 = -hc * pg.An;   // GLF
                if (HLL) {
                    double loL, hiL, loR, hiR;
                    hll_speeds64(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll,
                                 loL, hiL);
                    hll_speeds64(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll,
                                 loR, hiR);
                    hll_weights(loL, hiL, loR, hiR, pg.An, w1, w2, w3);
                }
                if (use) {
                    cE += (f1 & 1) + (f2 & 1);
                    cF += (f1 >> 1) + (f2 >> 1);
                    // Phi.A = w1 F_L.A + w2 F_R.A + w3 (U_R - U_L), the vector part
                    // (w1 a_L + w2 a_R) A + w1 b_L F_L + w2 b_R F_R + w3 (F_R - F_L)
                    const double al = __builtin_fma(w1, aL, w2 * aR);
                    const double bl = w1 * bL, br = w2 * bR;
                    acc[4 * g] += wkl * __builtin_fma(w3, qR[0] - qL[0],
                                                      __builtin_fma(w1, FAL, w2 * FAR));
                    const double Av[3] = {pg.Ax, pg.Ay, pg.Az};
#pragma unroll
                    for (int m = 1; m < 4; ++m)
                        acc[4 * g + m] +=
                            wkl * __builtin_fma(w3, qR[m] - qL[m],
                                                __builtin_fma(al, Av[m - 1],
                                                              __builtin_fma(bl, qL[m], br * qR[m])));
                }
            }
        }
    }
    // sum of the Q partial sums of each particle (a fixed butterfly: the same
    // bits on every lane of the particle; by LDS permutes in the time-bin
    // instantiations, where the DPP form left more registers spilled)
    if (Q > 1) {
#pragma unroll
        for (int q = 0; q < 4 * GW; ++q) {
            if constexpr (BIN) {
#pragma unroll
                for (int o = 1; o < Q; o <<= 1) acc[q] += __shfl_xor(acc[q], o, 64);
            } else {
                quad_sum<Q>(acc[q]);
            }
        }
    }
    // update, post-update guard, ledger, photon budget
    double red[2 * GW];
    int gE = 0, gF = 0;
    double chk = 0.0;   // NaN iff an updated state is NaN or infinite
    if (BIN && owner && !ends) {
        // no update in this tick: keep the pending sums, count the current state
        const double V = rk[R_V];
#pragma unroll
        for (int g = 0; g < GW; ++g) {
            if (touched) {
                double *a = accm + (i * G + g0 + g) * 4;
#pragma unroll
                for (int m = 0; m < 4; ++m) a[m] += acc[4 * g + m];
            }
            red[g] = V * ui(4 * g);
            red[GW + g] = 0.0;
        }
    } else if (owner) {
        const double V = rk[R_V];
        // the update: U - dt/V sum (global step), or U - (pending + this tick)/V
        const double dtV = BIN ? 1.0 / V : dtp[0] / V;
        if (BIN) {
#pragma unroll
            for (int g = 0; g < GW; ++g) {
                double *a = accm + (i * G + g0 + g) * 4;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    acc[4 * g + m] += a[m];
                    a[m] = 0.0;
                }
            }
        }
#pragma unroll
        for (int g = 0; g < GW; ++g) {
            double q0 = ui(4 * g + 0) - dtV * acc[4 * g + 0];
            double q1 = ui(4 * g + 1) - dtV * acc[4 * g + 1];
            double q2 = ui(4 * g + 2) - dtV * acc[4 * g + 2];
            double q3 = ui(4 * g + 3) - dtV * acc[4 * g + 3];
            const double Epre = q0;
            chk = __builtin_fma(q0, 0.0, chk);
            chk = __builtin_fma(q1, 0.0, chk);
            chk = __builtin_fma(q2, 0.0, chk);
            chk = __builtin_fma(q3, 0.0, chk);
            if (Uung) {
                double *u = Uung + i * NQ + 4 * (g0 + g);
                u[0] = q0;
                u[1] = q1;
                u[2] = q2;
                u[3] = q3;
            }
            const int f = guard64(q0, q1, q2, q3, c);
            gE += f & 1;
            gF += f >> 1;
            double *o = Uout + i * NQ + 4 * (g0 + g);
            o[0] = q0;
            o[1] = q1;
            o[2] = q2;
            o[3] = q3;
            red[g] = V * q0;
            red[GW + g] = (f & 1) ? -Epre * V : 0.0;
        }
    } else {
#pragma unroll
        for (int p = 0; p < 2 * GW; ++p) red[p] = 0.0;
    }
    if (chk != chk) atomicOr(status, ST_NONFINITE);
    // partials [nb][2G]: photon totals in columns 0..G-1, ledger in G..2G-1
    if (partials)
        block_reduce_store<2 * GW>(red, partials + blk * 2 * G, smem,
                                   [&](int p) { return p < GW ? g0 + p : G + g0 + p - GW; });
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

// Transport with the pairs inside a tile evaluated once (FP64, GLF or HLL,
// Hopkins or Ivanova surfaces, one global step, all G <= 3 groups in one
// wave).  Both solvers' pair fluxes and both surfaces are antisymmetric, so
// one evaluation serves both particles of a pair.
//
// A block owns one tile: the 64 consecutive Morton particles of one column
// block of the neighbour table, 16 per wave with 4 lanes each (the layout, and
// so the cache footprint, of the two-sided kernel).  A particle's task list
// (k_tasks, built with the geometry) holds its neighbours outside the tile and
// its share of the pairs inside it: an in-tile pair (k, l) is evaluated by one
// of its particles only (chosen to balance the lists' lengths), flagged by
// the sign bit.  That lane adds Phi_kl to its own sum and -Phi_kl, by an LDS
// atomic add, to the other particle's row of its own wave's copy of the
// tile's accumulator; the pair's face states are the same from either side,
// so its face-guard counts are taken twice.  After a block barrier each
// particle's sum is its own partial sums plus the 4 waves' rows, added in a
// fixed order, so runs are bitwise reproducible, and the in-tile pair flux
// is antisymmetric bit for bit.  49.5% of the neighbour entries of the 128^3
// lattice lie inside their tile, so a step evaluates 75% of the pair fluxes
// of the two-sided kernel.  (With a wave owning a whole tile in 4 passes the
// XCD's working set spanned 4 times the particles and its L2 hit rate fell
// from 92% to 38%.)

//
// BIN: one tick of the individual-time-step scheme on the tiles.  A pair is
// due when its smaller bin ends a step in this tick, a symmetric condition,
// and its flux weighted by dt 2^min(b_k, b_l) is antisymmetric as before; a
// particle none of whose pairs is due (binm) walks no list.  The particles
// that do not end a step add their sums to the pending sums accm, the others
// apply theirs, as in the two-sided binned kernel.
template <int G, bool OFF32, bool HLL, bool IVA, bool BIN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2, 2))) void
k_transport64_tile(int64_t n, int64_t nb, const double *__restrict__ geo,
                   const int32_t *__restrict__ task, const int64_t *__restrict__ wave_base,
                   const int32_t *__restrict__ n_task, const double *__restrict__ UD,
                   const double *__restrict__ dtp, double c, double box,
                   double *__restrict__ Uout, double *__restrict__ partials,
                   unsigned long long *__restrict__ counts, double *__restrict__ Uung,
                   int32_t *__restrict__ status, const double2 *__restrict__ hll,
                   int64_t tick = 0, double *__restrict__ accm = nullptr,
                   const uint8_t *__restrict__ binm = nullptr) {
    constexpr int NQ = 4 * G, MS = NQ + 1;     // accumulator row, padded against bank conflicts
    __shared__ double stage[kBlock / 64][64 * kStage];
    static_assert(kTile == 64 && kBlock == 256, "a block of 4 waves x 16 particles per tile");
    __shared__ double mir[kBlock / 64][kTile * MS];
    constexpr int DS = 3 * NQ + 1;              // own-gradient row, padded
    __shared__ double dsh[kBlock / 64][16 * DS];
    __shared__ double smem[(kBlock / 64) * 2 * G];
    __shared__ unsigned long long scnt[4];
    const int64_t blk = xcd_block(nb);
    if (blk >= nb) return;                      // whole block: no barrier is skipped
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int sub = lane & 3;
    const int64_t t0 = blk * kTile;             // the tile's first particle
    const bool wave_live = t0 + 16 * wv < n;    // wave-uniform
    const double ibox = 1.0 / box, hc = 0.5 * c, c3 = 3.0 * c;
    if (threadIdx.x < 4) scnt[threadIdx.x] = 0;
    double *sb = stage[wv];
    double *mw = mir[wv];                       // this wave's copy of the accumulator
    for (int e = lane; e < kTile * MS; e += 64) mw[e] = 0.0;
    wave_lds_sync();
    int cE = 0, cF = 0;
    const int pl = 16 * wv + (lane >> 2);       // the lane's particle in the tile
    double acc[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) acc[q] = 0.0;
    // BIN: this particle ends a step in this tick (ends), or some pair of its
    // neighbourhood is due (touched)
    const int64_t t1 = tick + 1;
    int32_t bk = 0;
    bool ends = true, touched = true;
    if constexpr (BIN) {
        const int64_t icb = t0 + pl < n ? t0 + pl : n - 1;
        bk = (int32_t)geo[(int64_t)kRec * icb + 12];
        const int32_t bm = binm ? (int32_t)binm[icb] : 0;
        ends = (t1 & ((int64_t(1) << bk) - 1)) == 0;
        touched = (t1 & ((int64_t(1) << bm) - 1)) == 0;
    }
    if (wave_live) {
        const int64_t wb = wave_base[blk];
        {
            const int64_t i = t0 + pl;
            const bool active = i < n;
            const int64_t ic = active ? i : n - 1;
            const int32_t nn = (active && touched) ? n_task[i] : 0;
            int32_t kmax = nn;                      // the longest list of the pass
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) kmax = max(kmax, __shfl_xor(kmax, o, 64));
            const double *rk = geo + (int64_t)kRec * ic;
            // IVA: the kernel-gradient sums, slots 13-15 of the records
            const double gk[3] = {IVA ? rk[13] : 0.0, IVA ? rk[14] : 0.0, IVA ? rk[15] : 0.0};
            double Ui[NQ];
#pragma unroll
            for (int g = 0; g < G; ++g) {
                const double *r = UD + (ic * G + g) * 16;
#pragma unroll
                for (int m = 0; m < 4; ++m) Ui[4 * g + m] = r[m];
            }
            // the own gradients live in LDS (4 lanes read one address); lane
            // sub copies component sub's
            double *Dsh = dsh[wv] + (lane >> 2) * DS;
#pragma unroll
            for (int g = 0; g < G; ++g)
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    Dsh[3 * (4 * g + sub) + a] = UD[(ic * G + g) * 16 + 4 + 3 * sub + a];
            wave_lds_sync();
            const int64_t base = wb + pl;   // the particle's column in the table
            // Lines in flight: v holds the loads of the next stage (the
            // geometry lines, then each group's record lines) while the
            // current stage is evaluated from the stage buffer.  The task of
            // the next iteration is loaded one iteration ahead.
            int32_t tc = sub < nn ? task[base + 64 * (int64_t)sub] : (int32_t)ic;
            int32_t rw[8];
            double2 v[8];
            {
                const int32_t j = tc & 0x7fffffff;
#pragma unroll
                for (int m = 0; m < 8; ++m) rw[m] = __shfl(j, 8 * m + (lane >> 3), 64);
                const RowLines<OFF32> gl(geo, rw, 1, lane);
                gl.load(0, v);
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
                const RowLines<OFF32> ul(UD, rw, G, lane);
                store_lines(v, sb, lane);       // the geometry lines
                ul.load(0, v);
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
                bool use = valid && pg.An > 0.0;
                double wkl = 1.0;                   // BIN: time integration of the exchange
                if constexpr (BIN) {
                    const int32_t bl = (int32_t)sb[lane * kStage + 12];
                    const int32_t bmin = bk < bl ? bk : bl;
                    use = use && (t1 & ((int64_t(1) << bmin) - 1)) == 0;
                    wkl = ldexp(dtp[0], bmin);
                }
                const double iAn = (HLL && pg.An > 0.0) ? rcp64(pg.An) : 0.0;
                const int cnt2 = mirror ? 2 : 1;
                const int mr = mirror ? (j - (int32_t)t0) * MS : 0;   // the partner's row
#pragma unroll
                for (int g = 0; g < G; ++g) {
                    // the stages in program order: each one's loads stay in
                    // flight across the evaluation of the previous one
                    __builtin_amdgcn_sched_barrier(0);
                    store_lines(v, sb, lane);   // group g's record lines
                    if (g + 1 < G) {
                        ul.load(g + 1, v);
                    } else {                    // the next iteration's geometry lines
                        const int32_t jn = tn & 0x7fffffff;
#pragma unroll
                        for (int m = 0; m < 8; ++m) rw[m] = __shfl(jn, 8 * m + (lane >> 3), 64);
                        const RowLines<OFF32> gn(geo, rw, 1, lane);
                        gn.load(0, v);
                    }
                    const double *Rl = sb + lane * kStage;
                    double qL[4], qR[4];
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const int q = 4 * g + m;
                        const double dk = Dsh[3 * q] * pg.sx + Dsh[3 * q + 1] * pg.sy + Dsh[3 * q + 2] * pg.sz;
                        const double dl = Rl[4 + 3 * m] * pg.sx + Rl[5 + 3 * m] * pg.sy + Rl[6 + 3 * m] * pg.sz;
                        const double mm = minmod_med(dk, dl);
                        qL[m] = Ui[q] + pg.fk * mm;
                        qR[m] = Rl[m] - pg.fl * mm;
                    }
                    double FAL, aL, bL, FAR, aR, bR;
                    const int f1 = face_m164(qL, pg.Ax, pg.Ay, pg.Az, c, c3, FAL, aL, bL);
                    const int f2 = face_m164(qR, pg.Ax, pg.Ay, pg.Az, c, c3, FAR, aR, bR);
                    double w1 = 0.5, w2 = 0.5, w3 = -hc * pg.An;   // GLF
                    if constexpr (HLL) {
                        double loL, hiL, loR, hiR;
                        hll_speeds64(qL[0], qL[1], qL[2], qL[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll,
                                     loL, hiL);
                        hll_speeds64(qR[0], qR[1], qR[2], qR[3], pg.Ax, pg.Ay, pg.Az, iAn, c, hll,
                                     loR, hiR);
                        hll_weights(loL, hiL, loR, hiR, pg.An, w1, w2, w3);
                    }
                    if (use) {
                        cE += cnt2 * ((f1 & 1) + (f2 & 1));
                        cF += cnt2 * ((f1 >> 1) + (f2 >> 1));
                        const double al = __builtin_fma(w1, aL, w2 * aR);
                        const double bl = w1 * bL, br = w2 * bR;
                        double phi[4];
                        phi[0] = __builtin_fma(w3, qR[0] - qL[0], __builtin_fma(w1, FAL, w2 * FAR));
                        const double Av[3] = {pg.Ax, pg.Ay, pg.Az};
#pragma unroll
                        for (int m = 1; m < 4; ++m)
                            phi[m] = __builtin_fma(w3, qR[m] - qL[m],
                                                   __builtin_fma(al, Av[m - 1],
                                                                 __builtin_fma(bl, qL[m], br * qR[m])));
                        if constexpr (BIN) {
#pragma unroll
                            for (int m = 0; m < 4; ++m) phi[m] *= wkl;
                        }
#pragma unroll
                        for (int m = 0; m < 4; ++m) acc[4 * g + m] += phi[m];
                        if (mirror) {
#pragma unroll
                            for (int m = 0; m < 4; ++m) atomicAdd(mw + mr + 4 * g + m, -phi[m]);
                        }
                    }
                }
                tc = tn;
                __builtin_amdgcn_sched_barrier(0);
            }
            // the 4 lanes' partial sums, combined by a fixed butterfly
#pragma unroll
            for (int q = 0; q < NQ; ++q)
                quad_sum<4>(acc[q]);
        }
    }
    // every wave's deposits are in its copy of the accumulator
    __syncthreads();
    // update, post-update guard, ledger, photon budget: the first lane of each
    // particle; its sum is its own partial sums plus the 4 waves' rows, in
    // that fixed order
    const int64_t i = t0 + pl;
    const bool owner = wave_live && sub == 0 && i < n;
    double red[2 * G];
    int gE = 0, gF = 0;
    double chk = 0.0;   // NaN iff an updated state is NaN or infinite
    if (BIN && owner && !ends) {
        // no update in this tick: keep the pending sums, count the current state
        const double V = geo[(int64_t)kRec * i + R_V];
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int v = 0; v < kBlock / 64; ++v) acc[q] += mir[v][pl * MS + q];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            if (touched) {
                double *a = accm + (i * G + g) * 4;
#pragma unroll
                for (int m = 0; m < 4; ++m) a[m] += acc[4 * g + m];
            }
            red[g] = V * UD[(i * G + g) * 16];
            red[G + g] = 0.0;
        }
    } else if (owner) {
        const double V = geo[(int64_t)kRec * i + R_V];
        // the update: U - dt/V sum (global step), or U - (pending + this tick)/V
        const double dtV = BIN ? 1.0 / V : dtp[0] / V;
#pragma unroll
        for (int q = 0; q < NQ; ++q)
#pragma unroll
            for (int v = 0; v < kBlock / 64; ++v) acc[q] += mir[v][pl * MS + q];
        if constexpr (BIN) {
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double *a = accm + (i * G + g) * 4;
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    acc[4 * g + m] += a[m];
                    a[m] = 0.0;
                }
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const double *u = UD + (i * G + g) * 16;
            double q0 = u[0] - dtV * acc[4 * g + 0];
            double q1 = u[1] - dtV * acc[4 * g + 1];
            double q2 = u[2] - dtV * acc[4 * g + 2];
            double q3 = u[3] - dtV * acc[4 * g + 3];
            const double Epre = q0;
            chk = __builtin_fma(q0, 0.0, chk);
            chk = __builtin_fma(q1, 0.0, chk);
            chk = __builtin_fma(q2, 0.0, chk);
            chk = __builtin_fma(q3, 0.0, chk);
            if (Uung) {
                double *uu = Uung + i * NQ + 4 * g;
                uu[0] = q0;
                uu[1] = q1;
                uu[2] = q2;
                uu[3] = q3;
            }
            const int f = guard64(q0, q1, q2, q3, c);
            gE += f & 1;
            gF += f >> 1;
            double *o = Uout + i * NQ + 4 * g;
            o[0] = q0;
            o[1] = q1;
            o[2] = q2;
            o[3] = q3;
            red[g] = V * q0;
            red[G + g] = (f & 1) ? -Epre * V : 0.0;
        }
    } else {
#pragma unroll
        for (int p = 0; p < 2 * G; ++p) red[p] = 0.0;
    }
    if (chk != chk) atomicOr(status, ST_NONFINITE);
    if (partials)
        block_reduce_store<2 * G>(red, partials + blk * 2 * G, smem, [&](int p) { return p; });
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

// ---------------------------------------------------------------------------
// Photon budget Q_g = sum_k V_k E_kg: block partials, then one block combines
// them with compensated (two-sum) arithmetic in a fixed order.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_total_partials(int64_t n, int G,
                                                           const double *__restrict__ geo,
                                                           const T *__restrict__ U,
                                                           double *__restrict__ partials) {
    __shared__ double smem[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    for (int g = 0; g < G; ++g) {
        double v = (i < n) ? geo[(int64_t)kRec * i + R_V] * (double)U[(i * G + g) * 4] : 0.0;
        smem[threadIdx.x] = v;
        __syncthreads();
        for (int s = kBlock / 2; s > 0; s >>= 1) {
            if (threadIdx.x < s) smem[threadIdx.x] += smem[threadIdx.x + s];
            __syncthreads();
        }
        if (threadIdx.x == 0) partials[(int64_t)blockIdx.x * 2 * G + g] = smem[0];
        __syncthreads();
    }
}

__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}

// part [nb][2G]: columns 0..G-1 photon totals, G..2G-1 ledger.  Q[g] = sum (written),
// ledger[g] += sum.  Two passes in a fixed order:
//  1. block k of kFinBlocks takes the rows [k m, (k+1) m), m = ceil(nb / kFinBlocks):
//     thread t sums rows t, t + kBlock, ... of it (whole rows, so consecutive
//     threads read consecutive rows), one compensated sum per column, and the
//     block's 256 sums of each column meet in a fixed tree;
//  2. one block combines the kFinBlocks compensated sums of each column.
constexpr int kFinBlocks = 32;

// Fixed tree over the block of the compensated pairs (ss, sc); the result is
// in ss[0] + sc[0].
__device__ __forceinline__ void block_two_sum_tree(double *ss, double *sc) {
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) {
            double t, err;
            two_sum(ss[threadIdx.x], ss[threadIdx.x + w], t, err);
            ss[threadIdx.x] = t;
            sc[threadIdx.x] += sc[threadIdx.x + w] + err;
        }
        __syncthreads();
    }
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_finalize_rows(int64_t nb, const double *__restrict__ part,
                                                          double *__restrict__ fin) {
    constexpr int C = 2 * G;
    __shared__ double ss[kBlock], sc[kBlock];
    const int64_t m = (nb + kFinBlocks - 1) / kFinBlocks;
    const int64_t r0 = blockIdx.x * m, r1 = min(nb, r0 + m);
    double s[C], e[C];
#pragma unroll
    for (int c = 0; c < C; ++c) s[c] = e[c] = 0.0;
    for (int64_t b = r0 + threadIdx.x; b < r1; b += kBlock) {
        const double *row = part + b * C;
#pragma unroll
        for (int c = 0; c < C; ++c) {
            double t, err;
            two_sum(s[c], row[c], t, err);
            s[c] = t;
            e[c] += err;
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        ss[threadIdx.x] = s[c];
        sc[threadIdx.x] = e[c];
        block_two_sum_tree(ss, sc);
        if (threadIdx.x == 0) {
            fin[(blockIdx.x * C + c) * 2] = ss[0];
            fin[(blockIdx.x * C + c) * 2 + 1] = sc[0];
        }
        __syncthreads();
    }
}

template <int G>
__global__ __launch_bounds__(kBlock) void k_finalize(const double *__restrict__ fin,
                                                     double *__restrict__ Q,
                                                     double *__restrict__ ledger) {
    constexpr int C = 2 * G;
    __shared__ double ss[kBlock], sc[kBlock];
    for (int c = 0; c < C; ++c) {
        double *dst = c < G ? Q : ledger;
        if (!dst) continue;
        const bool in = threadIdx.x < kFinBlocks;
        ss[threadIdx.x] = in ? fin[(threadIdx.x * C + c) * 2] : 0.0;
        sc[threadIdx.x] = in ? fin[(threadIdx.x * C + c) * 2 + 1] : 0.0;
        block_two_sum_tree(ss, sc);
        if (threadIdx.x == 0) {
            double v = ss[0] + sc[0];
            if (c < G) Q[c] = v;
            else ledger[c - G] += v;
        }
        __syncthreads();
    }
}

// part is ctx->partials; the kFinBlocks x 2G compensated pairs of the first
// pass go to the slack the buffer keeps after its rows.
template <int G>
void launch_finalize(rt_ctx *ctx, int64_t nb, const double *part, double *Q, double *ledger) {
    double *fin = ctx->partials + 2 * G * ctx->nblocks;
    k_finalize_rows<G><<<kFinBlocks, kBlock, 0, ctx->stream>>>(nb, part, fin);
    k_finalize<G><<<1, kBlock, 0, ctx->stream>>>(fin, Q, ledger);
}

// Groups per wave of the FP64 transport (0: the default slice below).  All
// groups in one wave compute the pair geometry once; each group costs about
// 40 registers, and with more than 3 groups a wave no longer fits the 256
// registers of 2 waves per SIMD (G = 3: 254 VGPRs), so larger G is cut into
// slices of 2 groups (or 3, or one group per wave as the last resort).
#ifndef RT_TRANSPORT_GW
#define RT_TRANSPORT_GW 0
#endif
constexpr int transport_slice(int G) {
    return G <= 3 ? G : (G % 2 == 0 ? 2 : (G % 3 == 0 ? 3 : 1));
}
// The HLL solver holds about 10 more registers per group in flight (the wave
// speeds of both face states).  With the particle's own state in LDS (OWNL)
// all groups fit one wave up to G = 3 (256 VGPRs, no spill), measured 15%
// faster on the 3-group 128^3 lattice than one group per wave at 3 waves per
// SIMD (6.2 against 7.3 ms); larger odd G runs one group per wave, held in
// registers at 3 waves per SIMD.
#ifndef RT_HLL_GW
#define RT_HLL_GW 0
#endif
constexpr int hll_slice(int G) { return G <= 3 ? G : (G % 2 == 0 ? 2 : 1); }

// Lanes per particle of the FP64 transport (1, 2 or 4): with Q > 1 a wave
// covers 64/Q particles whose neighbour lists overlap more, so the records
// one iteration stages repeat more often in the caches.  Q = 4 cut the
// calibrated fetch of the 3-group 128^3 lattice 14x (35 GB to 2.5 GB per
// launch) and the time by 11% against Q = 1.
#ifndef RT_TRANSPORT_Q
#define RT_TRANSPORT_Q 4
#endif
constexpr int kQ = RT_TRANSPORT_Q;
// rows of block partials the FP64 transport writes (one per block)
inline int64_t transport_rows(int64_t n) { return (n + kBlock / kQ - 1) / (kBlock / kQ); }

// The FP64 global step with GLF and the Hopkins surfaces (up to 3 groups, all
// in one wave) evaluates in-tile pairs once (k_transport64_tile); 0 selects
// the two-sided kernel for it too.
#ifndef RT_TRANSPORT_TILE
#define RT_TRANSPORT_TILE 1
#endif
// The HLL solver takes the tiles too (its flux is as antisymmetric as GLF's);
// 0 keeps it two-sided.
#ifndef RT_TRANSPORT_TILE_HLL
#define RT_TRANSPORT_TILE_HLL 1
#endif
// The Ivanova surfaces too (antisymmetric as well, A_lk = -A_kl; the
// kernel-gradient sums come with the geometry records); 0 keeps them
// two-sided.
#ifndef RT_TRANSPORT_TILE_IVA
#define RT_TRANSPORT_TILE_IVA 1
#endif
// The ticks of the individual time steps on the tiles too (a due pair's
// weighted flux is antisymmetric); 0 keeps them two-sided.
#ifndef RT_TICK_TILE
#define RT_TICK_TILE 1
#endif
// ... and their gradients from the neighbour unions; 0: staged.
#ifndef RT_TICK_UNION
#define RT_TICK_UNION 1
#endif
inline bool use_tile64(const rt_ctx *ctx) {
    return RT_TRANSPORT_TILE != 0 && ctx->p.precision == RT_FP64 &&
           (ctx->solver == RT_GLF || (RT_TRANSPORT_TILE_HLL != 0 && ctx->solver == RT_HLL)) &&
           (ctx->surfaces == RT_HOPKINS ||
            (RT_TRANSPORT_TILE_IVA != 0 && ctx->surfaces == RT_IVANOVA)) &&
           ctx->p.groups <= 3 && ctx->task != nullptr;
}
// rows of block partials the FP64 transport writes (one per block)
inline int64_t transport64_rows(const rt_ctx *ctx) {
    return use_tile64(ctx) ? (ctx->p.n + kTile - 1) / kTile : transport_rows(ctx->p.n);
}

template <int G>
void launch_transport64(rt_ctx *ctx, const double *UD, const double *dt, double *Uout,
                        double *partials, int64_t *counts, double *Uung) {
    constexpr int GW =
        (RT_TRANSPORT_GW == 0 || G % RT_TRANSPORT_GW != 0) ? transport_slice(G) : RT_TRANSPORT_GW;
    constexpr int HW = (RT_HLL_GW == 0 || G % RT_HLL_GW != 0) ? hll_slice(G) : RT_HLL_GW;
    const int64_t n = ctx->p.n, nb = transport_rows(n);
    const double2 *tab = (const double2 *)ctx->hll_table;
    const bool iva = ctx->surfaces == RT_IVANOVA;
    if constexpr (G <= 3) {
        if (use_tile64(ctx)) {
            const int64_t nt = transport64_rows(ctx);
            // rows addressed by 32-bit offsets while the gradient records fit 4 GiB
#define RT_TILE_LAUNCH(OFF32_, HLL_, IVA_)                                                     \
    k_transport64_tile<G, OFF32_, HLL_, IVA_, false><<<(unsigned)xcd_grid(nt), kBlock, 0, ctx->stream>>>( \
        n, nt, ctx->geo, ctx->task, ctx->wave_base, ctx->n_task, UD, dt, ctx->p.c_red,           \
        ctx->p.box, Uout, partials, (unsigned long long *)counts, Uung, ctx->status, tab)
#define RT_TILE_LAUNCH_S(HLL_, IVA_)                                                           \
    do {                                                                                       \
        if (off32) RT_TILE_LAUNCH(true, HLL_, IVA_);                                           \
        else RT_TILE_LAUNCH(false, HLL_, IVA_);                                                \
    } while (0)
            const bool off32 = (uint64_t)n * 128u * G < (uint64_t(1) << 32);
            if (ctx->solver == RT_HLL) {
                if (iva) RT_TILE_LAUNCH_S(true, true);
                else RT_TILE_LAUNCH_S(true, false);
            } else {
                if (iva) RT_TILE_LAUNCH_S(false, true);
                else RT_TILE_LAUNCH_S(false, false);
            }
#undef RT_TILE_LAUNCH_S
#undef RT_TILE_LAUNCH
            return;
        }
    }
#define RT_TRANSPORT_LAUNCH(W, HLL_, IVA_)                                                    \
    k_transport64<G, W, false, HLL_, IVA_, kQ, own_lds(HLL_, IVA_, W),                        \
                  pipe_on(HLL_, IVA_, W)>                                                     \
        <<<(unsigned)xcd_grid(nb * (G / W)), kBlock, 0, ctx->stream>>>(                       \
        n, nb, ctx->geo, ctx->nbr, ctx->wave_base, ctx->n_nbr, UD, dt, ctx->p.c_red,          \
        ctx->p.box, Uout, partials, (unsigned long long *)counts, Uung, ctx->status, 0,       \
        nullptr, tab, nullptr)
    if (ctx->solver == RT_HLL) {
        if (iva) RT_TRANSPORT_LAUNCH(HW, true, true);
        else RT_TRANSPORT_LAUNCH(HW, true, false);
    } else {
        if (iva) RT_TRANSPORT_LAUNCH(GW, false, true);
        else RT_TRANSPORT_LAUNCH(GW, false, false);
    }
#undef RT_TRANSPORT_LAUNCH
}

// Lanes per particle of the FP64 gradient (1, 2 or 4); Q = 4 measured 14%
// faster than Q = 1 on the 3-group 128^3 lattice.
#ifndef RT_GRADIENT_Q
#define RT_GRADIENT_Q 4
#endif
constexpr int kGQ = RT_GRADIENT_Q;

template <int G>
void launch_gradient64(rt_ctx *ctx, const double *U, double *UD) {
    constexpr int B = grad_block(G);
    if constexpr (union_cap(G) > 0 && kGQ == 4 && B == 256) {
        if (ctx->uoff) {
            // blocks whose union fits: from LDS; the others: staged, by list
            const int64_t nw = ctx->nwaves;
#define RT_UNION_LAUNCH(W_)                                                                    \
    k_gradient64u<G, kGQ, W_><<<(unsigned)xcd_grid(nw), kBlock, 0, ctx->stream>>>(            \
        ctx->p.n, nw, ctx->geo, ctx->xs, ctx->urow, ctx->uoff, ctx->gloc, ctx->goff,          \
        ctx->uown, ctx->n_gath, U, UD, ctx->status, ctx->p.box)
            if constexpr (union_cap3(G) > 0) {
                if (ctx->union_waves == 3) RT_UNION_LAUNCH(3);
                else RT_UNION_LAUNCH(2);
            } else {
                RT_UNION_LAUNCH(2);
            }
#undef RT_UNION_LAUNCH
            if (ctx->n_ublk > 0)
                k_gradient64<G, false, kGQ><<<(unsigned)xcd_grid(ctx->n_ublk), B, 0, ctx->stream>>>(
                    ctx->p.n, ctx->n_ublk, ctx->geo, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath,
                    U, UD, ctx->status, ctx->p.box, 0, ctx->ublk);
            return;
        }
    }
    const int64_t n = ctx->p.n, nb = (n + B / kGQ - 1) / (B / kGQ);
    k_gradient64<G, false, kGQ><<<(unsigned)xcd_grid(nb), B, 0, ctx->stream>>>(
        n, nb, ctx->geo, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath, U, UD, ctx->status,
        ctx->p.box);
}

template <int G>
void launch_tick64(rt_ctx *ctx, const double *U, double *UD, const double *dt, double *Uout,
                   double *partials, int64_t *counts, int64_t tick, double *accm) {
    const int64_t n = ctx->p.n;
    constexpr int B = grad_block(G);
    const int64_t ng = (n + B / kGQ - 1) / (B / kGQ);
    bool grad_done = false;
    if constexpr (union_cap(G) > 0 && kGQ == 4 && B == 256) {
        if (RT_TICK_UNION != 0 && ctx->uoff) {
            // the neighbour unions, in their time-bin mode; the blocks whose
            // union does not fit: staged, by list
            const int64_t nw = ctx->nwaves;
#define RT_TICK_UNION_LAUNCH(W_)                                                               \
    k_gradient64u<G, kGQ, W_, true><<<(unsigned)xcd_grid(nw), kBlock, 0, ctx->stream>>>(      \
        n, nw, ctx->geo, ctx->xs, ctx->urow, ctx->uoff, ctx->gloc, ctx->goff, ctx->uown,       \
        ctx->n_gath, U, UD, ctx->status, ctx->p.box, tick)
            if constexpr (union_cap3(G) > 0) {
                if (ctx->union_waves == 3) RT_TICK_UNION_LAUNCH(3);
                else RT_TICK_UNION_LAUNCH(2);
            } else {
                RT_TICK_UNION_LAUNCH(2);
            }
#undef RT_TICK_UNION_LAUNCH
            if (ctx->n_ublk > 0)
                k_gradient64<G, true, kGQ><<<(unsigned)xcd_grid(ctx->n_ublk), B, 0, ctx->stream>>>(
                    n, ctx->n_ublk, ctx->geo, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath,
                    U, UD, ctx->status, ctx->p.box, tick, ctx->ublk);
            grad_done = true;
        }
    }
    if (!grad_done)
        k_gradient64<G, true, kGQ><<<(unsigned)xcd_grid(ng), B, 0, ctx->stream>>>(
            n, ng, ctx->geo, ctx->xs, ctx->nbr, ctx->wave_base, ctx->n_gath, U, UD, ctx->status,
            ctx->p.box, tick);
    constexpr int GW = transport_slice(G), HW = hll_slice(G);
    const int64_t nt = transport_rows(n);
    const double2 *tab = (const double2 *)ctx->hll_table;
    const bool iva = ctx->surfaces == RT_IVANOVA;
    const uint8_t *binm = ctx->bin8 ? ctx->bin8 + n : nullptr;
    if constexpr (G <= 3) {
        if (RT_TICK_TILE != 0 && use_tile64(ctx)) {
            // the tiles in their time-bin mode (one row of partials per tile,
            // as many as the two-sided kernel's blocks)
            static_assert(kBlock / kQ == kTile, "a tile per two-sided block");
            const bool off32 = (uint64_t)n * 128u * G < (uint64_t(1) << 32);
#define RT_TICK_TILE_LAUNCH(OFF32_, HLL_, IVA_)                                                 \
    k_transport64_tile<G, OFF32_, HLL_, IVA_, true>                                             \
        <<<(unsigned)xcd_grid(nt), kBlock, 0, ctx->stream>>>(                                   \
            n, nt, ctx->geo, ctx->task, ctx->wave_base, ctx->n_task, UD, dt, ctx->p.c_red,      \
            ctx->p.box, Uout, partials, (unsigned long long *)counts, nullptr, ctx->status,     \
            tab, tick, accm, binm)
#define RT_TICK_TILE_S(HLL_, IVA_)                                                              \
    do {                                                                                        \
        if (off32) RT_TICK_TILE_LAUNCH(true, HLL_, IVA_);                                       \
        else RT_TICK_TILE_LAUNCH(false, HLL_, IVA_);                                            \
    } while (0)
            if (ctx->solver == RT_HLL) {
                if (iva) RT_TICK_TILE_S(true, true);
                else RT_TICK_TILE_S(true, false);
            } else {
                if (iva) RT_TICK_TILE_S(false, true);
                else RT_TICK_TILE_S(false, false);
            }
#undef RT_TICK_TILE_S
#undef RT_TICK_TILE_LAUNCH
            return;
        }
    }
#define RT_TICK_LAUNCH(W, HLL_, IVA_)                                                          \
    k_transport64<G, W, true, HLL_, IVA_, kQ, own_lds(HLL_, IVA_, W),                         \
                  pipe_on(HLL_, IVA_, W)>                                                     \
        <<<(unsigned)xcd_grid(nt * (G / W)), kBlock, 0, ctx->stream>>>(                        \
            n, nt, ctx->geo, ctx->nbr, ctx->wave_base, ctx->n_nbr, UD, dt, ctx->p.c_red,       \
            ctx->p.box, Uout, partials, (unsigned long long *)counts, nullptr, ctx->status,    \
            tick, accm, tab, binm)
    if (ctx->solver == RT_HLL) {
        if (iva) RT_TICK_LAUNCH(HW, true, true);
        else RT_TICK_LAUNCH(HW, true, false);
    } else {
        if (iva) RT_TICK_LAUNCH(GW, false, true);
        else RT_TICK_LAUNCH(GW, false, false);
    }
#undef RT_TICK_LAUNCH
}

#define RT_DISPATCH_G(G_, FN, ...)                                  \
    switch (G_) {                                                   \
        case 1: FN<1>(__VA_ARGS__); break;                          \
        case 2: FN<2>(__VA_ARGS__); break;                          \
        case 3: FN<3>(__VA_ARGS__); break;                          \
        case 4: FN<4>(__VA_ARGS__); break;                          \
        case 5: FN<5>(__VA_ARGS__); break;                          \
        case 6: FN<6>(__VA_ARGS__); break;                          \
        case 7: FN<7>(__VA_ARGS__); break;                          \
        case 8: FN<8>(__VA_ARGS__); break;                          \
        default: break;                                             \
    }

}  // namespace

// Combine nb rows of ctx->partials into Q (columns 0..G-1, written) and
// ledger (columns G..2G-1, accumulated); either may be NULL.
void rt_finalize_partials(rt_ctx *ctx, int64_t nb, double *Q, double *ledger) {
    RT_DISPATCH_G(ctx->p.groups, launch_finalize, ctx, nb, ctx->partials, Q, ledger);
}

rt_status rt_ensure_partials(rt_ctx *ctx) {
    // enough rows for every kernel that writes them (the FP64 transport runs
    // up to 4 lanes per particle, so up to 4 blocks per kBlock particles)
    const int64_t nb = (4 * ctx->p.n + kBlock - 1) / kBlock;
    if (ctx->partials && ctx->nblocks >= nb) return RT_OK;
    rt_free(ctx, ctx->partials);
    ctx->partials = nullptr;
    // the rows, then the first pass of the finalize (kFinBlocks x 2G pairs)
    rt_status rs = rt_alloc(ctx, (void **)&ctx->partials,
                            sizeof(double) * 2 * ctx->p.groups * (nb + 2 * kFinBlocks));
    if (rs != RT_OK) return rs;
    ctx->nblocks = nb;
    return RT_OK;
}

rt_status rt_inject_impl(rt_ctx *ctx, void *U, const double *L, const double *dt) {
    if (ctx->S == 0 || ctx->n_inj_gas == 0) return RT_OK;
    rt_timer_begin(ctx, "inject");
    if (ctx->p.precision == RT_FP64)
        k_inject<double><<<nblk(ctx->n_inj_gas), kBlock, 0, ctx->stream>>>(
            ctx->n_inj_gas, ctx->p.groups, ctx->inj_gptr, ctx->inj_gas, ctx->inj_src,
            ctx->inj_coef, L, dt, (double *)U);
    else
        k_inject<float><<<nblk(ctx->n_inj_gas), kBlock, 0, ctx->stream>>>(
            ctx->n_inj_gas, ctx->p.groups, ctx->inj_gptr, ctx->inj_gas, ctx->inj_src,
            ctx->inj_coef, L, dt, (float *)U);
    rt_timer_end(ctx, "inject");
    RT_HIP(hipGetLastError());
    return RT_OK;
}

rt_status rt_gradient_impl(rt_ctx *ctx, const void *U, void *UD) {
    rt_timer_begin(ctx, "gradient");
    if (ctx->p.precision == RT_FP64) {
        RT_DISPATCH_G(ctx->p.groups, launch_gradient64, ctx, (const double *)U, (double *)UD);
    } else {
        rt_gradient32(ctx, (const float *)U, (float *)UD);
    }
    rt_timer_end(ctx, "gradient");
    RT_HIP(hipGetLastError());
    return RT_OK;
}

rt_status rt_transport_impl(rt_ctx *ctx, const void *UD, const double *dt, void *U_out,
                            double *Q, int64_t *counts, double *ledger, void *Uung) {
    // rows of block partials: the FP64 kernel's blocks, or one per kBlock particles
    const int64_t nb = ctx->p.precision == RT_FP64 ? transport64_rows(ctx)
                                                   : rt_transport32_rows(ctx->p.n);
    double *part = (Q || ledger) ? ctx->partials : nullptr;
    rt_timer_begin(ctx, "transport");
    if (ctx->p.precision == RT_FP64) {
        RT_DISPATCH_G(ctx->p.groups, launch_transport64, ctx, (const double *)UD, dt,
                      (double *)U_out, part, counts, (double *)Uung);
    } else {
        rt_transport32(ctx, (const float *)UD, dt, (float *)U_out, part, counts, (float *)Uung);
    }
    rt_timer_end(ctx, "transport");
    RT_HIP(hipGetLastError());
    if (part) {
        RT_DISPATCH_G(ctx->p.groups, launch_finalize, ctx, nb, part, Q, ledger);
        RT_HIP(hipGetLastError());
    }
    return RT_OK;
}

// Gradient and transport of one tick of the individual-time-step scheme
// (FP64; injection and the refresh of the stored states are in rt_bins.hip).
rt_status rt_tick_step_impl(rt_ctx *ctx, double *U, double *UD, const double *dt, int64_t tick,
                            double *accm, double *Q, int64_t *counts, double *ledger) {
    const int64_t nb = transport_rows(ctx->p.n);
    double *part = (Q || ledger) ? ctx->partials : nullptr;
    rt_timer_begin(ctx, "tick");
    RT_DISPATCH_G(ctx->p.groups, launch_tick64, ctx, U, UD, dt, U, part, counts, tick, accm);
    rt_timer_end(ctx, "tick");
    RT_HIP(hipGetLastError());
    if (part) {
        RT_DISPATCH_G(ctx->p.groups, launch_finalize, ctx, nb, part, Q, ledger);
        RT_HIP(hipGetLastError());
    }
    return RT_OK;
}

rt_status rt_total_impl(rt_ctx *ctx, const void *U, double *Q) {
    const int64_t n = ctx->p.n, nb = (n + kBlock - 1) / kBlock;
    if (ctx->p.precision == RT_FP64)
        k_total_partials<double><<<(unsigned)nb, kBlock, 0, ctx->stream>>>(
            n, ctx->p.groups, ctx->geo, (const double *)U, ctx->partials);
    else
        k_total_partials<float><<<(unsigned)nb, kBlock, 0, ctx->stream>>>(
            n, ctx->p.groups, ctx->geo, (const float *)U, ctx->partials);
    RT_DISPATCH_G(ctx->p.groups, launch_finalize, ctx, nb, ctx->partials, Q, nullptr);
    RT_HIP(hipGetLastError());
    return RT_OK;
}
