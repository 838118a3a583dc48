// Internal declarations of the gfx950 photon-transport library.
// Device helpers shared by the build, step and adjoint translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <string>
#include <unordered_map>
#include <vector>

#include "../../include/rt.h"

namespace gearrt {

constexpr int kWave = 64;     // wavefront width on CDNA
constexpr int kBlock = 256;   // threads per block of the per-particle kernels
constexpr int kLeaf = 32;     // particles per leaf of the search tree
constexpr int kRec = 16;      // doubles per particle geometry record (one 128-byte line)
// Particles per tile of the FP64 tile transport: the 64 consecutive Morton
// particles of one column block of the neighbour table, whose pairs are
// evaluated once.  (Tiles of 16 and 32 particles, one wave per tile, ran
// 3.84 and 3.78 ms against 3.64 for 64 on the 3-group 128^3 lattice.)
constexpr int kTile = 64;
// Rows of a block's neighbour union that the FP64 gradient stages in LDS (a
// block of 64 particles, two blocks per CU: 4G + 3 doubles a row in at most
// 80 KB); 0: no union path at this group count.  At most kUnionSort.
constexpr int kUnionSort = 1024;
constexpr int union_cap(int G) { return G == 1 ? 1024 : G == 2 ? 880 : G == 3 ? 640 : G == 4 ? 512 : 0; }
// At 3 groups a smaller union (420 rows) lets three blocks share a CU, 3
// waves per SIMD; the build takes it when nearly every block's union fits.
constexpr int union_cap3(int G) { return G == 3 ? 420 : 0; }
// The compensated-FP32 gradient's union: FP32 states (16G bytes a row), FP64
// positions, three blocks per CU (at most 53 KB each).
constexpr int union_cap32(int G) { return G == 1 ? 1024 : G == 2 ? 880 : G == 3 ? 672 : G == 4 ? 576 : 0; }
// Rows of a block's union in the adjoint's transposed gradient, which stages
// one group at a time: position, 1/H and the 12 gradient cotangents (128
// bytes) plus the row index, 132 bytes a row.  2 or 3 blocks of 4 waves per CU.
constexpr int adj_union_cap(int waves) { return waves == 3 ? 400 : 600; }
constexpr double kPi = 3.14159265358979323846;
constexpr double kSigma3 = 16.0 / kPi;   // cubic spline normalisation in 3D

// Device status word bits.
enum : int32_t { ST_NOCONV = 1, ST_SINGULAR = 2, ST_BIGH = 4, ST_NONFINITE = 8 };

// Geometry record, one per particle (Morton order), 128 bytes (12 used):
//   0..2  x, y, z       position in [0, box)
//   3     1/H           inverse compact support radius, H = kappa h
//   4     h             smoothing length
//   5     V             particle volume 1/omega
//   6..11 Bv            V * S^{-1}, S = sum_j s s^T w(r/H) (upper triangle
//                       00 01 02 11 12 22); A_kl = (w_k Bv_k + w_l Bv_l) s
//                       and the gradient matrix is S^{-1} = Bv / V.
enum { R_X = 0, R_IH = 3, R_H = 4, R_V = 5, R_B = 6 };

// Record of the compensated-FP32 path, 64 bytes (16 floats): positions stay
// FP64 (floats 0..5 hold x, y, z as doubles; separations are formed in FP64
// and rounded once), then 1/H, h, Bv (6) and V in FP32.
enum { F_IH = 6, F_H = 7, F_B = 8, F_V = 14, F_BIN = 15, F_REC = 16 };

struct TimerRec {
    std::string name;
    hipEvent_t a, b;
};

}  // namespace gearrt

struct rt_ctx {
    rt_params p{};
    hipStream_t stream = nullptr;
    std::string err;
    int device = 0;
    int built = 0;

    // sorted particles and geometry
    double *xs = nullptr;        // [n][3] Morton-ordered positions
    double *geo = nullptr;       // [n][kRec]
    double *vol = nullptr;       // [n] V_i (copy of the record's slot R_V)
    float *geo32 = nullptr;      // [n][F_REC] (FP32C only)
    int32_t *perm32 = nullptr;   // [n]
    uint64_t *keys = nullptr;    // [n] sorted Morton keys
    double *dt_dev = nullptr;    // [1]
    int32_t *h_iters = nullptr;  // [n]

    // search tree over leaves of kLeaf consecutive sorted particles (heap layout)
    int64_t nleaf = 0, P = 0;    // P = leaves padded to a power of two
    double *node_lo = nullptr;   // [2P][3]
    double *node_hi = nullptr;   // [2P][3]
    double *node_hmax = nullptr; // [2P] max H below the node

    // wave-sliced neighbour table: wave w owns slots [wave_base[w], wave_base[w+1]),
    // slot (lane, j) at wave_base[w] + 64 j + lane
    int64_t nwaves = 0, slots = 0, n_entries = 0, n_gather_entries = 0;
    int32_t max_nbr = 0;
    int32_t *n_nbr = nullptr;    // [n]
    int32_t *n_gath = nullptr;   // [n]
    int64_t *wave_base = nullptr;// [nwaves + 1]
    int32_t *nbr = nullptr;      // [slots]
    int32_t *task = nullptr;     // [slots] task lists of the FP64 tile transport (same slots)
    int32_t *n_task = nullptr;   // [n]
    int64_t *tstat = nullptr;    // [2] over the tiles: the longest task list, its lower bound
    // neighbour unions of the FP64 gradient (k_union): per block of 64
    // particles its sorted distinct gather neighbours and own particles
    int64_t *uoff = nullptr;     // [nwaves + 1] offsets into urow (no rows: staged gradient)
    int32_t *urow = nullptr;     // [uoff[nwaves]]
    // a gather slot's position in its block's union, packed so that a lane's
    // entries of four consecutive iterations share 8 bytes: entry (p, k) of
    // block b at goff[b] + (k / 16) 1024 + (4 p + k % 4) 4 + (k / 4) % 4
    uint16_t *gloc = nullptr;
    int64_t *goff = nullptr;     // [nwaves + 1], 1024 ceil(rows / 16) entries per block
    uint16_t *uown = nullptr;    // [n] a particle's position in its block's union
    int32_t *ublk = nullptr;     // [n_ublk] blocks left to the staged gradient
    int64_t n_ublk = 0;
    int union_waves = 2;         // waves per SIMD of the union gradient (capacity by it)
    // the same over the symmetric lists, for the FP64 adjoint's transposed
    // gradient (entries packed as gloc, at the same goff)
    int64_t *aoff = nullptr;
    int32_t *arow = nullptr;
    uint16_t *agloc = nullptr;
    uint16_t *aown = nullptr;
    int32_t *ablk = nullptr;
    int64_t n_ablk = 0;
    int adj_union_waves = 2;

    // sources
    int32_t S = 0;
    double *src_h = nullptr;     // [S]
    int64_t n_inj = 0;           // injection entries
    int32_t n_inj_gas = 0;       // distinct gas particles receiving energy
    int32_t *inj_gptr = nullptr; // [n_inj_gas + 1] gas-major CSR
    int32_t *inj_gas = nullptr;  // [n_inj_gas]
    int32_t *inj_src = nullptr;  // [n_inj]
    double *inj_coef = nullptr;  // [n_inj] xi_sg / V_g
    double *inj_xi = nullptr;    // [n_inj] xi_sg
    int32_t *src_ptr = nullptr;  // [S + 1] source-major CSR into the arrays below
    int32_t *src_gas = nullptr;  // [n_inj]
    double *src_coef = nullptr;  // [n_inj]

    // scratch
    int32_t *status = nullptr;   // device status word
    double *partials = nullptr;  // [nblocks][2 G] block partial sums
    int64_t nblocks = 0;
    void *scan_tmp = nullptr;
    size_t scan_tmp_bytes = 0;
    void *adj_buf = nullptr;     // adjoint scratch (see rt_adjoint.hip)
    size_t adj_bytes = 0;

    int64_t device_bytes = 0;    // device memory the context holds now
    int64_t device_peak = 0;     // the most it held at once since rt_create
    std::unordered_map<void *, size_t> allocs;   // live allocations and their sizes
    int64_t h_list_overflow = 0; // particles whose h-solve candidate list overflowed
    int32_t h_iter_max = 0;
    int32_t h_iter_cap = 200;    // iteration cap of the smoothing-length solve
    int32_t bin_top = -1;        // largest time bin after rt_time_bins (-1: none)
    uint8_t *bin8 = nullptr;     // [2n] time bins as set by rt_time_bins, then the smallest
                                 // bin of each particle's neighbourhood (0 after a build)
    int32_t solver = RT_GLF;     // Riemann solver of the transport
    double *hll_table = nullptr; // [RT_HLL_NF][RT_HLL_NMU][2] wave speeds / c
    float *hll_table32 = nullptr;// the same in FP32 (FP32C contexts)
    int32_t surfaces = RT_HOPKINS; // effective surfaces of the transport
    double *ivan = nullptr;      // [n][4] sum_k grad W_k(x_i) (Ivanova surfaces)

    // timing: event pairs recorded around launches while timing is on
    int timing = 0;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    std::vector<gearrt::TimerRec> trecs;
    std::vector<hipEvent_t> ev_open;   // stack of open timers (nested launches)
};

namespace gearrt {

// ---------------------------------------------------------------------------
// device helpers

// Dimensionless cubic B-spline w(q), q = r/H, written branch-free:
// (1-q)^3 - 4 (1/2-q)^3 for q <= 1/2, (1-q)^3 for 1/2 < q < 1, 0 beyond.
// Exchange within a quad of lanes by DPP (a VALU move, no LDS round trip):
// quad_xor<O> returns the value of the lane whose index differs in bit O
// (1 or 2); quad_sum<Q> adds the Q lanes' values (Q = 1, 2 or 4) in the
// order xor 1, then xor 2, leaving the same bits on every lane.  Every lane of
// the quad must be active.
template <int O>
__device__ __forceinline__ int quad_xor_i(int v) {
    static_assert(O == 1 || O == 2, "a quad's bit 0 or 1");
    return __builtin_amdgcn_mov_dpp(v, O == 1 ? 0xB1 : 0x4E, 0xf, 0xf, false);
}
template <int O>
__device__ __forceinline__ float quad_xor(float v) {
    return __builtin_bit_cast(float, quad_xor_i<O>(__builtin_bit_cast(int, v)));
}
template <int O>
__device__ __forceinline__ double quad_xor(double v) {
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    const uint32_t lo = (uint32_t)quad_xor_i<O>((int)(uint32_t)b);
    const uint32_t hi = (uint32_t)quad_xor_i<O>((int)(uint32_t)(b >> 32));
    return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
template <int Q, class T>
__device__ __forceinline__ void quad_sum(T &v) {
    static_assert(Q == 1 || Q == 2 || Q == 4, "lanes per particle: 1, 2 or 4");
    if constexpr (Q >= 2) v += quad_xor<1>(v);
    if constexpr (Q >= 4) v += quad_xor<2>(v);
}

__device__ __forceinline__ double kern_w(double q) {
    double a = fmax(1.0 - q, 0.0);
    double b = fmax(0.5 - q, 0.0);
    return a * a * a - 4.0 * (b * b * b);
}
__device__ __forceinline__ float kern_wf(float q) {
    float a = fmaxf(1.0f - q, 0.0f);
    float b = fmaxf(0.5f - q, 0.0f);
    return a * a * a - 4.0f * (b * b * b);
}
// dw/dq
__device__ __forceinline__ double kern_dw(double q) {
    double a = fmax(1.0 - q, 0.0);
    double b = fmax(0.5 - q, 0.0);
    return -3.0 * a * a + 12.0 * (b * b);
}
__device__ __forceinline__ float kern_dwf(float q) {
    float a = fmaxf(1.0f - q, 0.0f);
    float b = fmaxf(0.5f - q, 0.0f);
    return -3.0f * a * a + 12.0f * (b * b);
}

// 1/x for normal x > 0: the hardware estimate (v_rcp_f64, about 2^-23
// relative) refined by two Newton-Raphson steps r <- r + r (1 - x r), which
// square the error each: about one ulp.
__device__ __forceinline__ double rcp64(double x) {
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
}
// 1/sqrt(x) for normal x > 0: hardware estimate (v_rsq_f64) and two Newton
// steps y <- y (3 - x y^2)/2.
__device__ __forceinline__ double rsq64(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double h = 0.5 * x;
    double t = __builtin_fma(-h * y, y, 0.5);
    y = __builtin_fma(y, t, y);
    t = __builtin_fma(-h * y, y, 0.5);
    return __builtin_fma(y, t, y);
}
// sqrt(x) for x >= 0: g = x / sqrt(x) from rsq64 and one Newton correction of
// the root, g <- g + (x - g^2) / (2 g); sqrt(0) = 0.
__device__ __forceinline__ double sqrt64(double x) {
    double y = rsq64(x);
    double g = x * y;
    double d = __builtin_fma(-g, g, x);
    g = __builtin_fma(d, 0.5 * y, g);
    return x > 0.0 ? g : 0.0;
}

// Periodic nearest-image separation component.
__device__ __forceinline__ double min_image(double d, double box, double ibox) {
    return d - box * rint(d * ibox);
}

// Squared distance from point p to the axis-aligned box [lo, hi] in a periodic
// domain of side `box` (boxes are given in [0, box) coordinates).
__device__ __forceinline__ double box_dist2(const double *lo, const double *hi, double px,
                                            double py, double pz, double box) {
    double p[3] = {px, py, pz};
    double d2 = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double in = fmax(0.0, fmax(lo[a] - p[a], p[a] - hi[a]));
        double up = fmax(0.0, p[a] + box - hi[a]);     // image p + box
        double dn = fmax(0.0, lo[a] - p[a] + box);     // image p - box
        double d = fmin(in, fmin(up, dn));
        d2 += d * d;
    }
    return d2;
}

// Stackless depth-first traversal of the heap-ordered complete binary tree:
// node v has children 2v, 2v+1; leaves are P .. 2P-1.  `accept(v)` decides
// whether to open node v; `leaf(l)` is called for accepted leaf l.
template <class Accept, class Leaf>
__device__ __forceinline__ void traverse(int64_t P, Accept &&accept, Leaf &&leaf) {
    int64_t v = 1;
    while (true) {
        if (accept(v)) {
            if (v >= P) {
                leaf(v - P);
            } else {
                v = 2 * v;
                continue;
            }
        }
        while (v & 1) v >>= 1;   // climb while v is a right child
        if (v == 0) break;       // passed the root
        v = v + 1;               // right sibling
    }
}

// XCD-aware block mapping: blocks are dispatched round-robin over the 8 XCDs
// of the chip; remap so that each XCD works on one contiguous range of
// particles (its L2 then holds that range's neighbour data).  The grid has
// 8 * ceil(nb / 8) blocks; blocks mapped past nb return.
__device__ __forceinline__ int64_t xcd_block(int64_t nb) {
    int64_t b = blockIdx.x;
    int64_t per = (nb + 7) / 8;
    return (b & 7) * per + (b >> 3);
}
inline int64_t xcd_grid(int64_t nb) { return 8 * ((nb + 7) / 8); }

// Wave-level sum of a double (all 64 lanes active or inactive lanes contributing 0).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}
__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

}  // namespace gearrt

// ---------------------------------------------------------------------------
// host-side helpers shared by the translation units

#define RT_HIP(expr)                                                              \
    do {                                                                          \
        hipError_t _e = (expr);                                                   \
        if (_e != hipSuccess) {                                                   \
            ctx->err = std::string(#expr) + ": " + hipGetErrorString(_e);         \
            return RT_EHIP;                                                       \
        }                                                                         \
    } while (0)

rt_status rt_fail(rt_ctx *ctx, rt_status st, const std::string &msg);
rt_status rt_alloc(rt_ctx *ctx, void **ptr, size_t bytes);
// rt_alloc for optional scratch: false (and no error message) when it fails
bool rt_try_alloc(rt_ctx *ctx, void **ptr, size_t bytes);
// free memory from rt_alloc / rt_try_alloc and take it off the context's count
void rt_free(rt_ctx *ctx, void *ptr);
void rt_timer_begin(rt_ctx *ctx, const char *name);
void rt_timer_end(rt_ctx *ctx, const char *name);

// build (rt_build.hip)
rt_status rt_build_impl(rt_ctx *ctx, const double *x, const double *h_in, int64_t *perm,
                        double *h, double *V, double *dt);
rt_status rt_sources_impl(rt_ctx *ctx, int32_t n_src, const double *xs, double eta_star);

// step (rt_step.hip)
rt_status rt_inject_impl(rt_ctx *ctx, void *U, const double *L, const double *dt);
rt_status rt_gradient_impl(rt_ctx *ctx, const void *U, void *UD);
rt_status rt_transport_impl(rt_ctx *ctx, const void *UD, const double *dt, void *U_out,
                            double *Q, int64_t *counts, double *ledger, void *Uung);
rt_status rt_total_impl(rt_ctx *ctx, const void *U, double *Q);
// compensated-FP32 launches (rt_step32.hip)
void rt_gradient32(rt_ctx *ctx, const float *U, float *UD);
void rt_transport32(rt_ctx *ctx, const float *UD, const double *dt, float *Uout,
                    double *partials, int64_t *counts, float *Uung);
int64_t rt_transport32_rows(int64_t n);   // rows of block partials rt_transport32 writes
void rt_adjoint32(rt_ctx *ctx, const float *UD, const float *Uung, const float *lam_next,
                  float *lam2, float *R, float *lam, const double *dt);
rt_status rt_ensure_partials(rt_ctx *ctx);
void rt_finalize_partials(rt_ctx *ctx, int64_t nb, double *Q, double *ledger);

// photo-absorption (rt_absorb.hip): group constants on the host, removal kernel
rt_status rt_photon_groups_impl(int32_t G, const double *edges_eV, double T_bb, double *sigma_N,
                                double *sigma_E, double *eps, double *frac, std::string &err);
rt_status rt_absorb_impl(rt_ctx *ctx, void *U, int32_t J, const double *n_old,
                         const double *n_new, const double *sigma, const double *dt, double *Q,
                         double *absorbed);

// individual time steps (rt_bins.hip; the binned gradient and transport in rt_step.hip)
rt_status rt_time_bins_impl(rt_ctx *ctx, int32_t max_bin, int32_t *bins, int64_t *cycle);
rt_status rt_tick_impl(rt_ctx *ctx, void *U, const double *L, int64_t tick, void *UD,
                       double *acc, double *Q, int64_t *counts, double *ledger);
// the gradient and transport of one tick (rt_step.hip, rt_step32.hip)
rt_status rt_tick_step_impl(rt_ctx *ctx, double *U, double *UD, const double *dt, int64_t tick,
                            double *accm, double *Q, int64_t *counts, double *ledger);
rt_status rt_tick_step32_impl(rt_ctx *ctx, float *U, float *UD, const double *dt, int64_t tick,
                              double *accm, double *Q, int64_t *counts, double *ledger);

// drift correction (rt_drift.hip)
rt_status rt_drift_impl(rt_ctx *ctx, const void *UD, const double *dx, void *U_out, double *Q,
                        int64_t *counts, double *ledger);

// Ivanova surfaces (rt_ivanova.hip): per-particle kernel-gradient sums
rt_status rt_ivanova_impl(rt_ctx *ctx);
rt_status rt_set_surfaces_impl(rt_ctx *ctx, int32_t kind);

// HLL wave speeds (rt_hll.hip): the host table and the solver switch
std::vector<double> rt_hll_speed_table(int nf, int nmu);
rt_status rt_set_riemann_impl(rt_ctx *ctx, int32_t solver);

// adjoint (rt_adjoint.hip)
rt_status rt_adjoint_impl(rt_ctx *ctx, const void *U_pre, const double *L, const double *dt,
                          const void *UD, const void *U_ung, const void *lam_next, void *lam,
                          double *dL_dL);
// the allocation-free adjoint (rt_adjoint.hip): per-device scratch lookup (from
// rt_create), the scratch bytes a context needs, and the entry point
void rt_adjoint_static_init(rt_ctx *ctx);
size_t rt_adjoint_static_bytes(const rt_ctx *ctx);
rt_status rt_adjoint_static_impl(rt_ctx *ctx, const double *L, const double *dt, const void *UD,
                                 const void *U_ung, const void *lam_next, void *lam,
                                 double *dL_dL);
