// Static geometry of the particle set: Morton order, search tree, smoothing
// lengths, wave-sliced neighbour table, particle volumes and the inverse
// least-squares matrices, global time step; point-source injection weights.
//
// Particles are static interpolation points for the radiation (Part III,
// "Using a particle based method: selecting reference frames"), so everything
// here is computed once and reused by every transport step.
#include <cstring>

#include <rocprim/rocprim.hpp>

#include <algorithm>
#include <numeric>
#include <vector>

#include "rt_internal.h"

using namespace gearrt;

namespace {

// ---------------------------------------------------------------------------
// Morton keys: 21 bits per axis, interleaved into 63 bits.
__device__ __forceinline__ uint64_t spread21(uint64_t v) {
    v &= 0x1fffffULL;
    v = (v | (v << 32)) & 0x1f00000000ffffULL;
    v = (v | (v << 16)) & 0x1f0000ff0000ffULL;
    v = (v | (v << 8)) & 0x100f00f00f00f00fULL;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ULL;
    v = (v | (v << 2)) & 0x1249249249249249ULL;
    return v;
}

__global__ void k_morton(int64_t n, const double *__restrict__ x, double ibox,
                         uint64_t *__restrict__ keys, int32_t *__restrict__ idx) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t c[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double f = x[3 * i + a] * ibox;
        f = fmin(fmax(f, 0.0), 1.0);
        uint64_t q = (uint64_t)(f * 2097152.0);
        c[a] = q > 2097151ULL ? 2097151ULL : q;
    }
    keys[i] = (spread21(c[0]) << 2) | (spread21(c[1]) << 1) | spread21(c[2]);
    idx[i] = (int32_t)i;
}

__global__ void k_gather_sorted(int64_t n, const double *__restrict__ x,
                                const int32_t *__restrict__ perm, const double *__restrict__ h_in,
                                double *__restrict__ xs, double *__restrict__ h,
                                int64_t *__restrict__ perm_out) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t j = perm[i];
    xs[3 * i + 0] = x[3 * j + 0];
    xs[3 * i + 1] = x[3 * j + 1];
    xs[3 * i + 2] = x[3 * j + 2];
    if (h_in) h[i] = h_in[j];
    if (perm_out) perm_out[i] = j;
}

// ---------------------------------------------------------------------------
// Search tree: leaves of kLeaf consecutive Morton-ordered particles, complete
// binary tree in heap layout above them.  Every node holds the bounding box
// of its particles and the largest compact support radius H below it.
__global__ void k_leaf_boxes(int64_t n, int64_t nleaf, int64_t P, const double *__restrict__ xs,
                             const double *__restrict__ H, double *__restrict__ lo,
                             double *__restrict__ hi, double *__restrict__ hmax) {
    int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= P) return;
    int64_t v = P + l;
    double bl[3] = {INFINITY, INFINITY, INFINITY}, bh[3] = {-INFINITY, -INFINITY, -INFINITY};
    double hm = 0.0;
    if (l < nleaf) {
        int64_t j0 = l * kLeaf, j1 = min(n, j0 + kLeaf);
        for (int64_t j = j0; j < j1; ++j) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                bl[a] = fmin(bl[a], xs[3 * j + a]);
                bh[a] = fmax(bh[a], xs[3 * j + a]);
            }
            if (H) hm = fmax(hm, H[j]);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        lo[3 * v + a] = bl[a];
        hi[3 * v + a] = bh[a];
    }
    hmax[v] = hm;
}

__global__ void k_merge_level(int64_t first, int64_t count, double *__restrict__ lo,
                              double *__restrict__ hi, double *__restrict__ hmax) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    int64_t v = first + t, a = 2 * v, b = 2 * v + 1;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        lo[3 * v + d] = fmin(lo[3 * a + d], lo[3 * b + d]);
        hi[3 * v + d] = fmax(hi[3 * a + d], hi[3 * b + d]);
    }
    hmax[v] = fmax(hmax[a], hmax[b]);
}

// Candidate-list capacity of the smoothing-length solve (entries per
// particle) and the most device memory the lists may take.
constexpr int kHList = 128;
// Entries per particle of the neighbour lists the count pass keeps (same budget).
constexpr int kNList = 128;
constexpr int64_t kHListBytes = int64_t(16) << 30;
// Bit of a particle's iteration count set when its candidate list overflowed
// (later evaluations at a smaller h walked the tree again).
constexpr int32_t kIterOverflow = 1 << 24;

struct Tree {
    const double *lo, *hi, *hmax;
    int64_t P;
};

// ---------------------------------------------------------------------------
// Smoothing length: root of g(h) = h^3 sum_j W(r_j, kappa h) - eta^3
// (eq:number-of-neighbors), i.e. (sigma/kappa^3) sum_j w(r_j / (kappa h)) = eta^3,
// by Newton-Raphson safeguarded with bisection.  An evaluation of g and dg/dh
// either walks the tree with radius kappa h or reads the particle's candidate
// list: the r^2 < (kappa h_l)^2 of the last walk, at h_l >= h, in walk order
// (entry k of particle i at list[k n + i]).  A walk at the smaller radius
// opens a subset of the same nodes in the same order, and a particle of a node
// it skips lies beyond kappa h, so both routes sum the same terms in the same
// order and give the same bits.  A particle whose list would overflow walks.
__device__ int h_eval(const Tree &T, const double *__restrict__ xs, int64_t n, double px,
                      double py, double pz, double h, double kappa, double box, double ibox,
                      double *__restrict__ list, int cap, double &sw, double &sdw) {
    const double H = kappa * h, H2 = H * H, iH = 1.0 / H;
    const double acc2 = H2 * (1.0 + 1e-12);
    double a = 0.0, b = 0.0;
    int cnt = 0;
    traverse(
        T.P,
        [&](int64_t v) { return box_dist2(T.lo + 3 * v, T.hi + 3 * v, px, py, pz, box) < acc2; },
        [&](int64_t l) {
            int64_t j0 = l * kLeaf, j1 = min(n, j0 + kLeaf);
            for (int64_t j = j0; j < j1; ++j) {
                double sx = min_image(xs[3 * j] - px, box, ibox);
                double sy = min_image(xs[3 * j + 1] - py, box, ibox);
                double sz = min_image(xs[3 * j + 2] - pz, box, ibox);
                double r2 = sx * sx + sy * sy + sz * sz;
                if (r2 < H2) {
                    if (cnt < cap) list[(int64_t)cnt * n] = r2;
                    ++cnt;
                    double q = sqrt(r2) * iH;
                    a += kern_w(q);
                    b += kern_dw(q) * q;
                }
            }
        });
    sw = a;
    sdw = b;
    return cnt;
}

__device__ void h_eval_list(const double *__restrict__ list, int64_t n, int cnt, double h,
                            double kappa, double &sw, double &sdw) {
    const double H = kappa * h, H2 = H * H, iH = 1.0 / H;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < cnt; ++k) {
        const double r2 = list[(int64_t)k * n];
        if (r2 < H2) {
            double q = sqrt(r2) * iH;
            a += kern_w(q);
            b += kern_dw(q) * q;
        }
    }
    sw = a;
    sdw = b;
}

__device__ double h_solve_point(const Tree &T, const double *__restrict__ xs, int64_t n,
                                double px, double py, double pz, double h0, double eta,
                                double kappa, double box, double hcap, double *__restrict__ list,
                                int cap, int32_t max_iter, int32_t &iters, int32_t &flags,
                                bool &overflow) {
    const double pref = kSigma3 / (kappa * kappa * kappa);
    const double eta3 = eta * eta * eta;
    const double eps4 = 4.0 * 2.220446049250313e-16;
    const double ibox = 1.0 / box;
    // iterates stay at or below hcap (compact support at most half the box);
    // a root beyond it is an error
    double lo = 0.0, hi = INFINITY, h = fmin(h0, hcap);
    double hl = 0.0;     // the list holds the walk at hl (0: no list)
    int lcnt = 0;
    int32_t it = 0;
    bool ok = false, big = false;
    for (it = 0; it < max_iter; ++it) {
        double sw, sdw;
        if (h <= hl) {
            h_eval_list(list, n, lcnt, h, kappa, sw, sdw);
        } else {
            lcnt = h_eval(T, xs, n, px, py, pz, h, kappa, box, ibox, list, cap, sw, sdw);
            hl = lcnt <= cap ? h : 0.0;
            if (list && lcnt > cap) overflow = true;
        }
        double g = pref * sw - eta3;
        double dg = -pref * sdw / h;
        if (g == 0.0) {
            ok = true;
            break;
        }
        if (g < 0.0) lo = h; else hi = h;
        double hn;
        if (hi == INFINITY) {
            if (h >= hcap) {                     // g < 0 at the cap
                big = true;
                break;
            }
            hn = 2.0 * h;                        // expand until bracketed
            if (dg > 0.0) {
                double nt = h - g / dg;
                if (nt > h && nt < 4.0 * h) hn = nt;
            }
            hn = fmin(hn, hcap);
        } else {
            // the step test comes before the bracket test: a Newton step that
            // rounds to h itself lands on a bracket end and would otherwise be
            // replaced by a bisection from a far end
            hn = (dg > 0.0) ? h - g / dg : -1.0;
            if (dg > 0.0 && fabs(hn - h) <= eps4 * h) {
                h = hn;
                ok = true;
                break;
            }
            if (!(hn > lo && hn < hi)) hn = 0.5 * (lo + hi);
            if (fabs(hn - h) <= eps4 * h || hi - lo <= eps4 * hi) {
                h = hn;
                ok = true;
                break;
            }
        }
        h = hn;
    }
    iters = it;
    if (big) flags |= ST_BIGH;
    else if (!ok) flags |= ST_NOCONV;
    return h;
}

// Starting point of the solve: the smaller of two density estimates (a walk
// costs about its radius cubed, so starting low is cheap and starting high is
// not):
//  - the particles per volume of the particle's leaf box (on a lattice about
//    0.7 of the root);
//  - from the fourth-nearest of the kGuessWin particles on either side in
//    Morton order, which bounds from above the distance to the fourth-nearest
//    particle, scaled by 0.8.  It stays local where a leaf straddles regions
//    of very different density and the leaf box overestimates h up to 35-fold.
constexpr int kGuessWin = 16;
__global__ void k_h_guess(int64_t n, int64_t P, const double *__restrict__ lo,
                          const double *__restrict__ hi, const double *__restrict__ xs,
                          double eta, double box, double *__restrict__ h) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t l = i / kLeaf, v = P + l;
    int64_t cnt = min((int64_t)kLeaf, n - l * kLeaf);
    double ext = 1.0;
    double floor_ext = box / 2097152.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) ext *= fmax(hi[3 * v + a] - lo[3 * v + a], floor_ext);
    double g = eta * cbrt(ext / (double)cnt);
    // four smallest r^2 in the Morton window, ascending
    const double ibox = 1.0 / box;
    const double px = xs[3 * i], py = xs[3 * i + 1], pz = xs[3 * i + 2];
    double d0 = INFINITY, d1 = INFINITY, d2 = INFINITY, d3 = INFINITY;
    const int64_t j0 = max((int64_t)0, i - kGuessWin), j1 = min(n, i + kGuessWin + 1);
    for (int64_t j = j0; j < j1; ++j) {
        if (j == i) continue;
        double sx = min_image(xs[3 * j] - px, box, ibox);
        double sy = min_image(xs[3 * j + 1] - py, box, ibox);
        double sz = min_image(xs[3 * j + 2] - pz, box, ibox);
        double r2 = sx * sx + sy * sy + sz * sz;
        if (r2 < d3) {
            d3 = r2;
            if (d3 < d2) { double t = d2; d2 = d3; d3 = t; }
            if (d2 < d1) { double t = d1; d1 = d2; d2 = t; }
            if (d1 < d0) { double t = d0; d0 = d1; d1 = t; }
        }
    }
    // n_local = 5 / ((4 pi / 3) r4^3)  ->  h = eta n_local^(-1/3)
    const double gm = eta * sqrt(d3) * 0.94269861348;      // cbrt((4 pi / 3) / 5)
    h[i] = fmin(fmin(g, 0.8 * gm), 0.25 * box);
}

__global__ void k_h_solve(int64_t n, Tree T, const double *__restrict__ xs, double eta,
                          double kappa, double box, double *__restrict__ h,
                          double *__restrict__ list, int cap, int32_t max_iter,
                          int32_t *__restrict__ iters, int32_t *__restrict__ status) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t it = 0, fl = 0;
    bool ovf = false;
    double hcap = 0.5 * box / kappa;
    double hv = h_solve_point(T, xs, n, xs[3 * i], xs[3 * i + 1], xs[3 * i + 2],
                              fmin(h[i], 0.5 * hcap), eta, kappa, box, hcap,
                              cap > 0 ? list + i : nullptr, cap, max_iter, it, fl, ovf);
    h[i] = hv;
    iters[i] = it | (ovf ? kIterOverflow : 0);
    if (fl) atomicOr(status, fl);
}

__global__ void k_scale(int64_t n, const double *__restrict__ a, double s, double *__restrict__ b) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = s * a[i];
}

// ---------------------------------------------------------------------------
// Neighbour lists N(i) = { j != i : r_ij < max(H_i, H_j) }: a pair exchanges
// flux whenever one of the two kernels reaches the other particle (then
// A_ij != 0).  The tree is opened when the node is within max(H_i, Hmax_node).
// The count pass also keeps, while they fit in cap entries, the neighbours it
// accepts in walk order (list[k n + i], a scatter neighbour with the sign bit
// set); the fill pass then places them from that list, gather neighbours first,
// in the order its own walk would, and walks only for the particles whose
// list overflowed.
template <bool FILL>
__global__ void k_neighbours(int64_t n, Tree T, const double *__restrict__ xs,
                             const double *__restrict__ H, double box,
                             int32_t *__restrict__ n_nbr, int32_t *__restrict__ n_gath,
                             const int64_t *__restrict__ wave_base, int32_t *__restrict__ nbr,
                             int32_t *__restrict__ list, int cap) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double ibox = 1.0 / box;
    const double px = xs[3 * i], py = xs[3 * i + 1], pz = xs[3 * i + 2];
    const double Hi = H[i], Hi2 = Hi * Hi;
    int32_t cg = 0, cs = 0;
    int64_t base = 0;
    int32_t gcount = 0, scount = 0;
    if (FILL) {
        base = wave_base[i >> 6] + (i & 63);
        gcount = n_gath[i];
        scount = n_nbr[i] - gcount;
        if (gcount + scount <= cap) {
            int32_t a = 0, b = 0;
            for (int32_t k = 0; k < gcount + scount; ++k) {
                const int32_t v = list[(int64_t)k * n + i];
                if (v >= 0) {
                    if (a < gcount) nbr[base + 64 * (int64_t)a] = v;
                    ++a;
                } else {
                    if (b < scount) nbr[base + 64 * (int64_t)(gcount + b)] = v & 0x7fffffff;
                    ++b;
                }
            }
            return;
        }
    }
    traverse(
        T.P,
        [&](int64_t v) {
            double R = fmax(Hi, T.hmax[v]);
            return box_dist2(T.lo + 3 * v, T.hi + 3 * v, px, py, pz, box) < R * R * (1.0 + 1e-12);
        },
        [&](int64_t l) {
            int64_t j0 = l * kLeaf, j1 = min(n, j0 + kLeaf);
            for (int64_t j = j0; j < j1; ++j) {
                if (j == i) continue;
                double sx = min_image(xs[3 * j] - px, box, ibox);
                double sy = min_image(xs[3 * j + 1] - py, box, ibox);
                double sz = min_image(xs[3 * j + 2] - pz, box, ibox);
                double r2 = sx * sx + sy * sy + sz * sz;
                double Hj = H[j];
                // the fill pass repeats the count pass exactly; the bounds only
                // keep a lane inside its own column of the wave's slice
                if (r2 < Hi2) {
                    if (FILL && cg < gcount) nbr[base + 64 * (int64_t)cg] = (int32_t)j;
                    if (!FILL && cg + cs < cap) list[(int64_t)(cg + cs) * n + i] = (int32_t)j;
                    ++cg;
                } else if (r2 < Hj * Hj) {
                    if (FILL && cs < scount) nbr[base + 64 * (int64_t)(gcount + cs)] = (int32_t)j;
                    if (!FILL && cg + cs < cap)
                        list[(int64_t)(cg + cs) * n + i] = (int32_t)j | INT32_MIN;
                    ++cs;
                }
            }
        });
    if (!FILL) {
        n_nbr[i] = cg + cs;
        n_gath[i] = cg;
    }
}

__global__ void k_wave_width(int64_t n, int64_t nwaves, const int32_t *__restrict__ n_nbr,
                             int64_t *__restrict__ width) {
    int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w > nwaves) return;
    if (w == nwaves) {
        width[w] = 0;
        return;
    }
    int32_t m = 0;
    int64_t i0 = w * 64, i1 = min(n, i0 + 64);
    for (int64_t i = i0; i < i1; ++i) m = max(m, n_nbr[i]);
    width[w] = 64 * (int64_t)m;
}

// ---------------------------------------------------------------------------
// Geometry (Part II "Partition of unity" and "Finite volume particle methods
// following Hopkins"): with w_ij = w(r_ij / H_i),
//   omega_i = (sigma/H_i^3) (w(0) + sum_j w_ij),  V_i = 1/omega_i,
//   E_i = sum_j s s^T psi_j(x_i) = (sigma/H_i^3) V_i S_i,  S_i = sum_j w_ij s s^T,
//   B_i = E_i^{-1} = S_i^{-1} / ((sigma/H_i^3) V_i).
// The record keeps Bv_i = V_i^2 (sigma/H_i^3) B_i = V_i S_i^{-1}, so that
//   A_kl = V_k psi~_l(x_k) - V_l psi~_k(x_l) = (w_kl Bv_k + w_lk Bv_l) s_kl.
// S_i is inverted in FP64 by cofactors.
__global__ void k_geometry(int64_t n, const double *__restrict__ xs, const double *__restrict__ h,
                           double kappa, double box, const int32_t *__restrict__ n_gath,
                           const int64_t *__restrict__ wave_base, const int32_t *__restrict__ nbr,
                           double *__restrict__ geo, float *__restrict__ geo32,
                           double *__restrict__ V_out, double *__restrict__ dxmin_part,
                           int32_t *__restrict__ status) {
    __shared__ double sm[kBlock / kWave];
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double dx = INFINITY;
    if (i < n) {
        const double ibox = 1.0 / box;
        const double px = xs[3 * i], py = xs[3 * i + 1], pz = xs[3 * i + 2];
        const double hi_ = h[i], H = kappa * hi_, iH = 1.0 / H;
        const int64_t base = wave_base[i >> 6] + (i & 63);
        const int32_t ng = n_gath[i];
        double sw = 0.0, s00 = 0, s01 = 0, s02 = 0, s11 = 0, s12 = 0, s22 = 0;
        for (int32_t k = 0; k < ng; ++k) {
            int64_t j = nbr[base + 64 * (int64_t)k];
            double sx = min_image(xs[3 * j] - px, box, ibox);
            double sy = min_image(xs[3 * j + 1] - py, box, ibox);
            double sz = min_image(xs[3 * j + 2] - pz, box, ibox);
            double r = sqrt(sx * sx + sy * sy + sz * sz);
            double w = kern_w(r * iH);
            sw += w;
            s00 += w * sx * sx; s01 += w * sx * sy; s02 += w * sx * sz;
            s11 += w * sy * sy; s12 += w * sy * sz; s22 += w * sz * sz;
        }
        double wnorm = kSigma3 * iH * iH * iH;
        double omega = wnorm * (0.5 + sw);
        double V = 1.0 / omega;
        // cofactor inverse of the symmetric S
        double c00 = s11 * s22 - s12 * s12;
        double c01 = s02 * s12 - s01 * s22;
        double c02 = s01 * s12 - s02 * s11;
        double c11 = s00 * s22 - s02 * s02;
        double c12 = s01 * s02 - s00 * s12;
        double c22 = s00 * s11 - s01 * s01;
        double det = s00 * c00 + s01 * c01 + s02 * c02;
        double tr = s00 + s11 + s22;
        if (!(det > 1e-12 * tr * tr * tr / 27.0)) {
            atomicOr(status, ST_SINGULAR);
            det = INFINITY;   // zero matrix: no gradient, no surface from this side
        }
        double f = V / det;
        double *rec = geo + (int64_t)kRec * i;
        rec[R_X + 0] = px;
        rec[R_X + 1] = py;
        rec[R_X + 2] = pz;
        rec[R_IH] = iH;
        rec[R_H] = hi_;
        rec[R_V] = V;
        rec[R_B + 0] = f * c00;
        rec[R_B + 1] = f * c01;
        rec[R_B + 2] = f * c02;
        rec[R_B + 3] = f * c11;
        rec[R_B + 4] = f * c12;
        rec[R_B + 5] = f * c22;
        rec[12] = rec[13] = rec[14] = rec[15] = 0.0;
        if (geo32) {
            float *r32 = geo32 + (int64_t)F_REC * i;
            double *xd = reinterpret_cast<double *>(r32);
            xd[0] = px;
            xd[1] = py;
            xd[2] = pz;
            r32[F_IH] = (float)iH;
            r32[F_H] = (float)hi_;
            r32[F_B + 0] = (float)(f * c00);
            r32[F_B + 1] = (float)(f * c01);
            r32[F_B + 2] = (float)(f * c02);
            r32[F_B + 3] = (float)(f * c11);
            r32[F_B + 4] = (float)(f * c12);
            r32[F_B + 5] = (float)(f * c22);
            r32[F_V] = (float)V;
            r32[15] = 0.0f;
        }
        V_out[i] = V;
        dx = cbrt(V * (3.0 / (4.0 * kPi)));
    }
    // block minimum of dx
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) dx = fmin(dx, __shfl_down(dx, o, 64));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = dx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = sm[0];
        for (int w = 1; w < kBlock / kWave; ++w) m = fmin(m, sm[w]);
        dxmin_part[blockIdx.x] = m;
    }
}

__global__ void k_dt(int64_t nb, const double *__restrict__ part, double cfl, double c,
                     double *__restrict__ dt) {
    __shared__ double sm[kBlock];
    double m = INFINITY;
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x) m = fmin(m, part[b]);
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int s = blockDim.x / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) sm[threadIdx.x] = fmin(sm[threadIdx.x], sm[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) dt[0] = cfl * sm[0] / c;
}

__global__ void k_copy_dt(const double *__restrict__ a, double *__restrict__ b) { b[0] = a[0]; }

// ---------------------------------------------------------------------------
// Sources (Part III "Weights for distribution of energy density of a star onto
// particles"): smoothing length of the source over the gas, then
//   psi_sg = W(r_sg, H_s) / sum_g' W(r_sg', H_s),
//   octant a(g) from the signs of x_g - x_s (components >= 0 count as +),
//   w_a = sum_{g in a} psi_sg,  mu_a = sum_b w_b / (q_nz w_a),
//   xi_sg = mu_a psi_sg   (eq:isotropy-correction-with-zero).
__global__ void k_src_h(int32_t S, Tree T, const double *__restrict__ xs, int64_t n,
                        const double *__restrict__ src_x, double eta, double kappa, double box,
                        double h0, int32_t max_iter, double *__restrict__ src_h,
                        int32_t *__restrict__ status) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    int32_t it = 0, fl = 0;
    bool ovf = false;
    double hcap = 0.5 * box / kappa;
    src_h[s] = h_solve_point(T, xs, n, src_x[3 * s], src_x[3 * s + 1], src_x[3 * s + 2], h0,
                             eta, kappa, box, hcap, nullptr, 0, max_iter, it, fl, ovf);
    if (fl) atomicOr(status, fl);
}

template <bool FILL>
__global__ void k_src_gas(int32_t S, Tree T, const double *__restrict__ xs, int64_t n,
                          const double *__restrict__ src_x, const double *__restrict__ src_h,
                          double kappa, double box, const double *__restrict__ geo,
                          int32_t *__restrict__ cnt, const int32_t *__restrict__ ptr,
                          int32_t *__restrict__ gas, double *__restrict__ xi,
                          double *__restrict__ coef) {
    int32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double ibox = 1.0 / box;
    const double px = src_x[3 * s], py = src_x[3 * s + 1], pz = src_x[3 * s + 2];
    const double H = kappa * src_h[s], H2 = H * H, iH = 1.0 / H;
    int32_t c = 0;
    int32_t o = FILL ? ptr[s] : 0;
    int32_t cap = FILL ? ptr[s + 1] - ptr[s] : 0;
    double wa[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    traverse(
        T.P,
        [&](int64_t v) {
            return box_dist2(T.lo + 3 * v, T.hi + 3 * v, px, py, pz, box) < H2 * (1.0 + 1e-12);
        },
        [&](int64_t l) {
            int64_t j0 = l * kLeaf, j1 = min(n, j0 + kLeaf);
            for (int64_t j = j0; j < j1; ++j) {
                double sx = min_image(xs[3 * j] - px, box, ibox);
                double sy = min_image(xs[3 * j + 1] - py, box, ibox);
                double sz = min_image(xs[3 * j + 2] - pz, box, ibox);
                double r2 = sx * sx + sy * sy + sz * sz;
                if (r2 < H2) {
                    if (FILL && c < cap) {
                        double w = kern_w(sqrt(r2) * iH);
                        int oc = (sx >= 0.0) | ((sy >= 0.0) << 1) | ((sz >= 0.0) << 2);
                        gas[o + c] = (int32_t)j;
                        xi[o + c] = w;
                        coef[o + c] = (double)oc;   // octant, replaced below
                        wa[oc] += w;
                    }
                    ++c;
                }
            }
        });
    if (!FILL) {
        cnt[s] = c;
        return;
    }
    int qnz = 0;
    for (int a = 0; a < 8; ++a) qnz += wa[a] > 0.0;
    // xi_sg = mu_a psi_sg with psi_sg = w_sg / wsum and w_a in units of wsum:
    // mu_a psi_sg = (wsum / (q_nz wa_a)) (w_sg / wsum) = w_sg / (q_nz wa_a)
    if (c > cap) c = cap;
    for (int32_t e = 0; e < c; ++e) {
        int oc = (int)coef[o + e];
        double x_ = xi[o + e] > 0.0 ? xi[o + e] / ((double)qnz * wa[oc]) : 0.0;
        xi[o + e] = x_;
        coef[o + e] = x_ / geo[(int64_t)kRec * gas[o + e] + R_V];
    }
}

// Second pass of the task lists: lower the tile's longest list, which sets
// how long the tile's block runs, by augmenting paths.  A particle k with the
// longest list (L entries) passes one of the pairs it evaluates, (k, l), to l;
// if l's list is not at least 2 shorter than L, l passes one of its own on,
// and so on along a breadth-first path (lowest indices first) that ends at a
// particle with at most L - 2 entries: k's list shrinks by one, the end's
// grows by one, the others keep their length.  Repeated while some particle
// with the longest list has such a path; each move lowers the sum of the
// squared lengths, so the loop ends.  On the lattices this reaches the lower
// bound, the larger of the longest list of neighbours outside the tile and
// the mean, in all but a few tiles.  One wave (lane = particle of the tile); cnt[k]:
// particle k's list length, bit l of own[k]: k evaluates the pair (k, l).
__device__ void level_tasks(bool active, int lane, int32_t *cnt, uint64_t *own) {
    __shared__ int32_t prev[64];
    for (int guard = 0; guard < 64 * 64; ++guard) {
        const int32_t c = active ? cnt[lane] : -1;
        int32_t top = c;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) top = max(top, __shfl_xor(top, o, 64));
        uint64_t tops = __ballot(active && c == top);
        bool moved = false;
        while (tops && !moved) {
            const int v = __ffsll((unsigned long long)tops) - 1;
            tops &= tops - 1;
            uint64_t visited = uint64_t(1) << v, frontier = visited;
            int found = -1;
            while (frontier && found < 0) {
                // each lane not yet reached finds the lowest particle of the
                // frontier that can pass it a pair
                int pu = -1;
                if (!((visited >> lane) & 1)) {
                    for (uint64_t f = frontier; f; f &= f - 1) {
                        const int u = __ffsll((unsigned long long)f) - 1;
                        if ((own[u] >> lane) & 1) {
                            pu = u;
                            break;
                        }
                    }
                }
                if (pu >= 0) prev[lane] = pu;
                const uint64_t disc = __ballot(pu >= 0);
                const uint64_t good = __ballot(pu >= 0 && c <= top - 2);
                if (good) found = __ffsll((unsigned long long)good) - 1;
                visited |= disc;
                frontier = disc;
            }
            if (found >= 0) {
                __syncthreads();
                if (lane == 0) {
                    for (int w = found; w != v;) {
                        const int u = prev[w];
                        own[u] &= ~(uint64_t(1) << w);
                        own[w] |= uint64_t(1) << u;
                        w = u;
                    }
                    --cnt[v];
                    ++cnt[found];
                }
                __syncthreads();
                moved = true;
            }
        }
        if (!moved) break;
    }
}

// Task lists of the tile transport (k_transport64_tile): particle i's
// neighbours outside its tile (kTile consecutive particles within its
// 64-particle column block of the neighbour table) and, flagged by the sign
// bit, the tile partners it evaluates for both.  Which of the two evaluates
// an in-tile pair is chosen to balance the lists, whose longest in each
// group of 16 particles (one wave of the transport) sets the
// iterations of a pass: one wave per tile starts from each particle's count
// of neighbours outside the tile and gives the tile's pairs, in a fixed order
// (by the lower index, then by its list order), one by one to the particle
// with the shorter list so far (the lower index on ties); level_tasks then
// lowers the tile's longest list.  On the 32^3 lattice the greedy pass takes
// the mean wave iterations of the transport to 0.75 of the two-sided
// kernel's (a fixed rule by index parity took them to 0.82 on the 64^3
// lattice) and the longest list of a tile, which sets its block's time, to
// 0.81; the leveling takes them to 0.70 and 0.69.  Same slots as the neighbour table, in table order; n_task[i]
// entries.  Launched with one wave (64 threads) per tile.
__global__ __launch_bounds__(64) void k_tasks(int64_t n, const int64_t *__restrict__ wave_base,
                                              const int32_t *__restrict__ n_nbr,
                                              const int32_t *__restrict__ nbr,
                                              int32_t *__restrict__ task,
                                              int32_t *__restrict__ n_task,
                                              int64_t *__restrict__ tstat) {
    __shared__ int32_t cnt[64];
    __shared__ uint64_t own[64];     // bit l of own[k]: particle k evaluates pair (k, l)
    const int lane = threadIdx.x;
    const int64_t t0 = (int64_t)blockIdx.x * 64, i = t0 + lane;
    const bool active = i < n;
    const int64_t base = wave_base[blockIdx.x] + lane;
    const int32_t nn = active ? n_nbr[i] : 0;
    int32_t out = 0;
    for (int32_t k = 0; k < nn; ++k)
        out += nbr[base + 64 * (int64_t)k] / kTile != (int32_t)(i / kTile);
    cnt[lane] = out;
    own[lane] = 0;
    __syncthreads();
    for (int src = 0; src < 64; ++src) {
        if (lane == src && active) {
            int32_t ci = cnt[src];
            uint64_t mine = 0;
            for (int32_t k = 0; k < nn; ++k) {
                const int32_t j = nbr[base + 64 * (int64_t)k];
                const int jl = j - (int32_t)t0;
                // outside the tile, or already given
                if (jl <= src || jl >= 64 || jl / kTile != src / kTile) continue;
                const int32_t cj = cnt[jl];
                if (cj < ci) {
                    cnt[jl] = cj + 1;
                    own[jl] |= uint64_t(1) << src;
                } else {
                    ++ci;
                    mine |= uint64_t(1) << jl;
                }
            }
            cnt[src] = ci;
            own[src] |= mine;
        }
        __syncthreads();
    }
    level_tasks(active, lane, cnt, own);
    {
        // the tile's longest list and its lower bound: the longest list of
        // neighbours outside the tile, or the mean length rounded up
        int32_t lm = active ? cnt[lane] : 0, om = out, sm = lm, na = active ? 1 : 0;
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lm = max(lm, __shfl_xor(lm, o, 64));
            om = max(om, __shfl_xor(om, o, 64));
            sm += __shfl_xor(sm, o, 64);
            na += __shfl_xor(na, o, 64);
        }
        if (lane == 0 && na > 0) {
            atomicAdd((unsigned long long *)&tstat[0], (unsigned long long)lm);
            atomicAdd((unsigned long long *)&tstat[1],
                      (unsigned long long)max(om, (sm + na - 1) / na));
        }
    }
    if (!active) return;
    const uint64_t mine = own[lane];
    int32_t c = 0;
    for (int32_t k = 0; k < nn; ++k) {
        int32_t j = nbr[base + 64 * (int64_t)k];
        const int jl = j - (int32_t)t0;
        if (jl >= 0 && jl < 64 && jl / kTile == lane / kTile) {
            if (!((mine >> jl) & 1)) continue;
            j |= int32_t(0x80000000u);
        }
        task[base + 64 * (int64_t)c] = j;
        ++c;
    }
    n_task[i] = c;
}

// Neighbour unions of the gradient (k_gradient64u, k_gradient32u; over the
// gather lists) and of the adjoint's transposed gradient (k_adj_grad64u; over
// the symmetric lists): for every block of 64 particles (a column block of the
// neighbour table) the sorted distinct indices of its particles and of the
// first len[i] neighbours of each, which the kernel stages in LDS once instead
// of fetching a neighbour's row for every pair (each row is used 6-8 times by
// a block).  Each of those slots gets the 16-bit position of its neighbour in
// the union (gloc), each particle its own (uown).  The distinct indices are collected in an LDS hash table (open
// addressing with bounded probing) and sorted (bitonic, kUnionSort keys).
// Count pass (FILL false): rows[b] = the union's size, or 0 if it does not
// fit `cap` (the block is left to the staged gradient); the fill pass writes
// the rows at uoff[b], gloc (packed, see rt_ctx) and uown.  One block of 256
// threads (4 per particle) per 64-particle block.
constexpr int kUnionHash = 4096;

template <bool FILL>
__global__ __launch_bounds__(256) void k_union(int64_t n, int cap,
                                               const int64_t *__restrict__ wave_base,
                                               const int32_t *__restrict__ len,
                                               const int32_t *__restrict__ nbr,
                                               int64_t *__restrict__ rows,
                                               const int64_t *__restrict__ uoff,
                                               int32_t *__restrict__ urow,
                                               const int64_t *__restrict__ goff,
                                               uint16_t *__restrict__ gloc,
                                               uint16_t *__restrict__ uown) {
    __shared__ int32_t keys[kUnionHash];
    __shared__ int32_t srt[kUnionSort];
    __shared__ int32_t cnt, fail;
    const int64_t b = blockIdx.x, t0 = b * 64;
    for (int e = threadIdx.x; e < kUnionHash; e += 256) keys[e] = -1;
    if (threadIdx.x == 0) {
        cnt = 0;
        fail = 0;
    }
    __syncthreads();
    const int p = threadIdx.x >> 2, sub = threadIdx.x & 3;
    const int64_t i = t0 + p;
    const bool active = i < n;
    const int64_t base = wave_base[b] + p;
    const int32_t ng = active ? len[i] : 0;
    auto insert = [&](int32_t j) {
        uint32_t h = ((uint32_t)j * 2654435761u) >> 20;     // 12 bits
        for (int probe = 0; probe < kUnionHash; ++probe) {
            const int32_t old = atomicCAS(&keys[h], -1, j);
            if (old == -1 || old == j) return;
            h = (h + 1) & (kUnionHash - 1);
        }
        atomicOr(&fail, 1);                                 // table full
    };
    if (active && sub == 0) insert((int32_t)i);
    for (int32_t k = sub; k < ng; k += 4) insert(nbr[base + 64 * (int64_t)k]);
    __syncthreads();
    // compact in any order (sorted next)
    for (int e = threadIdx.x; e < kUnionHash; e += 256) {
        const int32_t key = keys[e];
        if (key >= 0) {
            const int32_t pos = atomicAdd(&cnt, 1);
            if (pos < kUnionSort) srt[pos] = key;
        }
    }
    __syncthreads();
    const int32_t m = cnt;
    const bool fits = fail == 0 && m <= cap;                // block-uniform
    if (!FILL) {
        if (threadIdx.x == 0) rows[b] = fits ? m : 0;
        return;
    }
    if (!fits) return;
    for (int e = m + threadIdx.x; e < kUnionSort; e += 256) srt[e] = INT32_MAX;
    __syncthreads();
    for (int k = 2; k <= kUnionSort; k <<= 1)
        for (int jj = k >> 1; jj > 0; jj >>= 1) {
            for (int e = threadIdx.x; e < kUnionSort; e += 256) {
                const int l = e ^ jj;
                if (l > e) {
                    const int32_t a = srt[e], c = srt[l];
                    if ((a > c) == ((e & k) == 0)) {
                        srt[e] = c;
                        srt[l] = a;
                    }
                }
            }
            __syncthreads();
        }
    const int64_t u0 = uoff[b];
    for (int e = threadIdx.x; e < m; e += 256) urow[u0 + e] = srt[e];
    auto find = [&](int32_t j) {                            // j is in the union
        int lo = 0, hi = m - 1;
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (srt[mid] < j) lo = mid + 1;
            else hi = mid;
        }
        return (uint16_t)lo;
    };
    if (active && sub == 0) uown[i] = find((int32_t)i);
    uint16_t *g = gloc + goff[b] + 4 * (int64_t)threadIdx.x;   // lane 4p + sub
    for (int32_t k = sub; k < ng; k += 4)
        g[(int64_t)(k >> 4) * 1024 + ((k >> 2) & 3)] = find(nbr[base + 64 * (int64_t)k]);
}

inline unsigned nblk(int64_t n, int b = kBlock) { return (unsigned)((n + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
// host side

static void build_tree(rt_ctx *ctx, const double *H) {
    int64_t P = ctx->P;
    k_leaf_boxes<<<nblk(P), kBlock, 0, ctx->stream>>>(ctx->p.n, ctx->nleaf, P, ctx->xs, H,
                                                      ctx->node_lo, ctx->node_hi, ctx->node_hmax);
    for (int64_t first = P / 2; first >= 1; first /= 2)
        k_merge_level<<<nblk(first), kBlock, 0, ctx->stream>>>(first, first, ctx->node_lo,
                                                               ctx->node_hi, ctx->node_hmax);
}

// One set of neighbour unions (k_union) over the first len[i] entries of each
// particle's table column: sizes at capacity cap (w0 waves per SIMD), or at
// cap3 (3 waves) when cap3 > 0 and at least 95% of the blocks fit it.  Blocks
// over the capacity get no rows and are listed in *left.  The packed entries
// (nloc of them) go to the offsets ctx->goff, already on the device.
static rt_status build_union(rt_ctx *ctx, const int32_t *len, int cap, int w0, int cap3,
                             int64_t nloc, int64_t **off, int32_t **row, uint16_t **loc,
                             uint16_t **own, int32_t **left, int64_t *n_left, int *waves) {
    const int64_t n = ctx->p.n, nw = ctx->nwaves;
    hipStream_t st = ctx->stream;
    std::vector<int64_t> rows(nw + 1);
    int64_t *width = nullptr;
    rt_status rs = rt_alloc(ctx, (void **)&width, sizeof(int64_t) * (nw + 1));
    if (rs != RT_OK) return rs;
    k_union<false><<<(unsigned)nw, 256, 0, st>>>(n, cap, ctx->wave_base, len, ctx->nbr, width,
                                                 nullptr, nullptr, nullptr, nullptr, nullptr);
    hipError_t e = hipMemcpyAsync(rows.data(), width, sizeof(int64_t) * nw,
                                  hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    rt_free(ctx, width);
    if (e != hipSuccess) return rt_fail(ctx, RT_EHIP, hipGetErrorString(e));
    *waves = w0;
    if (cap3 > 0) {
        int64_t fit = 0;
        for (int64_t b = 0; b < nw; ++b) fit += rows[b] > 0 && rows[b] <= cap3;
        if (fit >= nw - nw / 20) {
            *waves = 3;
            cap = cap3;
            for (int64_t b = 0; b < nw; ++b)
                if (rows[b] > cap3) rows[b] = 0;
        }
    }
    // offsets (exclusive sums), and the blocks left out
    std::vector<int32_t> over;
    int64_t acc = 0;
    for (int64_t b = 0; b < nw; ++b) {
        const int64_t r = rows[b];
        rows[b] = acc;
        acc += r;
        if (r == 0) over.push_back((int32_t)b);
    }
    rows[nw] = acc;
    if ((rs = rt_alloc(ctx, (void **)off, sizeof(int64_t) * (nw + 1))) != RT_OK) return rs;
    RT_HIP(hipMemcpyAsync(*off, rows.data(), sizeof(int64_t) * (nw + 1), hipMemcpyHostToDevice, st));
    if ((rs = rt_alloc(ctx, (void **)row, sizeof(int32_t) * std::max<int64_t>(acc, 1))) != RT_OK)
        return rs;
    if ((rs = rt_alloc(ctx, (void **)loc, sizeof(uint16_t) * std::max<int64_t>(nloc, 4))) != RT_OK)
        return rs;
    if ((rs = rt_alloc(ctx, (void **)own, sizeof(uint16_t) * n)) != RT_OK) return rs;
    k_union<true><<<(unsigned)nw, 256, 0, st>>>(n, cap, ctx->wave_base, len, ctx->nbr, nullptr,
                                                *off, *row, ctx->goff, *loc, *own);
    *n_left = (int64_t)over.size();
    if (!over.empty()) {
        if ((rs = rt_alloc(ctx, (void **)left, sizeof(int32_t) * over.size())) != RT_OK) return rs;
        RT_HIP(hipMemcpyAsync(*left, over.data(), sizeof(int32_t) * over.size(),
                              hipMemcpyHostToDevice, st));
    }
    RT_HIP(hipStreamSynchronize(st));
    return RT_OK;
}

rt_status rt_build_impl(rt_ctx *ctx, const double *x, const double *h_in, int64_t *perm,
                        double *h, double *V, double *dt) {
    const int64_t n = ctx->p.n;
    hipStream_t st = ctx->stream;
    rt_status rs;
    // (re)allocate everything owned by a previous build
    rt_free(ctx, ctx->xs); rt_free(ctx, ctx->geo); rt_free(ctx, ctx->geo32); rt_free(ctx, ctx->perm32);
    rt_free(ctx, ctx->keys); rt_free(ctx, ctx->h_iters); rt_free(ctx, ctx->node_lo); rt_free(ctx, ctx->node_hi);
    rt_free(ctx, ctx->node_hmax); rt_free(ctx, ctx->n_nbr); rt_free(ctx, ctx->n_gath); rt_free(ctx, ctx->wave_base);
    rt_free(ctx, ctx->nbr); rt_free(ctx, ctx->vol); rt_free(ctx, ctx->ivan);
    rt_free(ctx, ctx->task); rt_free(ctx, ctx->n_task); rt_free(ctx, ctx->tstat);
    rt_free(ctx, ctx->uoff); rt_free(ctx, ctx->urow); rt_free(ctx, ctx->gloc);
    rt_free(ctx, ctx->uown); rt_free(ctx, ctx->ublk); rt_free(ctx, ctx->goff);
    rt_free(ctx, ctx->aoff); rt_free(ctx, ctx->arow); rt_free(ctx, ctx->agloc);
    rt_free(ctx, ctx->aown); rt_free(ctx, ctx->ablk);
    ctx->uoff = nullptr; ctx->urow = nullptr; ctx->gloc = nullptr; ctx->uown = nullptr;
    ctx->goff = nullptr;
    ctx->ublk = nullptr; ctx->n_ublk = 0;
    ctx->aoff = nullptr; ctx->arow = nullptr; ctx->agloc = nullptr; ctx->aown = nullptr;
    ctx->ablk = nullptr; ctx->n_ablk = 0;
    ctx->vol = nullptr;
    ctx->ivan = nullptr;
    ctx->task = nullptr;
    ctx->n_task = nullptr;
    ctx->tstat = nullptr;
    ctx->xs = nullptr; ctx->geo = nullptr; ctx->geo32 = nullptr; ctx->perm32 = nullptr;
    ctx->keys = nullptr; ctx->h_iters = nullptr; ctx->node_lo = nullptr; ctx->node_hi = nullptr;
    ctx->node_hmax = nullptr; ctx->n_nbr = nullptr; ctx->n_gath = nullptr;
    ctx->wave_base = nullptr; ctx->nbr = nullptr;
    ctx->built = 0;

    ctx->nleaf = (n + kLeaf - 1) / kLeaf;
    ctx->P = 1;
    while (ctx->P < ctx->nleaf) ctx->P *= 2;
    ctx->nwaves = (n + 63) / 64;

    uint64_t *keys_in = nullptr;
    int32_t *idx_in = nullptr;
    int32_t *nlist = nullptr;   // neighbours of the count pass (see k_neighbours)
    int ncap = 0;
    double *Htmp = nullptr, *dxpart = nullptr;
    int64_t *width = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_bytes = 0;

#define ALLOC(p, bytes)                                              \
    do {                                                             \
        if ((rs = rt_alloc(ctx, (void **)&(p), (bytes))) != RT_OK) goto fail; \
    } while (0)

    ALLOC(ctx->xs, sizeof(double) * 3 * n);
    ALLOC(ctx->geo, sizeof(double) * kRec * n);
    if (ctx->p.precision == RT_FP32C) ALLOC(ctx->geo32, sizeof(float) * F_REC * n);
    ALLOC(ctx->perm32, sizeof(int32_t) * n);
    ALLOC(ctx->keys, sizeof(uint64_t) * n);
    ALLOC(ctx->h_iters, sizeof(int32_t) * n);
    ALLOC(ctx->node_lo, sizeof(double) * 3 * 2 * ctx->P);
    ALLOC(ctx->node_hi, sizeof(double) * 3 * 2 * ctx->P);
    ALLOC(ctx->node_hmax, sizeof(double) * 2 * ctx->P);
    ALLOC(ctx->n_nbr, sizeof(int32_t) * n);
    ALLOC(ctx->n_gath, sizeof(int32_t) * n);
    ALLOC(ctx->wave_base, sizeof(int64_t) * (ctx->nwaves + 1));
    ALLOC(keys_in, sizeof(uint64_t) * n);
    ALLOC(idx_in, sizeof(int32_t) * n);
    ALLOC(Htmp, sizeof(double) * n);
    ALLOC(width, sizeof(int64_t) * (ctx->nwaves + 1));
    ALLOC(dxpart, sizeof(double) * nblk(n));

    {
        // Morton order
        k_morton<<<nblk(n), kBlock, 0, st>>>(n, x, 1.0 / ctx->p.box, keys_in, idx_in);
        if (rocprim::radix_sort_pairs(nullptr, sort_bytes, keys_in, ctx->keys, idx_in,
                                      ctx->perm32, (size_t)n, 0, 63, st) != hipSuccess) {
            rs = rt_fail(ctx, RT_EHIP, "radix sort size query failed");
            goto fail;
        }
        ALLOC(sort_tmp, sort_bytes);
        if (rocprim::radix_sort_pairs(sort_tmp, sort_bytes, keys_in, ctx->keys, idx_in,
                                      ctx->perm32, (size_t)n, 0, 63, st) != hipSuccess) {
            rs = rt_fail(ctx, RT_EHIP, "radix sort failed");
            goto fail;
        }
        k_gather_sorted<<<nblk(n), kBlock, 0, st>>>(n, x, ctx->perm32, h_in, ctx->xs, h, perm);

        // tree on positions; smoothing lengths
        build_tree(ctx, nullptr);
        Tree T{ctx->node_lo, ctx->node_hi, ctx->node_hmax, ctx->P};
        RT_HIP(hipMemsetAsync(ctx->status, 0, sizeof(int32_t), st));
        RT_HIP(hipMemsetAsync(ctx->h_iters, 0, sizeof(int32_t) * n, st));
        if (!h_in) {
            // candidate lists of kHList entries per particle while they fit in
            // kHListBytes (else every evaluation walks the tree)
            int cap = (int)std::min<int64_t>(kHList, kHListBytes / (8 * n));
            double *hlist = nullptr;
            if (cap < kHList / 2 || !rt_try_alloc(ctx, (void **)&hlist, sizeof(double) * cap * n)) {
                hlist = nullptr;
                cap = 0;
            }
            k_h_guess<<<nblk(n), kBlock, 0, st>>>(n, ctx->P, ctx->node_lo, ctx->node_hi,
                                                  ctx->xs, ctx->p.eta, ctx->p.box, h);
            k_h_solve<<<nblk(n), kBlock, 0, st>>>(n, T, ctx->xs, ctx->p.eta, ctx->p.kappa,
                                                  ctx->p.box, h, hlist, cap, ctx->h_iter_cap,
                                                  ctx->h_iters, ctx->status);
            if (hlist) {
                const hipError_t e = hipStreamSynchronize(st);
                rt_free(ctx, hlist);
                if (e != hipSuccess) {
                    rs = rt_fail(ctx, RT_EHIP, std::string("smoothing-length solve: ") + hipGetErrorString(e));
                    goto fail;
                }
            }
        }
        k_scale<<<nblk(n), kBlock, 0, st>>>(n, h, ctx->p.kappa, Htmp);
        int32_t stw = 0;
        RT_HIP(hipMemcpyAsync(&stw, ctx->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RT_HIP(hipStreamSynchronize(st));
        if (stw & ST_NOCONV) { rs = rt_fail(ctx, RT_ENOCONV, "smoothing length did not converge"); goto fail; }
        if (stw & ST_BIGH) { rs = rt_fail(ctx, RT_EINVAL, "compact support radius reaches half the box"); goto fail; }
        {
            // largest H must stay below half the box (nearest image is unique)
            std::vector<double> hmaxv(1);
            build_tree(ctx, Htmp);
            RT_HIP(hipMemcpyAsync(hmaxv.data(), ctx->node_hmax + 1, sizeof(double),
                                  hipMemcpyDeviceToHost, st));
            RT_HIP(hipStreamSynchronize(st));
            if (!(hmaxv[0] < 0.5 * ctx->p.box)) {
                rs = rt_fail(ctx, RT_EINVAL, "compact support radius reaches half the box");
                goto fail;
            }
        }
        // neighbour table: counts, wave widths, offsets, fill
        ncap = (int)std::min<int64_t>(kNList, kHListBytes / (4 * n));
        if (ncap < kNList / 2 || !rt_try_alloc(ctx, (void **)&nlist, sizeof(int32_t) * ncap * n)) {
            nlist = nullptr;
            ncap = 0;
        }
        k_neighbours<false><<<nblk(n), kBlock, 0, st>>>(n, T, ctx->xs, Htmp, ctx->p.box,
                                                        ctx->n_nbr, ctx->n_gath, nullptr, nullptr,
                                                        nlist, ncap);
        k_wave_width<<<nblk(ctx->nwaves + 1), kBlock, 0, st>>>(n, ctx->nwaves, ctx->n_nbr, width);
        size_t scan_bytes = 0;
        if (rocprim::exclusive_scan(nullptr, scan_bytes, width, ctx->wave_base,
                                    (int64_t)0, (size_t)(ctx->nwaves + 1),
                                    rocprim::plus<int64_t>(), st) != hipSuccess) {
            rs = rt_fail(ctx, RT_EHIP, "scan size query failed");
            goto fail;
        }
        if (scan_bytes > sort_bytes) {
            rt_free(ctx, sort_tmp);
            sort_tmp = nullptr;
            ALLOC(sort_tmp, scan_bytes);
            sort_bytes = scan_bytes;
        }
        if (rocprim::exclusive_scan(sort_tmp, scan_bytes, width, ctx->wave_base, (int64_t)0,
                                    (size_t)(ctx->nwaves + 1), rocprim::plus<int64_t>(),
                                    st) != hipSuccess) {
            rs = rt_fail(ctx, RT_EHIP, "scan failed");
            goto fail;
        }
        RT_HIP(hipMemcpyAsync(&ctx->slots, ctx->wave_base + ctx->nwaves, sizeof(int64_t),
                              hipMemcpyDeviceToHost, st));
        RT_HIP(hipStreamSynchronize(st));
        ALLOC(ctx->nbr, sizeof(int32_t) * std::max<int64_t>(ctx->slots, 1));
        RT_HIP(hipMemsetAsync(ctx->nbr, 0xff, sizeof(int32_t) * std::max<int64_t>(ctx->slots, 1), st));
        k_neighbours<true><<<nblk(n), kBlock, 0, st>>>(n, T, ctx->xs, Htmp, ctx->p.box,
                                                       ctx->n_nbr, ctx->n_gath, ctx->wave_base,
                                                       ctx->nbr, nlist, ncap);
        {
            // task lists of the tile transports
            ALLOC(ctx->task, sizeof(int32_t) * std::max<int64_t>(ctx->slots, 1));
            ALLOC(ctx->n_task, sizeof(int32_t) * n);
            ALLOC(ctx->tstat, 2 * sizeof(int64_t));
            RT_HIP(hipMemsetAsync(ctx->tstat, 0, 2 * sizeof(int64_t), st));
            k_tasks<<<(unsigned)ctx->nwaves, 64, 0, st>>>(n, ctx->wave_base, ctx->n_nbr, ctx->nbr,
                                                          ctx->task, ctx->n_task, ctx->tstat);
        }
        {
            // neighbour unions of the gradient (gather lists): FP64 at the
            // 2-wave capacity, then 3 waves per SIMD if nearly every block
            // fits that capacity; FP32C at its 3-wave capacity.  FP64 also
            // builds those of the adjoint's transposed gradient (the
            // symmetric lists), which stages one group at a time.
            const bool f64 = ctx->p.precision == RT_FP64;
            const int G = ctx->p.groups;
            const int cap = f64 ? union_cap(G) : union_cap32(G);
            if (cap > 0) {
                const int64_t nw = ctx->nwaves;
                // packed table entries: 1024 per group of 16 table rows of a block
                std::vector<int64_t> wb(nw + 1), go(nw + 1);
                RT_HIP(hipMemcpyAsync(wb.data(), ctx->wave_base, sizeof(int64_t) * (nw + 1),
                                      hipMemcpyDeviceToHost, st));
                RT_HIP(hipStreamSynchronize(st));
                go[0] = 0;
                for (int64_t b = 0; b < nw; ++b)
                    go[b + 1] = go[b] + 1024 * (((wb[b + 1] - wb[b]) / 64 + 15) / 16);
                ALLOC(ctx->goff, sizeof(int64_t) * (nw + 1));
                RT_HIP(hipMemcpyAsync(ctx->goff, go.data(), sizeof(int64_t) * (nw + 1),
                                      hipMemcpyHostToDevice, st));
                rs = build_union(ctx, ctx->n_gath, cap, f64 ? 2 : 3, f64 ? union_cap3(G) : 0,
                                 go[nw], &ctx->uoff, &ctx->urow, &ctx->gloc, &ctx->uown,
                                 &ctx->ublk, &ctx->n_ublk, &ctx->union_waves);
                if (rs != RT_OK) goto fail;
                if (f64) {
                    rs = build_union(ctx, ctx->n_nbr, adj_union_cap(2), 2, adj_union_cap(3), go[nw],
                                     &ctx->aoff, &ctx->arow, &ctx->agloc, &ctx->aown, &ctx->ablk,
                                     &ctx->n_ablk, &ctx->adj_union_waves);
                    if (rs != RT_OK) goto fail;
                }
            }
        }
        // geometry records, volumes, time step
        RT_HIP(hipMemsetAsync(ctx->status, 0, sizeof(int32_t), st));
        k_geometry<<<nblk(n), kBlock, 0, st>>>(n, ctx->xs, h, ctx->p.kappa, ctx->p.box,
                                               ctx->n_gath, ctx->wave_base, ctx->nbr, ctx->geo,
                                               ctx->geo32, V, dxpart, ctx->status);
        k_dt<<<1, kBlock, 0, st>>>(nblk(n), dxpart, ctx->p.cfl, ctx->p.c_red, ctx->dt_dev);
        if (dt) k_copy_dt<<<1, 1, 0, st>>>(ctx->dt_dev, dt);
        RT_HIP(hipGetLastError());
        // statistics
        std::vector<int32_t> nn(n), ng(n), it(n);
        RT_HIP(hipMemcpyAsync(nn.data(), ctx->n_nbr, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        RT_HIP(hipMemcpyAsync(ng.data(), ctx->n_gath, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        RT_HIP(hipMemcpyAsync(it.data(), ctx->h_iters, sizeof(int32_t) * n, hipMemcpyDeviceToHost, st));
        RT_HIP(hipMemcpyAsync(&stw, ctx->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RT_HIP(hipStreamSynchronize(st));
        if (stw & ST_SINGULAR) {
            rs = rt_fail(ctx, RT_ESINGULAR, "E_i not positive definite (coplanar or too few neighbours)");
            goto fail;
        }
        ctx->n_entries = 0;
        ctx->n_gather_entries = 0;
        ctx->max_nbr = 0;
        ctx->h_iter_max = 0;
        ctx->h_list_overflow = 0;
        for (int64_t i = 0; i < n; ++i) {
            ctx->n_entries += nn[i];
            ctx->n_gather_entries += ng[i];
            ctx->max_nbr = std::max(ctx->max_nbr, nn[i]);
            ctx->h_iter_max = std::max(ctx->h_iter_max, it[i] & (kIterOverflow - 1));
            ctx->h_list_overflow += (it[i] & kIterOverflow) ? 1 : 0;
        }
    }
    rt_free(ctx, keys_in); rt_free(ctx, idx_in); rt_free(ctx, Htmp); rt_free(ctx, width); rt_free(ctx, dxpart);
    rt_free(ctx, sort_tmp); rt_free(ctx, nlist);
    if ((rs = rt_ensure_partials(ctx)) != RT_OK) return rs;
    // compact copy of the volumes for the per-particle kernels that need
    // nothing else of the geometry record
    if ((rs = rt_alloc(ctx, (void **)&ctx->vol, sizeof(double) * n)) != RT_OK) return rs;
    RT_HIP(hipMemcpyAsync(ctx->vol, V, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    ctx->built = 1;
    if (ctx->surfaces == RT_IVANOVA && (rs = rt_ivanova_impl(ctx)) != RT_OK) return rs;
    ctx->bin_top = -1;   // the records were rewritten with all time bins 0
    if (ctx->bin8) RT_HIP(hipMemsetAsync(ctx->bin8, 0, 2 * (size_t)n, st));
    return RT_OK;
fail:
    // the conditions of the build are reported by its return code, not by a
    // later rt_sync
    (void)hipMemsetAsync(ctx->status, 0, sizeof(int32_t), st);
    (void)hipStreamSynchronize(st);
    rt_free(ctx, keys_in); rt_free(ctx, idx_in); rt_free(ctx, Htmp); rt_free(ctx, width); rt_free(ctx, dxpart);
    rt_free(ctx, sort_tmp); rt_free(ctx, nlist);
    return rs;
#undef ALLOC
}

rt_status rt_sources_impl(rt_ctx *ctx, int32_t S, const double *xs, double eta_star) {
    hipStream_t st = ctx->stream;
    rt_free(ctx, ctx->src_h); rt_free(ctx, ctx->inj_gptr); rt_free(ctx, ctx->inj_gas); rt_free(ctx, ctx->inj_src);
    rt_free(ctx, ctx->inj_coef); rt_free(ctx, ctx->inj_xi); rt_free(ctx, ctx->src_ptr); rt_free(ctx, ctx->src_gas);
    rt_free(ctx, ctx->src_coef);
    ctx->src_h = nullptr; ctx->inj_gptr = nullptr; ctx->inj_gas = nullptr; ctx->inj_src = nullptr;
    ctx->inj_coef = nullptr; ctx->inj_xi = nullptr; ctx->src_ptr = nullptr; ctx->src_gas = nullptr;
    ctx->src_coef = nullptr;
    ctx->S = 0;
    ctx->n_inj = 0;
    ctx->n_inj_gas = 0;
    if (S == 0) return RT_OK;
    const int64_t n = ctx->p.n;
    rt_status rs;
    double *sx = nullptr, *sxi = nullptr;
    int32_t *cnt = nullptr;
    std::vector<int32_t> hc(S), hptr(S + 1);
    Tree T{ctx->node_lo, ctx->node_hi, ctx->node_hmax, ctx->P};
    if ((rs = rt_alloc(ctx, (void **)&sx, sizeof(double) * 3 * S)) != RT_OK) return rs;
    if ((rs = rt_alloc(ctx, (void **)&ctx->src_h, sizeof(double) * S)) != RT_OK) goto fail;
    if ((rs = rt_alloc(ctx, (void **)&cnt, sizeof(int32_t) * S)) != RT_OK) goto fail;
    RT_HIP(hipMemcpyAsync(sx, xs, sizeof(double) * 3 * S, hipMemcpyDeviceToDevice, st));
    RT_HIP(hipMemsetAsync(ctx->status, 0, sizeof(int32_t), st));
    {
        // start below the mean spacing; the solver doubles h until bracketed
        double h0 = 0.05 * eta_star * ctx->p.box / cbrt((double)n);
        k_src_h<<<nblk(S, 64), 64, 0, st>>>(S, T, ctx->xs, n, sx, eta_star, ctx->p.kappa,
                                           ctx->p.box, h0, ctx->h_iter_cap, ctx->src_h,
                                           ctx->status);
        k_src_gas<false><<<nblk(S, 64), 64, 0, st>>>(S, T, ctx->xs, n, sx, ctx->src_h,
                                                    ctx->p.kappa, ctx->p.box, ctx->geo, cnt,
                                                    nullptr, nullptr, nullptr, nullptr);
        int32_t stw = 0;
        RT_HIP(hipMemcpyAsync(hc.data(), cnt, sizeof(int32_t) * S, hipMemcpyDeviceToHost, st));
        RT_HIP(hipMemcpyAsync(&stw, ctx->status, sizeof(int32_t), hipMemcpyDeviceToHost, st));
        RT_HIP(hipStreamSynchronize(st));
        if (stw & ST_NOCONV) { rs = rt_fail(ctx, RT_ENOCONV, "source smoothing length did not converge"); goto fail; }
        if (stw & ST_BIGH) { rs = rt_fail(ctx, RT_EINVAL, "source compact support reaches half the box"); goto fail; }
        hptr[0] = 0;
        for (int32_t s = 0; s < S; ++s) {
            if (hc[s] == 0) { rs = rt_fail(ctx, RT_EINVAL, "source without gas neighbours"); goto fail; }
            hptr[s + 1] = hptr[s] + hc[s];
        }
        const int64_t m = hptr[S];
        if ((rs = rt_alloc(ctx, (void **)&ctx->src_ptr, sizeof(int32_t) * (S + 1))) != RT_OK) goto fail;
        if ((rs = rt_alloc(ctx, (void **)&ctx->src_gas, sizeof(int32_t) * m)) != RT_OK) goto fail;
        if ((rs = rt_alloc(ctx, (void **)&ctx->src_coef, sizeof(double) * m)) != RT_OK) goto fail;
        if ((rs = rt_alloc(ctx, (void **)&sxi, sizeof(double) * m)) != RT_OK) goto fail;
        RT_HIP(hipMemcpyAsync(ctx->src_ptr, hptr.data(), sizeof(int32_t) * (S + 1),
                              hipMemcpyHostToDevice, st));
        k_src_gas<true><<<nblk(S, 64), 64, 0, st>>>(S, T, ctx->xs, n, sx, ctx->src_h, ctx->p.kappa,
                                                   ctx->p.box, ctx->geo, nullptr, ctx->src_ptr,
                                                   ctx->src_gas, sxi, ctx->src_coef);
        // gas-major copy for the per-step injection (deterministic gather)
        std::vector<int32_t> g(m), srcv(m);
        std::vector<double> xi(m), co(m);
        RT_HIP(hipMemcpyAsync(g.data(), ctx->src_gas, sizeof(int32_t) * m, hipMemcpyDeviceToHost, st));
        RT_HIP(hipMemcpyAsync(xi.data(), sxi, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        RT_HIP(hipMemcpyAsync(co.data(), ctx->src_coef, sizeof(double) * m, hipMemcpyDeviceToHost, st));
        RT_HIP(hipStreamSynchronize(st));
        for (int32_t s = 0; s < S; ++s)
            for (int32_t e = hptr[s]; e < hptr[s + 1]; ++e) srcv[e] = s;
        std::vector<int64_t> ord(m);
        std::iota(ord.begin(), ord.end(), 0);
        std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return g[a] < g[b]; });
        std::vector<int32_t> ig, igp, isr(m);
        std::vector<double> ico(m), ixi(m);
        for (int64_t e = 0; e < m; ++e) {
            int64_t o = ord[e];
            if (e == 0 || g[o] != g[ord[e - 1]]) {
                ig.push_back(g[o]);
                igp.push_back((int32_t)e);
            }
            isr[e] = srcv[o];
            ico[e] = co[o];
            ixi[e] = xi[o];
        }
        igp.push_back((int32_t)m);
        ctx->n_inj = m;
        ctx->n_inj_gas = (int32_t)ig.size();
        if ((rs = rt_alloc(ctx, (void **)&ctx->inj_gptr, sizeof(int32_t) * igp.size())) != RT_OK) goto fail;
        if ((rs = rt_alloc(ctx, (void **)&ctx->inj_gas, sizeof(int32_t) * ig.size())) != RT_OK) goto fail;
        if ((rs = rt_alloc(ctx, (void **)&ctx->inj_src, sizeof(int32_t) * m)) != RT_OK) goto fail;
        if ((rs = rt_alloc(ctx, (void **)&ctx->inj_coef, sizeof(double) * m)) != RT_OK) goto fail;
        if ((rs = rt_alloc(ctx, (void **)&ctx->inj_xi, sizeof(double) * m)) != RT_OK) goto fail;
        RT_HIP(hipMemcpyAsync(ctx->inj_gptr, igp.data(), sizeof(int32_t) * igp.size(), hipMemcpyHostToDevice, st));
        RT_HIP(hipMemcpyAsync(ctx->inj_gas, ig.data(), sizeof(int32_t) * ig.size(), hipMemcpyHostToDevice, st));
        RT_HIP(hipMemcpyAsync(ctx->inj_src, isr.data(), sizeof(int32_t) * m, hipMemcpyHostToDevice, st));
        RT_HIP(hipMemcpyAsync(ctx->inj_coef, ico.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
        RT_HIP(hipMemcpyAsync(ctx->inj_xi, ixi.data(), sizeof(double) * m, hipMemcpyHostToDevice, st));
        RT_HIP(hipStreamSynchronize(st));
    }
    ctx->S = S;
    rt_free(ctx, sx); rt_free(ctx, cnt); rt_free(ctx, sxi);
    return RT_OK;
fail:
    (void)hipMemsetAsync(ctx->status, 0, sizeof(int32_t), st);
    (void)hipStreamSynchronize(st);
    rt_free(ctx, sx); rt_free(ctx, cnt); rt_free(ctx, sxi);
    return rs;
}
