/*
 * rt.h -- C ABI of the MI355X (gfx950) photon-transport library.
 *
 * The library implements the transport step of Gear-RT, the particle-based
 * moment (M1) radiative transfer scheme of arXiv:2302.12727, Part III
 * ("Numerical solution strategy", sections "First step: injection" and
 * "Second step: transport"), on the finite volume particle method of Part II
 * (Hopkins formulation).  Particles are static interpolation points
 * (Part III, "Using a particle based method: selecting reference frames"), so
 * neighbour search and geometry are built once and reused by every step.
 *
 * Conventions shared by every entry point
 *  - All array pointers are DEVICE pointers (HIP, gfx950) allocated and freed
 *    by the caller, unless marked [host].  The library keeps no pointer to
 *    caller memory across calls.
 *  - Work is enqueued asynchronously on the context's HIP stream; nothing
 *    synchronises the host except rt_create, rt_build_cells, rt_set_sources,
 *    the rt_get_* queries and rt_sync.
 *  - Particle arrays (state, gradients, smoothing lengths, volumes) are in the
 *    library's Morton order once rt_build_cells has run: position i of those
 *    arrays is input particle perm[i].
 *  - The state U of one particle is G photon groups x (E, Fx, Fy, Fz), i.e.
 *    U[n][G][4].  The element type is double for RT_FP64 and float for
 *    RT_FP32C.
 *  - The gradient record UD[n][G][16] holds per particle and group the state
 *    followed by the gradient of each of its components:
 *    UD[i][g][0..4) = U[i][g][0..4) and UD[i][g][4 + 3 m + a] = d U[i][g][m] / d x_a.
 *    One group of one particle is one 128-byte line in FP64, so a neighbour's
 *    data is fetched in whole cache lines.
 *  - Errors: argument checks fail synchronously with RT_EINVAL and a message
 *    (rt_last_error).  rt_build_cells and rt_set_sources report their own
 *    device conditions (smoothing length not converged, singular E matrix)
 *    in their return code.  The per-step kernels raise a bit of a device
 *    status word instead: rt_gradient when a gradient record it writes holds
 *    a NaN or an infinity (a non-finite input state), rt_transport and rt_tick
 *    when an updated state does (before the post-update guard, which does not
 *    catch NaN).  The next rt_sync turns the word into its return code and
 *    clears it; the arrays are written all the same.
 *  - One context per stream; calls on a context are not re-entrant.
 */
#ifndef GEARRT_RT_H
#define GEARRT_RT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rt_ctx rt_ctx;

typedef enum {
    RT_OK = 0,
    RT_EINVAL = -1,     /* bad argument (message in rt_last_error)           */
    RT_ENOMEM = -2,     /* device allocation failed                          */
    RT_EHIP = -3,       /* HIP runtime error                                 */
    RT_ENOCONV = -4,    /* smoothing length iteration did not converge       */
    RT_ESINGULAR = -5,  /* E_i not positive definite (coplanar neighbours)   */
    RT_ESTATE = -6,     /* call out of order (e.g. step before build)        */
    RT_ENONFINITE = -7  /* a state or gradient left the finite range (NaN/inf) */
} rt_status;

typedef enum { RT_FP64 = 0, RT_FP32C = 1 } rt_precision;

/* Guard counters, accumulated by rt_transport (see there). */
enum { RT_CNT_FACE_E = 0, RT_CNT_FACE_F = 1, RT_CNT_CELL_E = 2, RT_CNT_CELL_F = 3,
       RT_NCOUNTS = 4 };

typedef struct {
    int64_t n;          /* particles, 1 .. 2^28                                  */
    int32_t groups;     /* photon groups G, 1 .. 8                               */
    int32_t precision;  /* rt_precision                                          */
    double box;         /* side of the periodic cube [0, box)^3                  */
    double eta;         /* resolution parameter eta_res (default 1.2348)         */
    double kappa;       /* compact support over smoothing length H/h (1.825742)  */
    double c_red;       /* (reduced) speed of light                              */
    double cfl;         /* Courant number of the global time step                */
    void *hip_stream;   /* hipStream_t the context enqueues on (NULL: default)   */
} rt_params;

/* Create a context for n particles.  [host] p, out.  Validates p (RT_EINVAL
 * with a message through *out when p is invalid, *out may then be NULL).
 * No device memory is touched before the arguments are validated. */
rt_status rt_create(const rt_params *p, rt_ctx **out);
void rt_destroy(rt_ctx *ctx);
/* Last error message of ctx (or of the last failed rt_create when ctx is NULL). */
const char *rt_last_error(const rt_ctx *ctx);
/* Rebind the stream the context enqueues on. */
rt_status rt_set_stream(rt_ctx *ctx, void *hip_stream);

/* Static geometry (Part II "Partition of unity", "Neighbor search",
 * "Finite volume particle methods following Hopkins"; Part III eq:rt-cfl).
 *   x    [n][3] positions in [0, box), input order.
 *   h_in [n] smoothing lengths in input order, or NULL to solve
 *        h^3 sum_j W(r_ij, kappa h) = eta^3 for every particle
 *        (eq:number-of-neighbors, Newton-Raphson with bisection).
 *   perm [n] out: perm[i] = input index of Morton-ordered particle i.
 *   h    [n] out (Morton order); V [n] out: V_i = 1/omega(x_i)
 *        (eq:particle-volume);  dt [1] out: C_cfl min_i dx_i / c with
 *        dx_i = (3 V_i / 4 pi)^{1/3}.
 * Builds Morton order, the search tree, the neighbour lists
 * {j : r_ij < max(H_i, H_j)} and per particle V_i and B_i = E_i^{-1}
 * (eq:matrix_E, eq:matrix_B, inverted in FP64).  Synchronises the stream.
 * Errors: RT_ENOCONV, RT_ESINGULAR, RT_EINVAL (compact support >= box/2). */
rt_status rt_build_cells(rt_ctx *ctx, const double *x, const double *h_in,
                         int64_t *perm, double *h, double *V, double *dt);

/* Iteration cap of the smoothing-length solve of rt_build_cells and
 * rt_set_sources (Part II "The neighbor search: determining the smoothing
 * length"; the thesis fixes no tolerance or cap).  A particle whose
 * Newton-Raphson/bisection iteration has not met the 4-ulp step test after
 * max_iter evaluations makes the build return RT_ENOCONV.  Default 200
 * (a C-level model of the iteration needs at most 8 on the synthetic sets);
 * 1 .. 10000, else RT_EINVAL.  Applies to later builds. */
rt_status rt_set_h_iterations(rt_ctx *ctx, int32_t max_iter);

/* Point sources (Part III "First step: injection", "Weights for distribution
 * of energy density of a star onto particles").  xs [S][3] device positions.
 * Solves each source's smoothing length over the gas with eta_star, then the
 * weights xi_sg = mu_a psi(x_s - x_g, h_s) with the octant correction
 * eq:isotropy-correction-with-zero.  S = 0 removes all sources.  Synchronises. */
rt_status rt_set_sources(rt_ctx *ctx, int32_t n_src, const double *xs, double eta_star);

/* Injection, in place on U (first operator of the RT step):
 *   E_g += dt * sum_s xi_sg L_s / V_g   for every group, no flux injected.
 * L [S][G] luminosities (double in both precisions), dt [1] device. */
rt_status rt_inject(rt_ctx *ctx, void *U, const double *L, const double *dt);

/* Least-squares gradients (eq:gradient) of every component of U:
 *   dU_i = sum_{j: r_ij < H_i} (U_j - U_i) psi_tilde_j(x_i).
 * U [n][G][4] in; UD [n][G][16] out (state and gradients, see above).
 * U and UD must not overlap and must be 16-byte aligned (RT_EINVAL
 * otherwise): the neighbours' states are moved in 16-byte pieces. */
rt_status rt_gradient(rt_ctx *ctx, const void *U, void *UD);

/* One transport step (eq:transport-update-explicit with one global dt):
 *   U_out_k = U_k - dt/V_k sum_l Flux_kl . A_kl
 * over all neighbours l, with A_kl of eq:HopkinsAij, the GLF solver of
 * eq:riemann-GLF (or HLL, see rt_set_riemann) on minmod-limited states
 * extrapolated to
 * x_kl = x_k + h_k/(h_k + h_l)(x_l - x_k) (eq:rt-riemann-problem), and the M1
 * closure (eq:eddington-group).  Face states and the updated state are
 * guarded: E < 0 is set to 0 (with F = 0) and |F| > c E is scaled to c E.
 *   UD        in: gradient record of the state, written by rt_gradient.
 *   U_out     [n][G][4] out, must not overlap UD.
 *   dt        [1] device.
 *   photon_total [G] out or NULL: Q_g = sum_k V_k E_kg of U_out (FP64,
 *             compensated, deterministic).
 *   counts    [RT_NCOUNTS] int64, accumulated, or NULL: face states with E
 *             clipped / F rescaled (each directed neighbour entry counts both
 *             faces), updated states with E clipped / F rescaled.
 *   ledger    [G] accumulated or NULL: sum_k V_k (energy density added by
 *             clipping E < 0 of the updated state).
 *   U_unguarded [n][G][4] out or NULL: the updated state before the
 *             post-update guard (consumed by rt_adjoint). */
rt_status rt_transport(rt_ctx *ctx, const void *UD, const double *dt, void *U_out,
                       double *photon_total, int64_t *counts, double *ledger,
                       void *U_unguarded);

/* Q_g = sum_k V_k E_kg of U, [G] out (FP64, compensated, deterministic). */
rt_status rt_photon_total(rt_ctx *ctx, const void *U, double *Q);

/* Riemann solver of rt_transport (Part III "Riemann solvers").
 *   RT_GLF  global Lax-Friedrichs, eq:riemann-GLF (the default).
 *   RT_HLL  HLL, eq:riemann-HLL:
 *             Phi = (l+ F_L - l- F_R + l+ l- (U_R - U_L)) / (l+ - l-),
 *             l+ = max(0, l_max), l- = min(0, l_min),
 *           l_max the larger and l_min the smaller of the extreme eigenvalues
 *           of the M1 flux Jacobian along the face normal A/|A| over the two
 *           face states; (F_L + F_R)/2 when l+ = l- = 0.  The eigenvalues
 *           depend on f = |F|/(cE) (clamped to 1) and mu = F.A/(|F||A|) only;
 *           the library tabulates them in units of c on RT_HLL_NF nodes
 *           uniform in f on [0, 1] times RT_HLL_NMU nodes uniform in mu on
 *           [-1, 1] and interpolates bilinearly (a state with E <= 0 or F = 0
 *           is looked up at f = 0).
 * HLL is implemented in rt_transport (FP64 and FP32C, the FP32C kernel
 * interpolating an FP32 copy of the table), in rt_tick and in rt_adjoint
 * (FP64 and FP32C: the derivative of the interpolated speeds, with the branch
 * the forward takes at the max/min of the speeds, the clamps of f and mu and
 * the table cells).  The table (RT_HLL_NF x RT_HLL_NMU
 * x 2 doubles) is computed on the host and uploaded on the first selection of
 * RT_HLL (synchronous). */
typedef enum { RT_GLF = 0, RT_HLL = 1 } rt_riemann;
#define RT_HLL_NF 65
#define RT_HLL_NMU 65
rt_status rt_set_riemann(rt_ctx *ctx, int32_t solver);

/* Effective surfaces A_kl of the transport (Part II).
 *   RT_HOPKINS  eq:HopkinsAij, A_kl = V_k psi~_l(x_k) - V_l psi~_k(x_l) with the
 *               least-squares psi~ (the default).
 *   RT_IVANOVA  eq:IvanovaAij, A_kl = V_k grad psi_l(x_k) - V_l grad psi_k(x_l)
 *               with the analytic gradients of the partition of unity,
 *               grad psi_l(x_k) = V_k grad W_l(x_k) - V_k^2 W(r_kl, H_k) g_k,
 *               g_k = sum_m grad W_m(x_k) over the gather neighbours, the kernel
 *               taken with H_k (the thesis' appendix on partition-of-unity
 *               gradients).
 * After rt_build_cells (RT_ESTATE before), FP64 and FP32C contexts (the
 * FP32C kernel forms A in FP32 from g rounded to FP32); selecting RT_IVANOVA
 * computes g (n x 4 doubles, kept and recomputed by
 * later builds).  rt_transport, rt_tick and rt_adjoint take either surfaces
 * (rt_adjoint differentiates the step with them held static).  The gradient
 * step (eq:gradient) is the same for both. */
typedef enum { RT_HOPKINS = 0, RT_IVANOVA = 1 } rt_surfaces;
rt_status rt_set_surfaces(rt_ctx *ctx, int32_t kind);

/* The HLL wave-speed table, [RT_HLL_NF][RT_HLL_NMU][2] doubles (l_min, l_max)
 * in units of c at f_i = i/(RT_HLL_NF - 1), mu_j = -1 + 2j/(RT_HLL_NMU - 1).
 *   tab [host] out.  ctx may be NULL (host code only, no device needed). */
rt_status rt_get_hll_table(rt_ctx *ctx, double *tab);

/* Photo-absorption constants of photon groups (Part III "Discretization of
 * Frequencies": eq:sigma_N and the energy-weighted average beside it, and the
 * mean photon energy), for cross sections of H0, He0 and He+ from the fits
 * eq:sigma-parametrizaiton with the parameters of tab:cross-sections (zero
 * below each species' ionization energy, eq:nuIonHI - eq:nuIonHeII) and a
 * blackbody spectrum eq:blackbody.  Host code: needs no context or device.
 *   G         groups, 1 .. 64.
 *   edges_eV  [G + 1] [host] increasing group edges in eV, edges_eV[0] > 0;
 *             edges_eV[G] may be +infinity.
 *   T_bb      blackbody temperature in K, > 0.
 *   sigma_N, sigma_E [G][3] [host] out: number- and energy-weighted group
 *             cross sections in cm^2, species H0, He0, He+.
 *   eps       [G] [host] out: mean photon energy of each group in erg.
 *   frac      [G] [host] out or NULL: the fraction of the photons above
 *             edges_eV[0] in each group (a source of Ndot photons/s above
 *             edges_eV[0] has group luminosities eps_i frac_i Ndot).
 * Errors: RT_EINVAL (edges, temperature, a group without photons). */
rt_status rt_photon_groups(int32_t G, const double *edges_eV, double T_bb, double *sigma_N,
                           double *sigma_E, double *eps, double *frac);

/* Photon removal of the thermochemistry step (Part III "Third step:
 * Thermochemistry"), in place on U: forward Euler over dt with the number
 * densities of the absorbing species averaged over the step,
 *   U_kg <- U_kg max(0, 1 - c dt sum_j sigma_gj (n_old_kj + n_new_kj)/2)
 * for E and F alike, c = c_red of the context.  A factor below zero (more
 * photons absorbed than present) is clamped to zero.
 *   U       [n][G][4] in/out, the context's state type.
 *   J       absorbing species, 1 .. 8.
 *   n_old   [n][J] double, densities at the start of the step (Morton order).
 *   n_new   [n][J] double or NULL (constant densities): at the end of the step.
 *   sigma   [G][J] double: group cross sections, in units consistent with n,
 *           c and dt (e.g. sigma_N of rt_photon_groups, rescaled).
 *   dt      [1] device.
 *   photon_total [G] out or NULL: Q_g of the updated U.
 *   absorbed [G] accumulated or NULL: sum_k V_k (E_kg before - E_kg after).
 * n_old, n_new and sigma must not overlap U. */
rt_status rt_absorb(rt_ctx *ctx, void *U, int32_t J, const double *n_old, const double *n_new,
                    const double *sigma, const double *dt, double *photon_total,
                    double *absorbed);

/* Drift correction (Part III "Dealing With Particle Drifts"): the state of a
 * particle moved by dx_i (its velocity times the drift time) is extrapolated
 * with its own gradients,
 *   U_out_i = U_i + grad U_i . dx_i     for every group and component,
 * then guarded as rt_transport guards the updated state (E < 0 -> 0 with
 * F = 0, |F| > cE -> scaled to cE).  Not conservative, as the thesis notes.
 * The geometry stays where it was: rebuild it with rt_build_cells at the new
 * positions before the next gradient or transport.
 *   UD      [n][G][16] in: gradient record of the state (rt_gradient),
 *           16-byte aligned.
 *   dx      [n][3] double: displacements (Morton order).
 *   U_out   [n][G][4] out, must not overlap UD or dx.
 *   photon_total [G] out or NULL: Q_g of U_out.
 *   counts  [RT_NCOUNTS] accumulated or NULL: moved states with E clipped
 *           (slot RT_CNT_CELL_E) or F rescaled (RT_CNT_CELL_F).
 *   ledger  [G] accumulated or NULL: sum_k V_k (energy added by the E clip). */
rt_status rt_drift(rt_ctx *ctx, const void *UD, const double *dx, void *U_out,
                   double *photon_total, int64_t *counts, double *ledger);

/* Individual power-of-two time steps (Part II "Individual time steps",
 * eq:meshless-explicit-individual-timesteps; Part III eq:transport-update-
 * explicit with min{dt_k, dt_l}; the factor-4 limiter of Part III "Dynamic
 * Sub-Cycling").  FP64 and FP32C contexts.
 *
 * rt_time_bins: particle i gets dt_i = dt 2^b_i, dt the step rt_build_cells
 * returned (the smallest CFL step), b_i the largest n <= max_bin (0 .. 30)
 * with dt 2^n <= C_cfl dx_i / c, then lowered until every interacting pair is
 * at most 2 bins apart.  The bins are kept in the context (all 0 after
 * rt_build_cells: the global step).
 *   bins        [n] int32 out (Morton order) or NULL.
 *   cycle_ticks [host] out or NULL: 2^max_i b_i, the ticks after which every
 *               particle has ended a step at the same time.
 * Synchronous (returns when the bins are set). */
rt_status rt_time_bins(rt_ctx *ctx, int32_t max_bin, int32_t *bins, int64_t *cycle_ticks);

/* One tick t (t = 0, 1, ...) of the individual-time-step scheme: the time
 * advances by dt; particle i ends a step at the end of tick t when (t + 1) is a
 * multiple of 2^b_i.  In the tick, the particles that end a step inject with
 * their own dt_i (sources set) and recompute their gradient record from the
 * current states; every pair whose smaller bin ends a step exchanges
 * dt 2^min(b_k, b_l) |A| Phi_kl (the flux of rt_transport, GLF or HLL as
 * selected by rt_set_riemann, through the surfaces selected by
 * rt_set_surfaces) into the flux
 * sums of both particles; the particles that end a step apply
 * U - (flux sum) / V, guard the result as rt_transport does, and clear their
 * sums.
 *   U    [n][G][4] in/out, 16-byte aligned: the states (double in FP64
 *        contexts, float in FP32C ones).
 *   L    [S][G] luminosities (NULL without sources).
 *   UD   [n][G][16] in/out, 16-byte aligned, the state's type: the stored
 *        gradient records.  Before tick 0 fill it with rt_gradient of the
 *        initial U; keep it between ticks.
 *   acc  [n][G][4] double in/out (both precisions): the pending flux sums
 *        (zero before tick 0; all zero again after a tick where every
 *        particle ends a step).  In FP32C the exchanges of a tick are summed
 *        with compensation in FP32 and added to acc in FP64.
 *   photon_total [G] out or NULL: sum_k V_k E_k of the states after the tick
 *        (the pending sums are not in it: with them, sum_k (V_k E_k - acc_k,E)
 *        is conserved up to injection and the ledger).
 *   counts, ledger: as rt_transport, accumulated. */
rt_status rt_tick(rt_ctx *ctx, void *U, const double *L, int64_t tick, void *UD,
                  double *acc, double *photon_total, int64_t *counts, double *ledger);

/* Adjoint (vector-Jacobian product) of one full step
 *   U_next = transport(inject(U_pre, L), gradient(inject(U_pre, L)))
 * with respect to U_pre and L.  (The thesis has no adjoint; this is the exact
 * derivative of the step above, taking the subgradient of the active branch at
 * the minmod switches and guards.)
 *   U_pre    [n][G][4] state before injection of this step.
 *   L        [S][G] luminosities used by the step (NULL if no sources).
 *   dt       [1] device.
 *   UD       gradient record of the post-injection state (rt_gradient after
 *            rt_inject), or NULL (recomputed into library scratch from U_pre).
 *   U_unguarded  the forward's unguarded updated state of this step, or NULL
 *            (recomputed).
 *   lam_next [n][G][4] dLoss/dU_next.  lam [n][G][4] out: dLoss/dU_pre; may
 *            alias lam_next.
 *   dL_dL    [S][G] double, accumulated (+=) dLoss/dL, or NULL.
 * U_pre is read only when UD is NULL.  Scratch (a few state-sized buffers) is
 * allocated by the library on first use.  The step differentiated uses the
 * selected Riemann solver and effective surfaces. */
rt_status rt_adjoint(rt_ctx *ctx, const void *U_pre, const double *L, const double *dt,
                     const void *UD, const void *U_unguarded, const void *lam_next, void *lam,
                     double *dL_dL);

/* rt_adjoint for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments and result as rt_adjoint with UD and U_unguarded given (both
 * required: recomputing them would need more scratch); it calls no hipMalloc,
 * hipFree or allocating library routine.  Its scratch (5 state-sized arrays:
 * the guarded cotangent and the pair-pass records) is a fixed 64 MiB device
 * array of the library, one copy per GPU held until the process ends, so
 * 256-byte-aligned n x G x 4 x sizeof(state element) x (1 + 4) bytes must fit
 * in 64 MiB: n G up to about 419 thousand in FP64, 838 thousand in FP32C, else
 * RT_EINVAL (before any device work).  Nothing in the array needs clearing
 * between calls, but every call on one GPU uses the same array: calls that
 * overlap on a GPU (two contexts or streams) race and must be serialized.
 * RT_ESTATE before rt_build_cells; RT_EINVAL if the context's device is not
 * current; RT_EHIP if the array's address could not be looked up when the
 * context was created. */
rt_status rt_adjoint_static(rt_ctx *ctx, const double *L, const double *dt, const void *UD,
                            const void *U_unguarded, const void *lam_next, void *lam,
                            double *dL_dL);

/* Wait for the stream; return the device-side error raised since the last
 * rt_sync (RT_ENONFINITE, see the conventions above) or RT_OK, and clear the
 * status word. */
rt_status rt_sync(rt_ctx *ctx);

/* ---- queries (synchronising; for tests and diagnostics) ---------------- */
typedef struct {
    int64_t n;
    int64_t n_entries;      /* directed neighbour entries sum_i |N(i)|          */
    int64_t n_pairs;        /* unordered interacting pairs = n_entries / 2      */
    int64_t n_gather;       /* directed entries with r_ij < H_i                 */
    int64_t sell_slots;     /* padded slots of the wave-sliced neighbour table  */
    int32_t max_neighbours;
    int32_t h_iter_max;     /* most Newton/bisection iterations of one particle */
    int64_t n_inject;       /* source-gas injection entries                     */
    int64_t device_bytes;   /* device memory the context holds now              */
    int64_t device_bytes_peak; /* the most it held at once since rt_create,
                               including the build's transient lists            */
    int64_t h_list_overflow;   /* particles of the last build whose smoothing-
                               length candidate list overflowed (their later
                               evaluations walked the tree again)               */
    int64_t union_blocks;      /* FP64, up to 4 groups: blocks of 64 particles
                               whose gradient reads its neighbours from their
                               union staged in LDS                              */
    int64_t union_staged_blocks; /* those whose union did not fit (the gradient
                               stages their rows per pair instead)              */
    int64_t adj_union_blocks;  /* FP64, up to 4 groups: blocks of 64 particles
                               whose adjoint transposed gradient reads the
                               union of their symmetric lists from LDS          */
    int64_t adj_union_staged_blocks; /* those whose union did not fit           */
    int64_t task_longest;      /* tile transports: the longest task list of each
                               64-particle tile, summed over the tiles          */
    int64_t task_bound;        /* its lower bound in each tile (the longest list
                               of neighbours outside the tile, or the mean list
                               length rounded up), summed over the tiles        */
} rt_stats;
rt_status rt_get_stats(rt_ctx *ctx, rt_stats *out /* [host] */);

/* Per particle (Morton order): B [n][6] = (B00, B01, B02, B11, B12, B22) of
 * B_i = E_i^{-1}; n_nbr [n] = |N(i)|, n_gath [n] = |{j : r_ij < H_i}|.
 * Any pointer may be NULL. */
rt_status rt_get_geometry(rt_ctx *ctx, double *B, int32_t *n_nbr, int32_t *n_gath);

/* Neighbour lists (Morton indices) as CSR: ptr [n+1] int64, idx [n_entries]
 * int32; row i lists first the gather neighbours (r_ij < H_i), then the
 * others, each part in increasing index order. */
rt_status rt_get_neighbours(rt_ctx *ctx, int64_t *ptr, int32_t *idx);

/* Injection entries (sorted by gas, then source): gas, src [n_inject] int32,
 * xi [n_inject] double; h_src [S] source smoothing lengths.  NULL allowed. */
rt_status rt_get_sources(rt_ctx *ctx, int32_t *gas, int32_t *src, double *xi, double *h_src);

/* Kernel timing with HIP events recorded on the context stream around each
 * launch of the named kernel ("transport", "gradient", "inject", "adjoint").
 * rt_timing(ctx, 1) starts recording and clears totals; rt_timing(ctx, 0)
 * stops.  rt_get_timing returns the summed milliseconds and launch count
 * (synchronising). */
rt_status rt_timing(rt_ctx *ctx, int32_t on);
rt_status rt_get_timing(rt_ctx *ctx, const char *kernel, double *ms_total, int64_t *launches);

#ifdef __cplusplus
}
#endif

#endif /* GEARRT_RT_H */
