/*
 * start.h -- C-ABI of libstart: photoionization rates of SPH particles lit by
 * many radiation sources, with the tree acceleration of START (Hasegawa &
 * Umemura 2010, "START: smoothed particle hydrodynamics with tree-based
 * accelerated radiative transfer", MNRAS 407, 2632), on AMD MI355X (gfx950).
 *
 * What is computed (one frequency, the Lyman limit, cross-section sigma):
 *
 *   Gamma_i = sigma / (4 pi) * sum_alpha L_alpha exp(-tau_alpha) / d_alpha^2
 *
 * for every target particle i: the photoionization rate per H I atom of
 * Appendix A eq. (A2) with on-the-spot attenuation (eq. 7).  The sum runs over
 * the virtual sources of section 2.2.2: the source octree is walked from the
 * root and a cell of side l at distance d (to the cell's closest point) is
 * used whole when l/d <= theta_crit (eq. 12) while its parent was not
 * (eq. 13); it then shines with the summed luminosity (eq. 14) from its centre
 * of luminosity (eq. 15).  Single sources are used as themselves.  The
 * target's own source (self_src) is never used: k_other of eqs. (25)-(26).
 * tau_alpha = sigma * integral of n_HI along the straight segment between the
 * (virtual) source and the target, through a G^3 grid of Shepard-normalised
 * SPH densities (kernel of section 2.1) that is integrated exactly cell by
 * cell.  k_ion,i = n_HI,i * Gamma_i if the caller needs the rate per volume.
 *
 * Conventions for every call:
 *  - Positions are structure-of-arrays [3][n] (all x, then all y, then all z)
 *    in any length unit; start_box.length_unit_cm converts it to cm.  Every
 *    position must lie in the closed cube [lo, lo + size]^3.
 *  - Array arguments are DEVICE pointers (hipMalloc'd or torch tensors on the
 *    context's device) unless marked "host or device"; the caller owns them
 *    and must keep them alive until the context stream has passed the call.
 *  - Calls are asynchronous on the context stream unless stated otherwise.
 *    Argument errors are returned at once.  Problems in device data found by
 *    an asynchronous call (non-finite or out-of-box targets, self_src out of
 *    range) are reported by the next start_synchronize.
 *  - Errors are status codes; nothing aborts and no exception crosses the
 *    ABI.  start_last_error gives a message for the last failing call.
 *  - A context is used by one host thread at a time.
 *  - n = 0 is a valid no-op (Gamma is not written).
 */
#ifndef START_H
#define START_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    START_OK = 0,
    START_EINVAL = -1,       /* bad argument: null pointer, n < 0, theta < 0, L < 0, h <= 0 ... */
    START_ENOMEM = -2,       /* device allocation failed */
    START_EHIP = -3,         /* HIP runtime error */
    START_EOUTOFBOX = -4,    /* a position outside the box */
    START_ENONFINITE = -5,   /* NaN or Inf in the input */
    START_EBUDGET = -6,      /* allocation would exceed the context's HBM budget */
    START_ENOTIMPL = -7,     /* not implemented */
    START_ECAPACITY = -8     /* output buffer or fixed scratch too small (required size is returned
                                where the call has an output for it) */
} start_status;

typedef enum {
    START_FP64 = 0,   /* march, exp and sums in FP64; Gamma written as double */
    START_FP32C = 1   /* FP64 opening test (same lists), FP32 march with Kahan-compensated
                         tau and Gamma sums; Gamma written as float */
} start_precision;

/* Cubic box [lo, lo+size]^3 holding sources, gas and targets. */
typedef struct {
    double lo[3];
    double size;              /* > 0 */
    double length_unit_cm;    /* cm per length unit, > 0 */
} start_box;

typedef struct start_ctx start_ctx;
typedef struct start_tree start_tree;
typedef struct start_grid start_grid;

/* Context on `device`.  hip_stream: a hipStream_t to run on, or NULL for a
 * stream of its own.  hbm_budget_bytes: cap on the device memory the library
 * allocates through this context (0 = no cap); allocations beyond it fail
 * with START_EBUDGET.  Device memory that the library releases (a freed tree
 * or grid, the temporaries of a call) stays with the context, up to 8 GiB,
 * and is reused for later requests of the same size; it goes back to the
 * device when a new allocation needs the room (budget or device memory
 * short) and at start_ctx_destroy. */
start_status start_ctx_create(int device, void *hip_stream, size_t hbm_budget_bytes, start_ctx **out);
void start_ctx_destroy(start_ctx *ctx);
/* Message of the last failing call on ctx; valid until the next call. */
const char *start_last_error(const start_ctx *ctx);
/* Waits for the context stream and reports device-side input errors. */
start_status start_synchronize(start_ctx *ctx);
/* Device memory currently held by trees, grids and scratch of ctx (the
 * released blocks kept for reuse not included). */
size_t start_bytes_in_use(const start_ctx *ctx);

/* Octree over n_s sources (section 2.2.2, eqs. 14-15).  src_xyz [3][n_s],
 * src_lum [n_s] photons per second, >= 0 and finite.  Synchronous: returns
 * after validation (START_EOUTOFBOX / START_ENONFINITE / START_EINVAL).  The
 * tree owns its device memory until start_tree_free. */
start_status start_build_source_tree(start_ctx *ctx, const start_box *box, int64_t n_s, const double *src_xyz,
                                     const double *src_lum, start_tree **out);
start_status start_tree_free(start_ctx *ctx, start_tree *tree);

/* Kernel-weighted luminosities of the virtual sources: the two SPH-kernel
 * forms that section 2.2.2 offers beside the sum of eq. (14), the second
 * suggested there for diffuse radiation where every particle emits.  For
 * every cell of two or more sources, with r its centre of luminosity (eq. 15,
 * still the virtual source's position) and W_j = W(|r - r_j|, h_j) the cubic
 * spline of section 2.1 with the member's own smoothing length:
 *   START_LUM_KERNEL_MEAN:   L = sum_j L_j W_j / sum_j W_j, 0 (the cell is
 *                            left out) when no member's kernel reaches r;
 *   START_LUM_KERNEL_VOLUME: L = sum_j V_j L_j W_j, V_j = m_j / rho_j.
 * Single sources keep their own luminosity.  The sums start from the
 * sources' own luminosities, so calling again gives the same tree and the
 * last form wins; a rebuild restores eq. (14).  src_h [n_s] > 0 in the box's
 * length units, src_vol [n_s] >= 0 in length units cubed (NULL allowed for
 * the mean form); both device arrays in the order the sources were given.
 * Synchronous: START_EINVAL for a bad form, a NULL array, h <= 0 or V < 0,
 * START_ENONFINITE for NaN or Inf (the tree is then unchanged). */
typedef enum { START_LUM_KERNEL_MEAN = 1, START_LUM_KERNEL_VOLUME = 2 } start_lum_form;
start_status start_tree_kernel_luminosity(start_ctx *ctx, start_tree *tree, start_lum_form form, const double *src_h,
                                          const double *src_vol);

/* Neutral-hydrogen grid: G = 2^grid_log2 cells per axis (1 <= grid_log2 <= 10;
 * 0 picks G = 2^ceil(log2(n_gas^(1/3)))), value at each cell centre
 *   n_c = sum_k nhi_k W(|x_c - r_k|, h_k) / sum_k W(|x_c - r_k|, h_k),
 * W the cubic spline of section 2.1 with support 2h, 0 where no kernel
 * reaches.  gas_xyz [3][n_gas], gas_h [n_gas] > 0, gas_nhi [n_gas] >= 0
 * (cm^-3).  Synchronous, validates like the tree. */
start_status start_build_gas_grid(start_ctx *ctx, const start_box *box, int64_t n_gas, const double *gas_xyz,
                                  const double *gas_h, const double *gas_nhi, int grid_log2, start_grid **out);
start_status start_grid_free(start_ctx *ctx, start_grid *grid);
/* The tree and the grid of one scene in one call: the same results as
 * start_build_source_tree and start_build_gas_grid with these arguments,
 * with the two builds running at the same time (the grid on a second stream
 * of the context, driven from a second host thread).  Synchronous; all
 * input pointers must stay valid until it returns.  On any failure both
 * outputs are NULL, nothing is left allocated, and the status and message
 * are those of the failing build (the tree's if both fail). */
start_status start_build_scene(start_ctx *ctx, const start_box *box, int64_t n_s, const double *src_xyz,
                               const double *src_lum, int64_t n_gas, const double *gas_xyz, const double *gas_h,
                               const double *gas_nhi, int grid_log2, start_tree **tree_out, start_grid **grid_out);
/* G of a grid (host). */
int start_grid_size(const start_grid *grid);

/* Gamma for n_t targets: tgt_xyz [3][n_t]; self_src [n_t] original source
 * index of each target's own emission, -1 for none, or NULL; theta_crit >= 0
 * (0 = every source individually); sigma_cm2 >= 0.  gamma_out [n_t], in the
 * targets' input order, double for START_FP64 and float for START_FP32C,
 * s^-1 per H I atom.  Tree and grid must have been built on the same box.
 * Asynchronous; uses context scratch that is grown when needed (so the first
 * call of a larger size allocates and synchronises). */
start_status start_compute_rates(start_ctx *ctx, const start_tree *tree, const start_grid *grid, int64_t n_t,
                                 const double *tgt_xyz, const int64_t *self_src, double theta_crit,
                                 double sigma_cm2, start_precision prec, void *gamma_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it): start_compute_rates with the same arguments and the same results (bit
 * for bit: the same kernels), whose temporaries (target order, sorted
 * positions, sort buffers, item and tile tables) live in a fixed 24 MiB
 * device array that the library holds on every GPU it runs on until the
 * process ends, instead of context scratch.  Its tables are written by a
 * kernel, so the call allocates nothing, stages nothing on the host and
 * never synchronises.  Limit: n_t <= 2^18 targets (any tile size);
 * beyond it START_ECAPACITY, with nothing enqueued.  Every call on one GPU
 * shares that array: calls that overlap on one GPU (other streams, other
 * contexts, other host threads) race and must be ordered by the caller.
 * Asynchronous; device-side input errors are reported by the next
 * start_synchronize, as for start_compute_rates. */
start_status start_compute_rates_noalloc(start_ctx *ctx, const start_tree *tree, const start_grid *grid,
                                         int64_t n_t, const double *tgt_xyz, const int64_t *self_src,
                                         double theta_crit, double sigma_cm2, start_precision prec,
                                         void *gamma_out);

/* H2 photodissociation rate (s^-1) of each target by the Lyman-Werner band
 * (Appendix B, eq. B1, summed over the interaction list as in eq. A5):
 *   k_dis,i = 1.13e8 * sum_alpha L_alpha / (4 pi d_alpha^2) * f_sh(N_alpha / 1e14),
 * f_sh(x) = 1 for x <= 1 and x^(-3/4) above (eq. B2), N_alpha the H2 column
 * (cm^-2) along the ray through the grid.  Same walk, lists and rays as
 * start_compute_rates; the tree holds Lyman-Werner luminosities
 * (erg s^-1 Hz^-1) and the grid n_H2 (cm^-3, built by start_build_gas_grid
 * from per-particle n_H2).  kdis_out [n_t]: double (FP64) or float (FP32C).
 * Asynchronous, errors as start_compute_rates. */
start_status start_compute_dissociation_rates(start_ctx *ctx, const start_tree *tree, const start_grid *grid,
                                              int64_t n_t, const double *tgt_xyz, const int64_t *self_src,
                                              double theta_crit, start_precision prec, void *kdis_out);

/* Gamma of every gas particle (the particles are the targets) with the
 * optical depths of the upstream-particle chain of section 2.2.1 (eqs. 8-9)
 * instead of the ray integral, on the same interaction lists: for each
 * (particle i, list entry alpha) the upstream particle is the neighbour j
 * (|r_j - r_i| <= 2 h_i, j != i) that is closer to alpha, has alpha in its
 * own list and is nearest to the ray (largest cos phi, lowest j on ties);
 *   tau_i = tau_j + sigma (d_i - d_j) (n_HI,i + n_HI,j) / 2,
 * and pairs without one (list-boundary particles) integrate along the ray
 * through `grid`.  FP64.  gas_xyz [3][n_gas], gas_h [n_gas] > 0 (SPH
 * smoothing lengths: 2h is the neighbour radius), gas_nhi [n_gas] >= 0 (the
 * particles' own n_HI), self_src as start_compute_rates.  gamma_out [n_gas]
 * double.  offsets_out [n_gas+1] (host or device, may be NULL) receives the
 * list offsets; parents_out [capacity] (host or device, may be NULL) the
 * upstream particle of each pair in the order of start_interaction_lists, or
 * -1; n_roots_out (host, may be NULL) the number of pairs integrated along
 * the ray.  Synchronous; allocates its work arrays (about 48 bytes per list
 * entry, 32 bytes per neighbour pair, and a membership table of
 * n_gas * ceil((n_nodes + n_src) / 32) 32-bit words where that takes at most
 * max(8 bytes per list entry, 64 MiB) and 4 GiB; larger trees search the
 * neighbours' sorted lists instead, with the same result) for the duration of
 * the call.  More than 2^31 list entries -> START_ECAPACITY. */
start_status start_compute_rates_upstream(start_ctx *ctx, const start_tree *tree, const start_grid *grid,
                                          int64_t n_gas, const double *gas_xyz, const double *gas_h,
                                          const double *gas_nhi, const int64_t *self_src, double theta_crit,
                                          double sigma_cm2, double *gamma_out, int64_t *offsets_out,
                                          int64_t *parents_out, int64_t capacity, int64_t *n_roots_out);

/* One independent rate problem for start_compute_rates_batched. */
typedef struct {
    const start_tree *tree;
    const start_grid *grid;
    int64_t n_t;
    const double *tgt_xyz;
    const int64_t *self_src;
    double theta_crit;
    double sigma_cm2;
    start_precision prec;
    void *gamma_out;
} start_item;

/* Several independent problems (each exactly as start_compute_rates would
 * compute it) enqueued together on the context stream. */
start_status start_compute_rates_batched(start_ctx *ctx, int n_items, const start_item *items);

/* A batch staged once and replayed from a HIP graph, for callers that repeat
 * the same rate problems (a served scene asked again, an iteration that
 * recomputes the rates after changing the gas): start_rates_plan_create
 * checks the items as start_compute_rates_batched does, stages the batch
 * (item and tile tables, the targets' order and a sorted copy of their
 * positions, in memory the plan owns), runs it once (so the outputs are
 * written) and captures its rate kernels; start_rates_plan_launch enqueues
 * that graph on the context stream, which recomputes every output from the
 * current contents of the trees, grids and self_src arrays, with the target
 * positions as they were at creation (a changed position needs a new plan).
 * Trees, grids, self_src and outputs must stay allocated, at the same
 * addresses and sizes, until start_rates_plan_free.  A plan is used with the
 * context that made it; launches of one plan on one stream run in order.
 * Create and free synchronise the context stream; launch is asynchronous.
 * Create captures the context stream (thread-local capture mode): another
 * host thread that frees device memory or synchronises the whole device
 * while it runs invalidates the capture, and create then returns
 * START_EHIP; callers with such threads serialise them with plan creation. */
typedef struct start_plan start_plan;
start_status start_rates_plan_create(start_ctx *ctx, int n_items, const start_item *items, start_plan **out);
start_status start_rates_plan_launch(start_ctx *ctx, start_plan *plan);
start_status start_rates_plan_free(start_ctx *ctx, start_plan *plan);

/* Work decomposition of the rate kernels: each wavefront walks the tree for
 * a tile of up to tile_targets targets (one per lane) and marches the rays of
 * that tile 64 at a time.  1 <= tile_targets <= 64 fixes the tile size for
 * every call on the context; 0 (the default) takes it from the autotuned
 * table for the call's total number of targets, or else uses about
 * total / 4096 (a power of two in [1, 64]) so that small calls still fill
 * the GPU.  Results do not depend on the tile size (bit for bit). */
start_status start_set_tile_targets(start_ctx *ctx, int tile_targets);

/* Times the batch (as start_compute_rates_batched, which it runs, writing
 * the outputs) with tiles of 64, 32, 16, 8, 4 and 1 targets, `reps` times
 * each (a size twice as slow as the best so far on its first run is not
 * repeated), and records the fastest for the batch's size class (total
 * targets rounded up to a power of two) in the context's table; 64 is kept
 * unless another size is at least 3% faster.  best_tile
 * and best_ms (host, may be NULL) receive the choice and its mean time.
 * Synchronous. */
start_status start_autotune_rates(start_ctx *ctx, int n_items, const start_item *items, int reps, int *best_tile,
                                  double *best_ms);

/* Upper bound of the device bytes a tree, grid and rate call of these sizes
 * hold at once (for admission by memory). */
size_t start_estimate_bytes(int64_t n_t, int64_t n_s, int64_t n_gas, int grid_log2, start_precision prec);

/* ---- photoionisation equilibrium (pure hydrogen, static gas) ---- */

/* Equilibrium neutral fraction of each particle for given rates: the
 * ionisations per volume x n_H Gamma (Appendix A, eq. A2) balance the
 * recombinations alpha (1 - x)^2 n_H^2 (n_e = n_p = (1 - x) n_H); alpha is the
 * case-B coefficient under the on-the-spot approximation of section 2.1.  The
 * root in [0, 1] is x = 2a / (2a + Gamma + sqrt(Gamma (Gamma + 4a))) with
 * a = alpha n_H; a = Gamma = 0 gives x = 1.
 *   n_h     [n] total hydrogen density, cm^-3, finite and >= 0
 *   gamma   [n] rate per H I atom, s^-1: double (START_FP64) or float
 *           (START_FP32C), finite and >= 0 (e.g. start_compute_rates output)
 *   alpha   recombination coefficient, cm^3 s^-1, > 0
 *   x_hi    [n] in: the previous neutral fraction; out: the new one
 *   n_hi    [n] or NULL: receives x n_H (the n_HI of the next gas grid)
 *   max_change  HOST pointer or NULL: receives max |x_new - x_old|; the call
 *           then waits for the stream and reports bad device data itself
 * Asynchronous when max_change is NULL; bad values in n_h, gamma or x_hi are
 * then reported by the next start_synchronize (START_EINVAL). */
start_status start_equilibrium_update(start_ctx *ctx, int64_t n, const double *n_h, const void *gamma,
                                      start_precision gamma_prec, double alpha, double *x_hi, double *n_hi,
                                      double *max_change);

/* Photoionisation equilibrium of the gas around the fixed sources of `tree`,
 * by fixed-point iteration: grid n_HI = x n_H (as start_build_gas_grid, on
 * the tree's box), Gamma of every gas particle (as start_compute_rates with
 * the particles as targets, no self term), then x from
 * start_equilibrium_update; stop after the first iteration whose largest
 * change of x is <= tol, or after max_iter.  From a neutral start the
 * iterates decrease monotonically towards the equilibrium; for one source in
 * uniform gas its ionised volume is the Stromgren sphere of eq. (17).
 *   gas_xyz [3][n_gas], gas_h [n_gas] > 0, n_h [n_gas] >= 0 (cm^-3)
 *   grid_log2 in [1, 10]; theta_crit, sigma_cm2 as start_compute_rates;
 *   alpha > 0; prec: precision of the rate calls; max_iter >= 1; tol >= 0
 *   x_hi [n_gas] in: initial neutral fraction in [0, 1]; out: the last iterate
 *   gamma_out [n_gas] (double or float by prec): the rates the last iterate
 *           was computed from
 *   iterations, last_change (host, may be NULL): iterations run and the
 *           largest change of the last one
 * Synchronous (one stream synchronisation per iteration); allocates its
 * grid, particle bins and one n_HI buffer for the duration of the call.  The
 * first iteration stages the rate call (tables, target order); the others
 * repeat its kernels with the grid refill and the update, replayed from one
 * captured HIP graph unless start_set_graph_replay turned graphs off.  The
 * context stream must not be used by other threads during the call. */
start_status start_ionization_equilibrium(start_ctx *ctx, const start_tree *tree, int64_t n_gas,
                                          const double *gas_xyz, const double *gas_h, const double *n_h,
                                          int grid_log2, double theta_crit, double sigma_cm2, double alpha,
                                          start_precision prec, int max_iter, double tol, double *x_hi,
                                          void *gamma_out, int *iterations, double *last_change);

/* Photoionisation equilibrium with the transfer of recombination photons
 * (section 4.1) instead of the on-the-spot approximation: each iteration
 * makes every gas particle an emitter of alpha_1 n_e n_p V (eq. 19) next to
 * the n_star stars, builds the source tree of both (once: later iterations
 * put the new luminosities into it and redo its moments, which gives the
 * rebuilt tree bit for bit), grids n_HI = x n_H,
 * evaluates Gamma of every particle from every other emitter (self
 * excluded, k_other of eqs. 25-26) and solves
 *   x Gamma = alpha_eff n_H (1 - x)^2,  alpha_eff = alpha_A - alpha_1 (1 - exp(-tau_self)),
 * i.e. k_other + k_self = alpha_A n_e n_p with k_self of eq. (30) taking its
 * optical depth (eq. 28) from the previous iterate.  Stops as
 * start_ionization_equilibrium.  box: the cube of the particles and stars;
 * volume_cm3 [n_gas] >= 0 (V of each particle); star_xyz [3][n_star],
 * star_lum [n_star] (photons/s); alpha_A > alpha_1 >= 0.  Other arguments as
 * start_ionization_equilibrium.  Synchronous; allocates its tree, grid and
 * work arrays for the duration of the call. */
start_status start_diffuse_equilibrium(start_ctx *ctx, const start_box *box, int64_t n_gas, const double *gas_xyz,
                                       const double *gas_h, const double *n_h, const double *volume_cm3,
                                       int64_t n_star, const double *star_xyz, const double *star_lum, int grid_log2,
                                       double theta_crit, double sigma_cm2, double alpha_a, double alpha_1,
                                       start_precision prec, int max_iter, double tol, double *x_hi, void *gamma_out,
                                       int *iterations, double *last_change);

/* Whether start_ionization_equilibrium replays its iterations from a
 * captured HIP graph (default on) or launches them one by one.  The results
 * are the same either way (bit for bit). */
start_status start_set_graph_replay(start_ctx *ctx, int enable);

/* Whether the equilibrium loops (start_ionization_equilibrium,
 * start_diffuse_equilibrium) record, after their first iteration, every
 * (grid cell, gas particle) pair inside the kernel support with its weight
 * (12 bytes per pair, ~32 pairs per cell at one particle per cell) and
 * refill the grid from them (default on), or search the stencil at every
 * refill.  The grids, and so all results, are the same either way (bit for
 * bit); the recording is skipped by itself when its memory is not there. */
start_status start_set_grid_pairs(start_ctx *ctx, int enable);

/* ---- transfer of recombination photons (section 4.1) ---- */

/* Per particle, with n_e = n_p = (1 - x) n_H:
 *   lum_out    [n] or NULL: recombination photons per second to the ground
 *              state, alpha_1 n_e n_p V (eq. 19; alpha_1 = alpha_A - alpha_B),
 *              the luminosity of the particle as an emitter (source tree)
 *   k_self_out [n] or NULL: ionisations per cm^3 per s by the particle's own
 *              photons, alpha_1 n_e n_p (1 - exp(-tau)) (eq. 30), with
 *              tau = sigma n_HI (3 V / (4 pi))^(1/3) from its edge to its
 *              centre (eq. 28)
 * n_h [n] >= 0 (cm^-3), x_hi [n] neutral fraction in [0, 1], volume_cm3 [n]
 * >= 0; sigma_cm2, alpha_1 >= 0.  Asynchronous; bad values in the arrays are
 * reported by the next start_synchronize (START_EINVAL). */
start_status start_recombination_emission(start_ctx *ctx, int64_t n, const double *n_h, const double *x_hi,
                                          const double *volume_cm3, double sigma_cm2, double alpha_1,
                                          double *lum_out, double *k_self_out);

/* Total photoionisations per cm^3 per s of each particle, eq. (25):
 * k_ion = k_other + k_self with k_other = x n_H Gamma (eq. 26), Gamma [n] the
 * rate per H I atom from every other emitter (start_compute_rates with
 * self_src set; double for START_FP64, float for START_FP32C); k_self [n] or
 * NULL (= 0).  k_ion_out [n] double.  Asynchronous; bad values are reported
 * by the next start_synchronize (START_EINVAL). */
start_status start_total_ionization(start_ctx *ctx, int64_t n, const double *n_h, const double *x_hi,
                                    const void *gamma, start_precision gamma_prec, const double *k_self,
                                    double *k_ion_out);

/* ---- parity and diagnostics (synchronous; buffers host or device) ---- */

/* Tree in depth-first order.  *n_nodes (host) receives the node count; each
 * array may be NULL.  keys_sorted [n_s] Morton keys in sorted order (bit
 * 3b+2 = x bit b, 3b+1 = y, 3b = z, 21 bits per axis); perm [n_s] original
 * index of each sorted source; node_geo [n][4] = (cx, cy, cz, level | kind<<8)
 * with kind 0 = cell that splits, 1 = level-21 bucket, 2 = single source;
 * node_link [n][4] = (index after the subtree, first sorted source, source
 * count, original source index of a single source or -1); node_mom [n][4] =
 * (centre of luminosity x, y, z; luminosity) in FP64. */
start_status start_tree_export(start_ctx *ctx, const start_tree *tree, int64_t *n_nodes, uint64_t *keys_sorted,
                               uint32_t *perm, int32_t *node_geo, int32_t *node_link, double *node_mom);

/* Interaction lists of the walk, per target in input order.  offsets [n_t+1]
 * (host or device) receives the prefix of the list lengths; entries
 * [capacity] (host or device) receives, per target in depth-first order, the
 * node index of each cell used whole, or -(original source index)-1 of each
 * source used individually.  Returns START_ECAPACITY, with offsets filled,
 * when offsets[n_t] > capacity. */
start_status start_interaction_lists(start_ctx *ctx, const start_tree *tree, int64_t n_t, const double *tgt_xyz,
                                     const int64_t *self_src, double theta_crit, int64_t *offsets,
                                     int64_t *entries, int64_t capacity);

/* Grid values [G^3] (host or device), index (ix*G + iy)*G + iz, FP64. */
start_status start_grid_export(start_ctx *ctx, const start_grid *grid, double *values);

/* Per-target work counters [n_t][4] (host or device) of the rate walk:
 * opening tests, entries used, grid cells crossed, entries skipped at zero
 * distance. */
start_status start_rate_counters(start_ctx *ctx, const start_tree *tree, const start_grid *grid, int64_t n_t,
                                 const double *tgt_xyz, const int64_t *self_src, double theta_crit,
                                 start_precision prec, int64_t *counters);

/* Kernel timing of the rate walk (the dominant kernel): while enabled, every
 * start_compute_rates records HIP events on the context stream around its
 * walk kernel.  start_profile_read waits for the stream, returns the number
 * of timed launches with the total and largest duration in milliseconds
 * (host pointers, each may be NULL) and clears the record. */
start_status start_profile_enable(start_ctx *ctx, int enable);
start_status start_profile_read(start_ctx *ctx, int64_t *launches, double *total_ms, double *max_ms);

#ifdef __cplusplus
}
#endif
#endif
