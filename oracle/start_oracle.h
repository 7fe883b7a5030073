/*
 * start_oracle.h -- CPU FP64 reference for the photoionization-rate path of
 * START (Hasegawa & Umemura 2010, "START: smoothed particle hydrodynamics
 * with tree-based accelerated radiative transfer", MNRAS 407, 2632).
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle that the HIP library is
 * compared against.  It is plain, slow and written to be read against the
 * paper: recursive geometric subdivision of the source cube (section 2.2.2),
 * the opening test of eqs. (12)-(13), virtual sources of eqs. (14)-(15),
 * on-the-spot attenuation (eq. 7) with the optical depth integrated exactly
 * along each ray, and the sum over sources of Appendix A, eq. (A2), for a
 * single frequency.  It shares no code with the HIP library.  Only tests, the
 * smoke check and the CPU-baseline leg of the benchmark may call it.
 *
 * Conventions: positions are structure-of-arrays [3][n] in any length unit;
 * box_unit_cm converts that unit to cm.  All arithmetic is IEEE FP64 with
 * contraction disabled; fma() is used only where written.
 */
#ifndef START_ORACLE_H
#define START_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ENOMEM (-2)
#define OR_EOUTOFBOX (-4)
#define OR_ENONFINITE (-5)
#define OR_ECAPACITY (-6)

#define OR_MAX_LEVEL 21

typedef struct or_tree or_tree;

/* Cubic box [lo, lo+size]^3.  unit_cm: cm per length unit. */
typedef struct {
    double lo[3];
    double size;
    double unit_cm;
} or_box;

/* Octree over the sources: cubes split into 8 until one source remains or
 * level 21 is reached (section 2.2.2).  xyz is [3][n]; lum[n] >= 0. */
int or_tree_build(const or_box *box, int64_t n, const double *xyz, const double *lum,
                  or_tree **out);
void or_tree_free(or_tree *t);

/* Number of cells of the full octree (every cell holding >= 1 source). */
int64_t or_tree_ncells(const or_tree *t);

/* Export of every cell: level, integer coordinates [3], member count,
 * number of non-empty children, luminosity and centre of luminosity [3]
 * (eqs. 14-15), and the offset of its members in member_idx.  The members
 * of a cell are contiguous, in depth-first octant order of its sub-cubes;
 * a cell that is not split (one source or a level-21 bucket) lists them in
 * ascending source index. */
int or_tree_export(const or_tree *t, int32_t *level, int64_t *coord, int64_t *count,
                   int32_t *nchild, double *lum, double *com, int64_t *member_off,
                   int64_t *member_idx);

/* Replaces the luminosity of every cell of >= 2 sources by a kernel-weighted
 * one (section 2.2.2, the forms offered beside eq. (14)), evaluated at the
 * cell's centre of luminosity r (eq. 15) with the members' smoothing lengths
 * h[n] > 0: form 1 = sum L_j W_j / sum W_j (0 if every W_j = 0), form 2 =
 * sum vol_j L_j W_j with vol[n] = m_j / rho_j >= 0, W_j = W(|r - r_j|, h_j).
 * Single sources keep their own L; calling again gives the same cells. */
int or_tree_kernel_luminosity(or_tree *t, const double *h, const double *vol, int form);

/* Normalised position u = min((x - lo) / size, 1) as used for the tree. */
void or_normalise(const or_box *box, const double x[3], double u[3]);

/* Opening test of eqs. (12)-(13) for one cell and one normalised point:
 * returns 1 when l^2 <= theta^2 d^2 with d the distance to the closest point
 * of the cell. */
int or_accept(int32_t level, const int64_t coord[3], const double u[3], double theta);

/* Interaction lists: for each target, the sequence of entries of the walk in
 * depth-first octant order.  Each entry is 4 int64: (level, c0, c1, c2) for a
 * virtual source (the deepest cell with the same member set) or
 * (-1, source_index, 0, 0) for an individual source.  offsets has n_t+1
 * elements; entries capacity is counted in entries.  Returns OR_ECAPACITY
 * (with offsets filled) when the lists do not fit. */
int or_interaction_lists(const or_tree *t, int64_t n_t, const double *tgt_xyz,
                         const int64_t *self_src, double theta, int64_t *offsets,
                         int64_t *entries, int64_t capacity);

/* SPH kernel of section 2.1: cubic spline with support 2h, 3-D normalisation. */
double or_kernel_w(double r, double h);

/* Neutral-hydrogen density at the centres of a G^3 grid over the box:
 * Shepard-normalised SPH interpolant, 0 where no kernel reaches.
 * out[(ix*G + iy)*G + iz]. */
int or_grid_build(const or_box *box, int64_t n, const double *xyz, const double *h,
                  const double *nhi, int grid_log2, double *out);

/* Same value for a subset of cells given by linear index (brute force over
 * all particles, used to check sampled cells of large grids). */
int or_grid_cells(const or_box *box, int64_t n, const double *xyz, const double *h,
                  const double *nhi, int grid_log2, int64_t m, const int64_t *cells,
                  double *out);

/* Column integral of n_HI (cm^-3 times length units) along the segment a->b
 * of the piecewise-constant grid field; ncells (may be NULL) receives the
 * number of cells with a chord of positive length. */
double or_column(const or_box *box, int grid_log2, const double *grid, const double a[3],
                 const double b[3], int64_t *ncells);

/* Photoionization rate per H I atom (s^-1) of each target:
 *   Gamma_i = sigma/(4 pi) sum_alpha L_alpha exp(-tau_alpha) / d_alpha^2
 * over the entries of the target's interaction list.
 * counters (may be NULL): [n_t][4] = tests, entries, grid cells, zero-distance skips. */
int or_rates(const or_tree *t, int grid_log2, const double *grid, int64_t n_t,
             const double *tgt_xyz, const int64_t *self_src, double theta, double sigma,
             double *gamma_out, int64_t *counters, int nthreads);

/* H2 self-shielding function of Appendix B: f_sh(x) = 1 for x <= 1 and
 * x^(-3/4) above, x = N_H2 / 1e14 cm^-2. */
double or_fsh(double x);

/* H2 photodissociation rate (s^-1) of each target, Appendix B eq. (B1) summed
 * over the interaction list as in eq. (A5):
 *   k_dis,i = 1.13e8 sum_alpha F_alpha f_sh(N_H2,alpha / 1e14 cm^-2),
 * F_alpha = L_alpha / (4 pi d_alpha^2) the Lyman-Werner flux without
 * shielding (L in erg s^-1 Hz^-1 as the tree's luminosities), N_H2,alpha the
 * column of the gridded n_H2 (grid as or_grid_build of n_H2) along the ray. */
int or_lw_rates(const or_tree *t, int grid_log2, const double *grid, int64_t n_t,
                const double *tgt_xyz, const int64_t *self_src, double theta,
                double *kdis_out, int nthreads);

/* Photoionization rates with the optical depths of the upstream-particle
 * chain of section 2.2.1 (eqs. 8-9) on the lists of section 2.2.2: the gas
 * particles are the targets; for each (particle i, virtual source alpha) the
 * upstream particle is the neighbour j of i (|r_j - r_i| <= 2 h_i, j != i)
 * that is closer to alpha, has alpha in its own list, and is nearest to the
 * ray (largest cos phi, lowest index on ties); then
 *   tau_i = tau_j + sigma (d_i - d_j) (n_HI,i + n_HI,j) / 2,
 * and a pair without an upstream particle (a list-boundary particle)
 * integrates the column along the ray through the grid.  nhi: particle
 * n_HI.  offsets_out [n+1] (may be NULL) receives the list offsets;
 * parent_out [capacity] (may be NULL) the upstream particle of each pair of
 * each list, in list order, or -1.  stats [n][2] (may be NULL): pairs, pairs
 * integrated along the ray.  Neighbours are searched through a cell list
 * (cells within 2 h_i plus one of margin, candidates in increasing index),
 * which only skips particles that fail the distance test. */
int or_upstream_rates(const or_tree *t, int grid_log2, const double *grid, int64_t n,
                      const double *xyz, const double *h, const double *nhi,
                      const int64_t *self_src, double theta, double sigma,
                      double *gamma_out, int64_t *offsets_out, int64_t *parent_out,
                      int64_t capacity, int64_t *stats);
/* The same with the neighbour search chosen: all_pairs != 0 tests every
 * other particle (O(n^2), the definition as written), 0 the cell list. */
int or_upstream_rates_ex(const or_tree *t, int grid_log2, const double *grid, int64_t n,
                         const double *xyz, const double *h, const double *nhi,
                         const int64_t *self_src, double theta, double sigma,
                         double *gamma_out, int64_t *offsets_out, int64_t *parent_out,
                         int64_t capacity, int64_t *stats, int all_pairs);

#ifdef __cplusplus
}
#endif
#endif
