/*
 * start_oracle.c -- CPU FP64 reference for the photoionization-rate path of
 * START (Hasegawa & Umemura 2010).  TEST INFRASTRUCTURE ONLY: the oracle the
 * HIP library is compared against.  It shares no code with that library.
 *
 * What it computes, in the paper's order:
 *   1. the octree of the radiation sources: the cube is split into 8 sub-cubes
 *      until a cube holds a single source (section 2.2.2); capped at level 21,
 *      where a cube with several sources is a bucket whose sources are used
 *      one by one;
 *   2. the virtual source of every cell: total luminosity, eq. (14), at the
 *      centre of luminosity, eq. (15); optionally one of the two kernel-weighted
 *      luminosities of section 2.2.2 instead of the total;
 *   3. for every target particle the cells that pass the opening test
 *      l^n / d^n <= theta (eq. 12) while their parent fails it (eq. 13), with d
 *      the distance to the closest point of the cell, found top-down;
 *   4. the optical depth from each (virtual) source to the target, integrated
 *      along the straight ray (sections 2.2.1-2.2.2) through the neutral
 *      hydrogen field, here a grid of SPH-interpolated densities (section 2.1
 *      kernel), with exact chord lengths;
 *   5. the rate per H I atom, the monochromatic form of Appendix A eq. (A2)
 *      with on-the-spot attenuation (eq. 7):
 *         Gamma_i = sigma / (4 pi) * sum_alpha L_alpha exp(-tau_alpha) / d_alpha^2,
 *      excluding the target's own emission (k_other of eqs. 25-26);
 *   6. the H2 photodissociation rate of Appendix B on the same lists and
 *      rays: 1.13e8 sum_alpha L_alpha / (4 pi d_alpha^2) f_sh(N_H2 / 1e14),
 *      with the H2 column integrated like tau.
 *
 * Built with -O2 -ffp-contract=off and no fast-math: every rounding is the
 * one written here.
 */
#include "start_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t level;
    int32_t nchild;
    int64_t c[3];
    int64_t first, count;   /* members: t->idx[first .. first+count) */
    int64_t child[8];       /* cell index per octant, -1 when empty */
    double lum;             /* eq. (14) */
    double com[3];          /* eq. (15) */
} or_cell;

struct or_tree {
    or_box box;
    int64_t n;
    double *x;      /* [3][n] physical positions */
    double *u;      /* [3][n] normalised positions */
    double *lum;    /* [n] */
    int64_t *idx;   /* [n] source indices grouped cell by cell */
    or_cell *cells;
    int64_t ncells, cap;
};

static int finite3(const double *xyz, int64_t n, int64_t i)
{
    return isfinite(xyz[i]) && isfinite(xyz[n + i]) && isfinite(xyz[2 * n + i]);
}

static int in_box(const or_box *b, const double *xyz, int64_t n, int64_t i)
{
    for (int k = 0; k < 3; ++k) {
        double v = xyz[(int64_t)k * n + i];
        if (v < b->lo[k] || v > b->lo[k] + b->size) return 0;
    }
    return 1;
}

static int check_box(const or_box *b)
{
    if (!b) return OR_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!isfinite(b->lo[k])) return OR_ENONFINITE;
    if (!isfinite(b->size) || !isfinite(b->unit_cm)) return OR_ENONFINITE;
    if (!(b->size > 0) || !(b->unit_cm > 0)) return OR_EINVAL;
    return OR_OK;
}

static int check_points(const or_box *b, int64_t n, const double *xyz)
{
    for (int64_t i = 0; i < n; ++i) {
        if (!finite3(xyz, n, i)) return OR_ENONFINITE;
        if (!in_box(b, xyz, n, i)) return OR_EOUTOFBOX;
    }
    return OR_OK;
}

void or_normalise(const or_box *box, const double x[3], double u[3])
{
    double inv = 1.0 / box->size;
    for (int k = 0; k < 3; ++k) {
        double v = (x[k] - box->lo[k]) * inv;
        u[k] = v > 1.0 ? 1.0 : v;
    }
}

/* ---------------------------------------------------------------- tree --- */

static int64_t new_cell(or_tree *t)
{
    if (t->ncells == t->cap) {
        int64_t nc = t->cap ? 2 * t->cap : 1024;
        or_cell *p = (or_cell *)realloc(t->cells, (size_t)nc * sizeof(or_cell));
        if (!p) return -1;
        t->cells = p;
        t->cap = nc;
    }
    return t->ncells++;
}

/* Make the cell (level, c) holding idx[first..first+count) and, unless it is
 * a single source or a level-21 bucket, its 8 sub-cubes (section 2.2.2). */
static int64_t build_cell(or_tree *t, int32_t level, const int64_t c[3], int64_t first,
                          int64_t count, int64_t *tmp)
{
    int64_t ci = new_cell(t);
    if (ci < 0) return -1;
    or_cell *cell = &t->cells[ci];
    cell->level = level;
    cell->nchild = 0;
    for (int k = 0; k < 3; ++k) cell->c[k] = c[k];
    cell->first = first;
    cell->count = count;
    for (int o = 0; o < 8; ++o) cell->child[o] = -1;

    /* eqs. (14)-(15): summed over the members in ascending source index */
    double L = 0.0, S[3] = {0.0, 0.0, 0.0};
    for (int64_t m = first; m < first + count; ++m) {
        int64_t j = t->idx[m];
        L += t->lum[j];
        for (int k = 0; k < 3; ++k) S[k] += t->lum[j] * t->x[(int64_t)k * t->n + j];
    }
    cell->lum = L;
    for (int k = 0; k < 3; ++k) cell->com[k] = L > 0.0 ? S[k] / L : 0.0;

    if (count < 2 || level >= OR_MAX_LEVEL) return ci;

    /* split the cube at its mid-planes; octant o = 4*bx + 2*by + bz */
    double mid[3];
    for (int k = 0; k < 3; ++k) mid[k] = ldexp((double)(2 * c[k] + 1), -(level + 1));
    int64_t cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int64_t m = first; m < first + count; ++m) {
        int64_t j = t->idx[m];
        int o = 0;
        for (int k = 0; k < 3; ++k) o = 2 * o + (t->u[(int64_t)k * t->n + j] >= mid[k]);
        tmp[m] = o;
    }
    for (int64_t m = first; m < first + count; ++m) cnt[tmp[m]]++;
    int64_t start[8], pos[8];
    start[0] = first;
    for (int o = 1; o < 8; ++o) start[o] = start[o - 1] + cnt[o - 1];
    for (int o = 0; o < 8; ++o) pos[o] = start[o];
    /* stable partition keeps each child's members in ascending index order */
    int64_t *moved = (int64_t *)malloc((size_t)count * sizeof(int64_t));
    if (!moved) return -1;
    for (int64_t m = first; m < first + count; ++m) moved[pos[tmp[m]]++ - first] = t->idx[m];
    memcpy(t->idx + first, moved, (size_t)count * sizeof(int64_t));
    free(moved);

    int nchild = 0;
    for (int o = 0; o < 8; ++o) {
        if (!cnt[o]) continue;
        int64_t cc[3] = {2 * c[0] + ((o >> 2) & 1), 2 * c[1] + ((o >> 1) & 1), 2 * c[2] + (o & 1)};
        int64_t ch = build_cell(t, level + 1, cc, start[o], cnt[o], tmp);
        if (ch < 0) return -1;
        t->cells[ci].child[o] = ch;   /* t->cells may have moved */
        ++nchild;
    }
    t->cells[ci].nchild = nchild;
    return ci;
}

int or_tree_build(const or_box *box, int64_t n, const double *xyz, const double *lum,
                  or_tree **out)
{
    int rc = check_box(box);
    if (rc) return rc;
    if (!out || n < 0 || (n > 0 && (!xyz || !lum))) return OR_EINVAL;
    rc = check_points(box, n, xyz);
    if (rc) return rc;
    for (int64_t j = 0; j < n; ++j) {
        if (!isfinite(lum[j])) return OR_ENONFINITE;
        if (lum[j] < 0.0) return OR_EINVAL;
    }
    or_tree *t = (or_tree *)calloc(1, sizeof(or_tree));
    if (!t) return OR_ENOMEM;
    t->box = *box;
    t->n = n;
    size_t nb = (size_t)(n > 0 ? n : 1);
    t->x = (double *)malloc(3 * nb * sizeof(double));
    t->u = (double *)malloc(3 * nb * sizeof(double));
    t->lum = (double *)malloc(nb * sizeof(double));
    t->idx = (int64_t *)malloc(nb * sizeof(int64_t));
    int64_t *tmp = (int64_t *)malloc(nb * sizeof(int64_t));
    if (!t->x || !t->u || !t->lum || !t->idx || !tmp) {
        free(tmp);
        or_tree_free(t);
        return OR_ENOMEM;
    }
    if (n > 0) {
        memcpy(t->x, xyz, 3 * (size_t)n * sizeof(double));
        memcpy(t->lum, lum, (size_t)n * sizeof(double));
    }
    for (int64_t j = 0; j < n; ++j) {
        double x[3] = {xyz[j], xyz[n + j], xyz[2 * n + j]}, u[3];
        or_normalise(box, x, u);
        for (int k = 0; k < 3; ++k) t->u[(int64_t)k * n + j] = u[k];
        t->idx[j] = j;
    }
    if (n > 0) {
        int64_t root[3] = {0, 0, 0};
        if (build_cell(t, 0, root, 0, n, tmp) < 0) {
            free(tmp);
            or_tree_free(t);
            return OR_ENOMEM;
        }
    }
    free(tmp);
    *out = t;
    return OR_OK;
}

void or_tree_free(or_tree *t)
{
    if (!t) return;
    free(t->x);
    free(t->u);
    free(t->lum);
    free(t->idx);
    free(t->cells);
    free(t);
}

int64_t or_tree_ncells(const or_tree *t) { return t ? t->ncells : 0; }

int or_tree_export(const or_tree *t, int32_t *level, int64_t *coord, int64_t *count,
                   int32_t *nchild, double *lum, double *com, int64_t *member_off,
                   int64_t *member_idx)
{
    if (!t) return OR_EINVAL;
    for (int64_t i = 0; i < t->ncells; ++i) {
        const or_cell *c = &t->cells[i];
        if (level) level[i] = c->level;
        if (nchild) nchild[i] = c->nchild;
        if (count) count[i] = c->count;
        if (lum) lum[i] = c->lum;
        if (member_off) member_off[i] = c->first;
        for (int k = 0; k < 3; ++k) {
            if (coord) coord[3 * i + k] = c->c[k];
            if (com) com[3 * i + k] = c->com[k];
        }
    }
    if (member_idx && t->n > 0) memcpy(member_idx, t->idx, (size_t)t->n * sizeof(int64_t));
    return OR_OK;
}

/* ---------------------------------------------------------------- walk --- */

/* Eq. (12) with l the side of the level-n cube and d the distance from the
 * target to the closest point of the closed cube (0 inside).  Normalised
 * units, so l = 2^-n and the cube is [c 2^-n, (c+1) 2^-n] per axis exactly. */
int or_accept(int32_t level, const int64_t coord[3], const double u[3], double theta)
{
    double l = ldexp(1.0, -level);
    double d[3];
    for (int k = 0; k < 3; ++k) {
        double lo = ldexp((double)coord[k], -level);
        double hi = ldexp((double)(coord[k] + 1), -level);
        double a = lo - u[k];
        double b = u[k] - hi;
        double m = a > b ? a : b;
        d[k] = m > 0.0 ? m : 0.0;
    }
    double d2 = fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
    double theta2 = theta * theta;
    return l * l <= theta2 * d2;
}

typedef struct {
    int64_t cell;   /* >= 0: virtual source in this cell; -1: individual source */
    int64_t src;
} or_entry;

typedef struct {
    or_entry *e;
    int64_t n, cap;
    int64_t ntest;
    int failed;
} or_list;

static void push(or_list *L, int64_t cell, int64_t src)
{
    if (L->failed) return;
    if (L->n == L->cap) {
        int64_t nc = L->cap ? 2 * L->cap : 256;
        or_entry *p = (or_entry *)realloc(L->e, (size_t)nc * sizeof(or_entry));
        if (!p) {
            L->failed = 1;
            return;
        }
        L->e = p;
        L->cap = nc;
    }
    L->e[L->n].cell = cell;
    L->e[L->n].src = src;
    L->n++;
}

/* A cell whose members all sit in one sub-cube has the same member set as
 * that sub-cube; the entry is named by the deepest such cell. */
static int64_t deepest_same_set(const or_tree *t, int64_t ci)
{
    for (;;) {
        const or_cell *c = &t->cells[ci];
        if (c->nchild != 1) return ci;
        for (int o = 0; o < 8; ++o)
            if (c->child[o] >= 0) {
                ci = c->child[o];
                break;
            }
    }
}

static void emit_source(const or_tree *t, or_list *L, int64_t j, int64_t self)
{
    if (j != self && t->lum[j] > 0.0) push(L, -1, j);
}

/* Top-down: a cell passing eq. (12) is used as one virtual source and its
 * sub-cubes are not looked at, so every used cell also satisfies eq. (13).
 * A single source is used as itself; a level-21 bucket that fails the test
 * gives its sources one by one.  The target's own source is never used, and
 * sources or cells of zero luminosity contribute nothing and are left out. */
static void walk(const or_tree *t, int64_t ci, const double u[3], int64_t self,
                 double theta, or_list *L)
{
    const or_cell *c = &t->cells[ci];
    if (c->count == 1) {
        emit_source(t, L, t->idx[c->first], self);
        return;
    }
    int acc = or_accept(c->level, c->c, u, theta);
    /* count tests as a walk over the tree without single-child chains does */
    if (acc || c->nchild != 1) L->ntest++;
    if (acc) {
        if (c->lum > 0.0) push(L, deepest_same_set(t, ci), -1);
        return;
    }
    if (c->nchild == 0) {   /* level-21 bucket */
        for (int64_t m = c->first; m < c->first + c->count; ++m) emit_source(t, L, t->idx[m], self);
        return;
    }
    for (int o = 0; o < 8; ++o)
        if (c->child[o] >= 0) walk(t, c->child[o], u, self, theta, L);
}

static int list_for(const or_tree *t, const double x[3], int64_t self, double theta, or_list *L)
{
    L->n = 0;
    L->ntest = 0;
    L->failed = 0;
    if (t->ncells == 0) return OR_OK;
    double u[3];
    or_normalise(&t->box, x, u);
    walk(t, 0, u, self, theta, L);
    return L->failed ? OR_ENOMEM : OR_OK;
}

static int check_targets(const or_box *b, int64_t n_t, const double *tgt, const int64_t *self_src,
                         int64_t n_s, double theta)
{
    if (n_t < 0 || (n_t > 0 && !tgt)) return OR_EINVAL;
    if (!isfinite(theta)) return OR_ENONFINITE;
    if (theta < 0.0) return OR_EINVAL;
    int rc = check_points(b, n_t, tgt);
    if (rc) return rc;
    if (self_src)
        for (int64_t i = 0; i < n_t; ++i)
            if (self_src[i] < -1 || self_src[i] >= n_s) return OR_EINVAL;
    return OR_OK;
}

int or_interaction_lists(const or_tree *t, int64_t n_t, const double *tgt_xyz,
                         const int64_t *self_src, double theta, int64_t *offsets,
                         int64_t *entries, int64_t capacity)
{
    if (!t || !offsets) return OR_EINVAL;
    int rc = check_targets(&t->box, n_t, tgt_xyz, self_src, t->n, theta);
    if (rc) return rc;
    or_list L = {0};
    offsets[0] = 0;
    int over = 0;
    for (int64_t i = 0; i < n_t; ++i) {
        double x[3] = {tgt_xyz[i], tgt_xyz[n_t + i], tgt_xyz[2 * n_t + i]};
        rc = list_for(t, x, self_src ? self_src[i] : -1, theta, &L);
        if (rc) {
            free(L.e);
            return rc;
        }
        int64_t base = offsets[i];
        offsets[i + 1] = base + L.n;
        if (offsets[i + 1] > capacity || !entries) {
            over = 1;
            continue;
        }
        for (int64_t k = 0; k < L.n; ++k) {
            int64_t *e = entries + 4 * (base + k);
            if (L.e[k].cell >= 0) {
                const or_cell *c = &t->cells[L.e[k].cell];
                e[0] = c->level;
                e[1] = c->c[0];
                e[2] = c->c[1];
                e[3] = c->c[2];
            } else {
                e[0] = -1;
                e[1] = L.e[k].src;
                e[2] = 0;
                e[3] = 0;
            }
        }
    }
    free(L.e);
    return over ? OR_ECAPACITY : OR_OK;
}

/* ---------------------------------------------------------------- grid --- */

/* Cubic spline of section 2.1 (Monaghan 1992): support 2h,
 * W = f(r/h) / (pi h^3), f = 1 - 1.5 q^2 + 0.75 q^3 (q <= 1),
 * 0.25 (2 - q)^3 (1 < q <= 2), 0 beyond. */
double or_kernel_w(double r, double h)
{
    double q = r / h;
    double f;
    if (q <= 1.0)
        f = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    else if (q <= 2.0)
        f = 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
    else
        f = 0.0;
    return f / (M_PI * h * h * h);
}

static int check_gas(const or_box *box, int64_t n, const double *xyz, const double *h,
                     const double *nhi, int grid_log2)
{
    int rc = check_box(box);
    if (rc) return rc;
    if (n < 0 || grid_log2 < 0 || grid_log2 > 10) return OR_EINVAL;
    if (n > 0 && (!xyz || !h || !nhi)) return OR_EINVAL;
    rc = check_points(box, n, xyz);
    if (rc) return rc;
    for (int64_t k = 0; k < n; ++k) {
        if (!isfinite(h[k]) || !isfinite(nhi[k])) return OR_ENONFINITE;
        if (!(h[k] > 0.0) || nhi[k] < 0.0) return OR_EINVAL;
    }
    return OR_OK;
}

static void cell_centre(const or_box *box, int G, int64_t lin, double xc[3])
{
    int64_t ia = lin / ((int64_t)G * G), ib = (lin / G) % G, ic = lin % G;
    int64_t a[3] = {ia, ib, ic};
    double delta = box->size / G;
    for (int k = 0; k < 3; ++k) xc[k] = box->lo[k] + ((double)a[k] + 0.5) * delta;
}

static double dist3(const double a[3], const double *xyz, int64_t n, int64_t k)
{
    double dx = a[0] - xyz[k], dy = a[1] - xyz[n + k], dz = a[2] - xyz[2 * n + k];
    return sqrt(dx * dx + dy * dy + dz * dz);
}

/* Kernel-weighted luminosity of every cell of two or more sources, the two
 * SPH-kernel forms offered in section 2.2.2 beside the sum of eq. (14).  Both
 * are evaluated at the cell's centre of luminosity r (eq. 15, which stays the
 * virtual source's position) with each member's own smoothing length h_j:
 *   form 1:  L = sum_j L_j W(|r - r_j|, h_j) / sum_j W(|r - r_j|, h_j),
 *            0 when no member's kernel reaches r;
 *   form 2:  L = sum_j (m_j / rho_j) L_j W(|r - r_j|, h_j),  vol[j] = m_j / rho_j.
 * Sums run over the members in the cell's own order.  A single source keeps
 * its own luminosity (it is used as itself), and the members' luminosities
 * are not changed, so a second call gives the same cells. */
int or_tree_kernel_luminosity(or_tree *t, const double *h, const double *vol, int form)
{
    if (!t || (form != 1 && form != 2)) return OR_EINVAL;
    if (t->n > 0 && (!h || (form == 2 && !vol))) return OR_EINVAL;
    for (int64_t j = 0; j < t->n; ++j) {
        if (!isfinite(h[j]) || (form == 2 && !isfinite(vol[j]))) return OR_ENONFINITE;
        if (!(h[j] > 0.0) || (form == 2 && vol[j] < 0.0)) return OR_EINVAL;
    }
    for (int64_t ci = 0; ci < t->ncells; ++ci) {
        or_cell *c = &t->cells[ci];
        if (c->count < 2) continue;
        double num = 0.0, den = 0.0;
        for (int64_t m = c->first; m < c->first + c->count; ++m) {
            int64_t j = t->idx[m];
            double w = or_kernel_w(dist3(c->com, t->x, t->n, j), h[j]);
            if (form == 1) {
                num += t->lum[j] * w;
                den += w;
            } else {
                num += vol[j] * t->lum[j] * w;
            }
        }
        if (form == 1)
            c->lum = den > 0.0 ? num / den : 0.0;
        else
            c->lum = num;
    }
    return OR_OK;
}

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

/* Shepard-normalised SPH interpolant at the cell centres:
 *   n_c = sum_k nhi_k W(|x_c - r_k|, h_k) / sum_k W(|x_c - r_k|, h_k),
 * summed in ascending particle index; 0 where no kernel reaches.  Particles
 * are binned only to skip those whose kernel cannot reach a centre. */
int or_grid_build(const or_box *box, int64_t n, const double *xyz, const double *h,
                  const double *nhi, int grid_log2, double *out)
{
    int rc = check_gas(box, n, xyz, h, nhi, grid_log2);
    if (rc) return rc;
    if (!out) return OR_EINVAL;
    const int G = 1 << grid_log2;
    const int64_t ncell = (int64_t)G * G * G;
    if (n == 0) {
        memset(out, 0, (size_t)ncell * sizeof(double));
        return OR_OK;
    }
    double rmax = 0.0;
    for (int64_t k = 0; k < n; ++k) rmax = fmax(rmax, 2.0 * h[k]);
    int64_t nb = (int64_t)floor(box->size / (rmax * 1.000001));
    if (nb < 1) nb = 1;
    if (nb > 256) nb = 256;
    double w = box->size / (double)nb;
    int64_t nbins = nb * nb * nb;
    int64_t *head = (int64_t *)calloc((size_t)nbins + 1, sizeof(int64_t));
    int64_t *bin = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    int64_t *sorted = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    if (!head || !bin || !sorted) {
        free(head);
        free(bin);
        free(sorted);
        return OR_ENOMEM;
    }
    for (int64_t k = 0; k < n; ++k) {
        int64_t b[3];
        for (int a = 0; a < 3; ++a) {
            int64_t v = (int64_t)floor((xyz[(int64_t)a * n + k] - box->lo[a]) / w);
            b[a] = v < 0 ? 0 : (v >= nb ? nb - 1 : v);
        }
        bin[k] = (b[0] * nb + b[1]) * nb + b[2];
        head[bin[k] + 1]++;
    }
    for (int64_t b = 0; b < nbins; ++b) head[b + 1] += head[b];
    {
        int64_t *fill = (int64_t *)malloc((size_t)nbins * sizeof(int64_t));
        if (!fill) {
            free(head);
            free(bin);
            free(sorted);
            return OR_ENOMEM;
        }
        memcpy(fill, head, (size_t)nbins * sizeof(int64_t));
        for (int64_t k = 0; k < n; ++k) sorted[fill[bin[k]]++] = k;
        free(fill);
    }
    int err = 0;
#pragma omp parallel
    {
        int64_t cap = 1024;
        int64_t *cand = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
        if (!cand) {
#pragma omp atomic write
            err = 1;
        }
#pragma omp for schedule(dynamic, 256)
        for (int64_t lin = 0; lin < ncell; ++lin) {
            if (!cand) continue;
            double xc[3];
            cell_centre(box, G, lin, xc);
            int64_t cb[3];
            for (int a = 0; a < 3; ++a) {
                int64_t v = (int64_t)floor((xc[a] - box->lo[a]) / w);
                cb[a] = v < 0 ? 0 : (v >= nb ? nb - 1 : v);
            }
            int64_t m = 0;
            for (int64_t i0 = cb[0] - 1; i0 <= cb[0] + 1; ++i0)
                for (int64_t i1 = cb[1] - 1; i1 <= cb[1] + 1; ++i1)
                    for (int64_t i2 = cb[2] - 1; i2 <= cb[2] + 1; ++i2) {
                        if (i0 < 0 || i1 < 0 || i2 < 0 || i0 >= nb || i1 >= nb || i2 >= nb)
                            continue;
                        int64_t b = (i0 * nb + i1) * nb + i2;
                        for (int64_t s = head[b]; s < head[b + 1]; ++s) {
                            int64_t k = sorted[s];
                            if (dist3(xc, xyz, n, k) < 2.0 * h[k]) {
                                if (m == cap) {
                                    int64_t *p = (int64_t *)realloc(cand, (size_t)(2 * cap) * sizeof(int64_t));
                                    if (!p) {
#pragma omp atomic write
                                        err = 1;
                                        goto next_cell;
                                    }
                                    cand = p;
                                    cap *= 2;
                                }
                                cand[m++] = k;
                            }
                        }
                    }
            qsort(cand, (size_t)m, sizeof(int64_t), cmp_i64);
            {
                double num = 0.0, den = 0.0;
                for (int64_t s = 0; s < m; ++s) {
                    int64_t k = cand[s];
                    double wk = or_kernel_w(dist3(xc, xyz, n, k), h[k]);
                    num += nhi[k] * wk;
                    den += wk;
                }
                out[lin] = den > 0.0 ? num / den : 0.0;
            }
        next_cell:;
        }
        free(cand);
    }
    free(head);
    free(bin);
    free(sorted);
    return err ? OR_ENOMEM : OR_OK;
}

int or_grid_cells(const or_box *box, int64_t n, const double *xyz, const double *h,
                  const double *nhi, int grid_log2, int64_t m, const int64_t *cells,
                  double *out)
{
    int rc = check_gas(box, n, xyz, h, nhi, grid_log2);
    if (rc) return rc;
    const int G = 1 << grid_log2;
    const int64_t ncell = (int64_t)G * G * G;
    if (m < 0 || (m > 0 && (!cells || !out))) return OR_EINVAL;
    for (int64_t s = 0; s < m; ++s)
        if (cells[s] < 0 || cells[s] >= ncell) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < m; ++s) {
        double xc[3];
        cell_centre(box, G, cells[s], xc);
        double num = 0.0, den = 0.0;
        for (int64_t k = 0; k < n; ++k) {
            double wk = or_kernel_w(dist3(xc, xyz, n, k), h[k]);
            num += nhi[k] * wk;
            den += wk;
        }
        out[s] = den > 0.0 ? num / den : 0.0;
    }
    return OR_OK;
}

/* ----------------------------------------------------------- ray column --- */

static int cmp_dbl(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Exact integral of the piecewise-constant grid field along a -> b.  In grid
 * units g = (x - lo) G / size the ray is P(t) = A + t (B - A), t in [0, 1].
 * Every crossing of an integer plane splits it; each piece lies in the cell
 * holding its midpoint and contributes n_cell * (t_b - t_a).  The sum times
 * |b - a| is the column in cm^-3 x length units. */
static double column_buf(const or_box *box, int grid_log2, const double *grid, const double a[3],
                         const double b[3], int64_t *ncells, double *ts)
{
    const int G = 1 << grid_log2;
    const double s = (double)G / box->size;
    double A[3], B[3], D[3];
    for (int k = 0; k < 3; ++k) {
        A[k] = (a[k] - box->lo[k]) * s;
        B[k] = (b[k] - box->lo[k]) * s;
        D[k] = B[k] - A[k];
    }
    int64_t m = 0;
    ts[m++] = 0.0;
    ts[m++] = 1.0;
    for (int k = 0; k < 3; ++k) {
        if (D[k] == 0.0) continue;
        double lo = A[k] < B[k] ? A[k] : B[k];
        double hi = A[k] < B[k] ? B[k] : A[k];
        for (double p = floor(lo) + 1.0; p < hi; p += 1.0) {
            double t = (p - A[k]) / D[k];
            if (t > 0.0 && t < 1.0) ts[m++] = t;
        }
    }
    qsort(ts, (size_t)m, sizeof(double), cmp_dbl);
    double sum = 0.0;
    int64_t nc = 0;
    for (int64_t q = 0; q + 1 < m; ++q) {
        double ta = ts[q], tb = ts[q + 1];
        if (!(tb > ta)) continue;
        double tm = 0.5 * (ta + tb);
        int64_t c[3];
        for (int k = 0; k < 3; ++k) {
            double p = A[k] + tm * D[k];
            int64_t v = (int64_t)floor(p);
            c[k] = v < 0 ? 0 : (v >= G ? G - 1 : v);
        }
        sum += grid[(c[0] * G + c[1]) * G + c[2]] * (tb - ta);
        ++nc;
    }
    if (ncells) *ncells = nc;
    double dx = b[0] - a[0], dy = b[1] - a[1], dz = b[2] - a[2];
    return sum * sqrt(dx * dx + dy * dy + dz * dz);
}

double or_column(const or_box *box, int grid_log2, const double *grid, const double a[3],
                 const double b[3], int64_t *ncells)
{
    const int G = 1 << grid_log2;
    double *ts = (double *)malloc((size_t)(3 * G + 4) * sizeof(double));
    if (!ts) return NAN;
    double v = column_buf(box, grid_log2, grid, a, b, ncells, ts);
    free(ts);
    return v;
}

/* --------------------------------------------------------------- rates --- */

int or_rates(const or_tree *t, int grid_log2, const double *grid, int64_t n_t,
             const double *tgt_xyz, const int64_t *self_src, double theta, double sigma,
             double *gamma_out, int64_t *counters, int nthreads)
{
    if (!t || !gamma_out || grid_log2 < 0 || grid_log2 > 10 || !grid) return OR_EINVAL;
    if (!isfinite(sigma)) return OR_ENONFINITE;
    if (sigma < 0.0) return OR_EINVAL;
    int rc = check_targets(&t->box, n_t, tgt_xyz, self_src, t->n, theta);
    if (rc) return rc;
    const int G = 1 << grid_log2;
    const double ucm = t->box.unit_cm;
    const double four_pi = 4.0 * M_PI;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        or_list L = {0};
        double *ts = (double *)malloc((size_t)(3 * G + 4) * sizeof(double));
        if (!ts) {
#pragma omp atomic write
            err = OR_ENOMEM;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n_t; ++i) {
            if (!ts) continue;
            double x[3] = {tgt_xyz[i], tgt_xyz[n_t + i], tgt_xyz[2 * n_t + i]};
            if (list_for(t, x, self_src ? self_src[i] : -1, theta, &L) != OR_OK) {
#pragma omp atomic write
                err = OR_ENOMEM;
                continue;
            }
            double sum = 0.0;
            int64_t ncell_tot = 0, nzero = 0;
            for (int64_t e = 0; e < L.n; ++e) {
                const double *r;
                double ra[3], La;
                if (L.e[e].cell >= 0) {
                    const or_cell *c = &t->cells[L.e[e].cell];
                    r = c->com;
                    La = c->lum;
                } else {
                    int64_t j = L.e[e].src;
                    for (int k = 0; k < 3; ++k) ra[k] = t->x[(int64_t)k * t->n + j];
                    r = ra;
                    La = t->lum[j];
                }
                double dx = x[0] - r[0], dy = x[1] - r[1], dz = x[2] - r[2];
                double dist = sqrt(dx * dx + dy * dy + dz * dz);
                if (dist == 0.0) {
                    ++nzero;
                    continue;
                }
                int64_t nc = 0;
                double col = column_buf(&t->box, grid_log2, grid, r, x, &nc, ts);
                ncell_tot += nc;
                double tau = sigma * col * ucm;
                double dcm = dist * ucm;
                sum += La * exp(-tau) / (dcm * dcm);
            }
            gamma_out[i] = sigma / four_pi * sum;
            if (counters) {
                counters[4 * i + 0] = L.ntest;
                counters[4 * i + 1] = L.n;
                counters[4 * i + 2] = ncell_tot;
                counters[4 * i + 3] = nzero;
            }
        }
        free(ts);
        free(L.e);
    }
    return err;
}

/* H2 self-shielding function of Appendix B (eq. B2): 1 up to a column of
 * 1e14 cm^-2, then (N / 1e14)^(-3/4). */
double or_fsh(double x)
{
    return x <= 1.0 ? 1.0 : pow(x, -0.75);
}

int or_lw_rates(const or_tree *t, int grid_log2, const double *grid, int64_t n_t,
                const double *tgt_xyz, const int64_t *self_src, double theta,
                double *kdis_out, int nthreads)
{
    if (!t || !kdis_out || grid_log2 < 0 || grid_log2 > 10 || !grid) return OR_EINVAL;
    int rc = check_targets(&t->box, n_t, tgt_xyz, self_src, t->n, theta);
    if (rc) return rc;
    const int G = 1 << grid_log2;
    const double ucm = t->box.unit_cm;
    const double four_pi = 4.0 * M_PI;
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
#pragma omp parallel
    {
        or_list L = {0};
        double *ts = (double *)malloc((size_t)(3 * G + 4) * sizeof(double));
        if (!ts) {
#pragma omp atomic write
            err = OR_ENOMEM;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n_t; ++i) {
            if (!ts) continue;
            double x[3] = {tgt_xyz[i], tgt_xyz[n_t + i], tgt_xyz[2 * n_t + i]};
            if (list_for(t, x, self_src ? self_src[i] : -1, theta, &L) != OR_OK) {
#pragma omp atomic write
                err = OR_ENOMEM;
                continue;
            }
            double sum = 0.0;
            for (int64_t e = 0; e < L.n; ++e) {
                const double *r;
                double ra[3], La;
                if (L.e[e].cell >= 0) {
                    const or_cell *c = &t->cells[L.e[e].cell];
                    r = c->com;
                    La = c->lum;
                } else {
                    int64_t j = L.e[e].src;
                    for (int k = 0; k < 3; ++k) ra[k] = t->x[(int64_t)k * t->n + j];
                    r = ra;
                    La = t->lum[j];
                }
                double dx = x[0] - r[0], dy = x[1] - r[1], dz = x[2] - r[2];
                double dist = sqrt(dx * dx + dy * dy + dz * dz);
                if (dist == 0.0) continue;
                int64_t nc = 0;
                /* H2 column in cm^-2 along the ray, unshielded flux L / (4 pi d^2) */
                double col = column_buf(&t->box, grid_log2, grid, r, x, &nc, ts) * ucm;
                double dcm = dist * ucm;
                sum += La / (four_pi * dcm * dcm) * or_fsh(col / 1e14);
            }
            kdis_out[i] = 1.13e8 * sum;
        }
        free(ts);
        free(L.e);
    }
    return err;
}

/* ------------------------------------------------ upstream-particle chain --- */

typedef struct {
    int64_t id;    /* virtual source: cell index; individual source: ncells + index */
    int64_t pos;   /* position in the target's list */
} or_idpos;

static int cmp_idpos(const void *a, const void *b)
{
    const or_idpos *x = (const or_idpos *)a, *y = (const or_idpos *)b;
    return x->id < y->id ? -1 : (x->id > y->id ? 1 : 0);
}

static int cmp_i64v(const void *a, const void *b)
{
    const int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return x < y ? -1 : (x > y ? 1 : 0);
}

/* Cell list over the box for the neighbour search: M^3 cubic cells of side
 * at least the largest 2h (at most 128 per axis), particles counting-sorted
 * by cell in index order. */
typedef struct {
    int M;
    double side;
    int64_t *start;   /* [M^3 + 1] */
    int64_t *order;   /* [n] */
} or_cells;

static int cell_axis(double x, double lo, double side, int M)
{
    const double f = floor((x - lo) / side);
    return f < 0.0 ? 0 : (f > (double)(M - 1) ? M - 1 : (int)f);
}

static int cells_build(const or_box *box, int64_t n, const double *xyz, const double *h, or_cells *cl)
{
    double rmax = 0.0;
    for (int64_t i = 0; i < n; ++i) rmax = 2.0 * h[i] > rmax ? 2.0 * h[i] : rmax;
    int M = rmax > 0.0 ? (int)floor(box->size / rmax) : 128;
    M = M < 1 ? 1 : (M > 128 ? 128 : M);
    cl->M = M;
    cl->side = box->size / M;
    const int64_t nc = (int64_t)M * M * M;
    cl->start = (int64_t *)calloc((size_t)nc + 1, sizeof(int64_t));
    cl->order = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    int64_t *cell = (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
    if (!cl->start || !cl->order || !cell) {
        free(cl->start); free(cl->order); free(cell);
        return OR_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        int a[3];
        for (int k = 0; k < 3; ++k) a[k] = cell_axis(xyz[(int64_t)k * n + i], box->lo[k], cl->side, M);
        cell[i] = ((int64_t)a[0] * M + a[1]) * M + a[2];
        cl->start[cell[i] + 1]++;
    }
    for (int64_t c = 0; c < nc; ++c) cl->start[c + 1] += cl->start[c];
    int64_t *fill = (int64_t *)malloc((size_t)nc * sizeof(int64_t));
    if (!fill) { free(cl->start); free(cl->order); free(cell); return OR_ENOMEM; }
    memcpy(fill, cl->start, (size_t)nc * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) cl->order[fill[cell[i]]++] = i;
    free(fill);
    free(cell);
    return OR_OK;
}

/* Every particle in the cells that a ball of radius r around x can touch,
 * with one cell of margin on each side (the cell of a point is found by a
 * rounded division), in increasing index.  Returns the count. */
static int64_t cells_candidates(const or_cells *cl, const or_box *box, const double x[3], double r, int64_t *out)
{
    int a0[3], a1[3];
    for (int k = 0; k < 3; ++k) {
        a0[k] = cell_axis(x[k] - r, box->lo[k], cl->side, cl->M) - 1;
        a1[k] = cell_axis(x[k] + r, box->lo[k], cl->side, cl->M) + 1;
        a0[k] = a0[k] < 0 ? 0 : a0[k];
        a1[k] = a1[k] > cl->M - 1 ? cl->M - 1 : a1[k];
    }
    int64_t m = 0;
    for (int a = a0[0]; a <= a1[0]; ++a)
        for (int b = a0[1]; b <= a1[1]; ++b)
            for (int c = a0[2]; c <= a1[2]; ++c) {
                const int64_t cell = ((int64_t)a * cl->M + b) * cl->M + c;
                for (int64_t s = cl->start[cell]; s < cl->start[cell + 1]; ++s) out[m++] = cl->order[s];
            }
    qsort(out, (size_t)m, sizeof(int64_t), cmp_i64v);
    return m;
}

int or_upstream_rates(const or_tree *t, int grid_log2, const double *grid, int64_t n,
                      const double *xyz, const double *h, const double *nhi,
                      const int64_t *self_src, double theta, double sigma,
                      double *gamma_out, int64_t *offsets_out, int64_t *parent_out,
                      int64_t capacity, int64_t *stats)
{
    return or_upstream_rates_ex(t, grid_log2, grid, n, xyz, h, nhi, self_src, theta, sigma, gamma_out, offsets_out,
                                parent_out, capacity, stats, 0);
}

int or_upstream_rates_ex(const or_tree *t, int grid_log2, const double *grid, int64_t n,
                         const double *xyz, const double *h, const double *nhi,
                         const int64_t *self_src, double theta, double sigma,
                         double *gamma_out, int64_t *offsets_out, int64_t *parent_out,
                         int64_t capacity, int64_t *stats, int all_pairs)
{
    or_cells cl = {0, 0.0, NULL, NULL};
    if (!t || !gamma_out || !grid || !h || !nhi || grid_log2 < 0 || grid_log2 > 10) return OR_EINVAL;
    if (!isfinite(sigma)) return OR_ENONFINITE;
    if (sigma < 0.0) return OR_EINVAL;
    int rc = check_targets(&t->box, n, xyz, self_src, t->n, theta);
    if (rc) return rc;
    const double ucm = t->box.unit_cm;
    const int G = 1 << grid_log2;
    /* 1. the interaction list of every particle (eqs. 12-13) */
    int64_t *off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t cap = 1024, E = 0;
    int64_t *ids = (int64_t *)malloc((size_t)cap * sizeof(int64_t));
    if (!off || !ids) { free(off); free(ids); return OR_ENOMEM; }
    or_list L = {0};
    for (int64_t i = 0; i < n; ++i) {
        double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
        rc = list_for(t, x, self_src ? self_src[i] : -1, theta, &L);
        if (rc) break;
        if (E + L.n > cap) {
            while (E + L.n > cap) cap *= 2;
            int64_t *p = (int64_t *)realloc(ids, (size_t)cap * sizeof(int64_t));
            if (!p) { rc = OR_ENOMEM; break; }
            ids = p;
        }
        for (int64_t k = 0; k < L.n; ++k)
            ids[E + k] = L.e[k].cell >= 0 ? L.e[k].cell : t->ncells + L.e[k].src;
        E += L.n;
        off[i + 1] = E;
    }
    free(L.e);
    if (rc) { free(off); free(ids); return rc; }
    if (offsets_out) memcpy(offsets_out, off, ((size_t)n + 1) * sizeof(int64_t));
    if (parent_out && E > capacity) { free(off); free(ids); return OR_ECAPACITY; }

    /* per pair: source position, luminosity, distance to the particle */
    double *ra = (double *)malloc((size_t)(E ? E : 1) * 3 * sizeof(double));
    double *La = (double *)malloc((size_t)(E ? E : 1) * sizeof(double));
    double *dist = (double *)malloc((size_t)(E ? E : 1) * sizeof(double));
    int64_t *par = (int64_t *)malloc((size_t)(E ? E : 1) * sizeof(int64_t));
    double *tau = (double *)malloc((size_t)(E ? E : 1) * sizeof(double));
    char *done = (char *)calloc((size_t)(E ? E : 1), 1);
    or_idpos *sorted = (or_idpos *)malloc((size_t)(E ? E : 1) * sizeof(or_idpos));
    double *ts = (double *)malloc((size_t)(3 * G + 4) * sizeof(double));
    int64_t *stack = (int64_t *)malloc((size_t)(E ? E : 1) * sizeof(int64_t));
    if (!ra || !La || !dist || !par || !tau || !done || !sorted || !ts || !stack) { rc = OR_ENOMEM; goto out; }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
        for (int64_t p = off[i]; p < off[i + 1]; ++p) {
            const int64_t id = ids[p];
            if (id < t->ncells) {
                const or_cell *c = &t->cells[id];
                for (int k = 0; k < 3; ++k) ra[3 * p + k] = c->com[k];
                La[p] = c->lum;
            } else {
                const int64_t j = id - t->ncells;
                for (int k = 0; k < 3; ++k) ra[3 * p + k] = t->x[(int64_t)k * t->n + j];
                La[p] = t->lum[j];
            }
            const double dx = x[0] - ra[3 * p], dy = x[1] - ra[3 * p + 1], dz = x[2] - ra[3 * p + 2];
            dist[p] = sqrt(dx * dx + dy * dy + dz * dz);
            sorted[p].id = id;
            sorted[p].pos = p;
        }
        qsort(sorted + off[i], (size_t)(off[i + 1] - off[i]), sizeof(or_idpos), cmp_idpos);
    }

    /* 2-3. the upstream particle of every (particle, source) pair: among the
     * particle's neighbours (within its 2h) that are closer to the same
     * (virtual) source and have it in their own list, the one nearest to the
     * ray (largest cos phi; the lowest index on ties).  None: the pair is a
     * list-boundary particle and integrates along the ray. */
    if (!all_pairs) {
        rc = cells_build(&t->box, n, xyz, h, &cl);
        if (rc) goto out;
    }
    int failed = 0;
#pragma omp parallel
    {
        int64_t *cand = all_pairs ? NULL : (int64_t *)malloc((size_t)(n ? n : 1) * sizeof(int64_t));
        double *best = NULL;
        int64_t best_cap = 0;
        if (!all_pairs && !cand) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < n; ++i) {
            if (failed) continue;
            const double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
            const double r2 = (2.0 * h[i]) * (2.0 * h[i]);
            for (int64_t p = off[i]; p < off[i + 1]; ++p) par[p] = -1;
            if (off[i + 1] - off[i] + 1 > best_cap) {
                free(best);
                best_cap = off[i + 1] - off[i] + 1;
                best = (double *)malloc((size_t)best_cap * sizeof(double));
                if (!best) {
                    best_cap = 0;
#pragma omp atomic write
                    failed = 1;
                    continue;
                }
            }
            const int64_t m = all_pairs ? n : cells_candidates(&cl, &t->box, x, 2.0 * h[i], cand);
            for (int64_t k = 0; k < m; ++k) {
                const int64_t j = all_pairs ? k : cand[k];
                if (j == i) continue;
                const double ex = xyz[j] - x[0], ey = xyz[n + j] - x[1], ez = xyz[2 * n + j] - x[2];
                if (!(ex * ex + ey * ey + ez * ez <= r2)) continue;       /* not a neighbour */
                const double y[3] = {xyz[j], xyz[n + j], xyz[2 * n + j]};
                for (int64_t p = off[i]; p < off[i + 1]; ++p) {
                    or_idpos key = {ids[p], 0};
                    const or_idpos *f = (const or_idpos *)bsearch(&key, sorted + off[j],
                                                                  (size_t)(off[j + 1] - off[j]), sizeof(or_idpos),
                                                                  cmp_idpos);
                    if (!f) continue;                                     /* not in the same list */
                    const int64_t q = f->pos;
                    if (!(dist[q] < dist[p])) continue;                   /* not upstream */
                    const double *a = ra + 3 * p;
                    const double dot = (x[0] - a[0]) * (y[0] - a[0]) + (x[1] - a[1]) * (y[1] - a[1]) +
                                       (x[2] - a[2]) * (y[2] - a[2]);
                    const double cphi = dot / (dist[p] * dist[q]);
                    if (par[p] < 0 || cphi > best[p - off[i]]) {
                        par[p] = q;
                        best[p - off[i]] = cphi;
                    }
                }
            }
        }
        free(best);
        free(cand);
    }
    if (failed) { rc = OR_ENOMEM; goto out; }

    /* 4. optical depths: tau = tau_up + sigma dl (n_target + n_up) / 2
     * (eqs. 8-9), dl = d_target - d_up; a pair without an upstream particle
     * integrates the column along the ray (exact, through the grid). */
    for (int64_t p0 = 0; p0 < E; ++p0) {
        int64_t sp = 0, p = p0;
        while (p >= 0 && !done[p]) {
            stack[sp++] = p;
            p = par[p];
        }
        while (sp > 0) {
            p = stack[--sp];
            /* target particle of pair p */
            int64_t lo = 0, hi = n;
            while (hi - lo > 1) {
                int64_t mid = (lo + hi) / 2;
                if (off[mid] <= p) lo = mid; else hi = mid;
            }
            const int64_t i = lo;
            const double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
            if (par[p] < 0) {
                if (dist[p] == 0.0) {
                    tau[p] = 0.0;
                } else {
                    int64_t nc = 0;
                    tau[p] = sigma * column_buf(&t->box, grid_log2, grid, ra + 3 * p, x, &nc, ts) * ucm;
                }
            } else {
                const int64_t q = par[p];
                int64_t lo2 = 0, hi2 = n;
                while (hi2 - lo2 > 1) {
                    int64_t mid = (lo2 + hi2) / 2;
                    if (off[mid] <= q) lo2 = mid; else hi2 = mid;
                }
                const int64_t j = lo2;
                tau[p] = tau[q] + sigma * ((dist[p] - dist[q]) * ucm) * (0.5 * (nhi[i] + nhi[j]));
            }
            done[p] = 1;
        }
    }

    /* 5. the rate per H I atom (eq. A2) with these optical depths */
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double sum = 0.0;
        int64_t roots = 0;
        for (int64_t p = off[i]; p < off[i + 1]; ++p) {
            if (par[p] < 0) ++roots;
            if (dist[p] == 0.0) continue;
            const double dcm = dist[p] * ucm;
            sum += La[p] * exp(-tau[p]) / (dcm * dcm);
        }
        gamma_out[i] = sigma / (4.0 * M_PI) * sum;
        if (stats) {
            stats[2 * i] = off[i + 1] - off[i];
            stats[2 * i + 1] = roots;
        }
    }
    if (parent_out) {
        /* parent as the upstream particle's index (-1: integrated along the ray) */
        for (int64_t p = 0; p < E; ++p) {
            if (par[p] < 0) { parent_out[p] = -1; continue; }
            int64_t lo = 0, hi = n;
            while (hi - lo > 1) {
                int64_t mid = (lo + hi) / 2;
                if (off[mid] <= par[p]) lo = mid; else hi = mid;
            }
            parent_out[p] = lo;
        }
    }
out:
    free(off); free(ids); free(ra); free(La); free(dist); free(par); free(tau); free(done);
    free(sorted); free(ts); free(stack);
    free(cl.start); free(cl.order);
    return rc;
}
