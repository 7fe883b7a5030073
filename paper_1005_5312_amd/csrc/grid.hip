// Neutral-hydrogen field for the ray integrals, on a G^3 grid over the box.
//
// The paper integrates the optical depth along each light ray through the SPH
// particles (sections 2.2.1-2.2.2).  Here the field is first interpolated to
// the grid cell centres with the SPH kernel of section 2.1 (cubic spline,
// support 2h) in Shepard-normalised form,
//     n_c = sum_k n_k W(|x_c - r_k|, h_k) / sum_k W(|x_c - r_k|, h_k),
// 0 where no kernel reaches, and every ray then integrates the piecewise-
// constant field exactly.  Particles are counting-sorted into the grid cells
// (stable, so sums run in a fixed order) and each cell centre gathers from
// the cells within the largest kernel radius.
#include "internal.h"

#include <cstring>

namespace start {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

__global__ void __launch_bounds__(kThreads) grid_keys(start_box box, double gs, int G, int64_t n,
                                                      const double *xyz, const double *h, const double *nhi,
                                                      uint64_t *keys, unsigned *idx, unsigned *flags,
                                                      unsigned long long *hmax_bits)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    unsigned bad = 0;
    int c[3];
    for (int a = 0; a < 3; ++a) {
        const double x = xyz[(int64_t)a * n + k];
        if (!isfinite(x)) bad |= kFlagNonFinite;
        else if (x < box.lo[a] || x > box.lo[a] + box.size) bad |= kFlagOutOfBox;
        double g = isfinite(x) ? (x - box.lo[a]) * gs : 0.0;
        int v = (int)floor(g);
        c[a] = v < 0 ? 0 : (v >= G ? G - 1 : v);
    }
    const double hk = h[k], nk = nhi[k];
    if (!isfinite(hk) || !isfinite(nk)) bad |= kFlagNonFinite;
    else if (!(hk > 0.0) || nk < 0.0) bad |= kFlagNegative;
    if (bad) atomicOr(flags, bad);
    else atomicMax(hmax_bits, (unsigned long long)__double_as_longlong(2.0 * hk));
    keys[k] = ((uint64_t)c[0] * G + c[1]) * G + c[2];
    idx[k] = (unsigned)k;
}

__global__ void __launch_bounds__(kThreads) cell_counts(const uint64_t *keys, int64_t n, unsigned *start)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    atomicAdd(&start[keys[k]], 1u);
}

__global__ void __launch_bounds__(kThreads) gather_particles(int64_t n, const unsigned *perm, const double *xyz,
                                                             const double *h, const double *nhi, double4 *pos_h,
                                                             double2 *kern, double *ns)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const unsigned o = perm[k];
    const double hk = h[o];
    pos_h[k] = make_double4(xyz[o], xyz[n + o], xyz[2 * n + o], hk);
    // 1/h and the 3-D normalisation 1/(pi h^3) of the kernel, once per particle
    kern[k] = make_double2(1.0 / hk, 1.0 / (M_PI * hk * hk * hk));
    ns[k] = nhi[o];
}

__global__ void __launch_bounds__(kThreads) gather_values(int64_t n, const unsigned *perm, const double *nhi,
                                                          double *ns)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    ns[k] = nhi[perm[k]];
}

// M4 cubic spline of section 2.1 with 3-D normalisation 1/(pi h^3), from
// q = r / h and the normalisation.
__device__ inline double kernel_w(double q, double norm)
{
    double f;
    if (q <= 1.0)
        f = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    else if (q <= 2.0)
        f = 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
    else
        f = 0.0;
    return f * norm;
}

__global__ void __launch_bounds__(kThreads) shepard_gather(start_box box, double delta, int G, int R,
                                                           double reach, const unsigned *start,
                                                           const double4 *__restrict__ pos_h,
                                                           const double2 *__restrict__ kern,
                                                           const double *__restrict__ ns, double *val, float *valf,
                                                           int sx, int sy)
{
    const int64_t lin = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t ncell = (int64_t)G * G * G;
    if (lin >= ncell) return;
    const int ia = (int)(lin / ((int64_t)G * G)), ib = (int)((lin / G) % G), ic = (int)(lin % G);
    const double xc = box.lo[0] + ((double)ia + 0.5) * delta;
    const double yc = box.lo[1] + ((double)ib + 0.5) * delta;
    const double zc = box.lo[2] + ((double)ic + 0.5) * delta;
    double num = 0.0, den = 0.0;
    const int a0 = ia - R < 0 ? 0 : ia - R, a1 = ia + R >= G ? G - 1 : ia + R;
    const int b0 = ib - R < 0 ? 0 : ib - R, b1 = ib + R >= G ? G - 1 : ib + R;
    const int c0 = ic - R < 0 ? 0 : ic - R, c1 = ic + R >= G ? G - 1 : ic + R;
    const double reach2 = reach * reach;
    for (int a = a0; a <= a1; ++a) {
        const int da = a < ia ? ia - a - 1 : (a > ia ? a - ia - 1 : 0);
        for (int b = b0; b <= b1; ++b) {
            const int db = b < ib ? ib - b - 1 : (b > ib ? b - ib - 1 : 0);
            // skip rows of cells entirely beyond the largest kernel reach,
            // and trim the row to the cells the reach can touch
            const double dab2 = (double)(da * da + db * db) * delta * delta;
            if (dab2 > reach2) continue;
            const int rz = (int)(sqrt(reach2 - dab2) / delta) + 1;
            const int z0 = ic - rz > c0 ? ic - rz : c0, z1 = ic + rz < c1 ? ic + rz : c1;
            const int64_t row = ((int64_t)a * G + b) * G;
            const unsigned s0 = start[row + z0], s1 = start[row + z1 + 1];
            for (unsigned s = s0; s < s1; ++s) {
                const double4 p = pos_h[s];
                const double dx = xc - p.x, dy = yc - p.y, dz = zc - p.z;
                const double r2 = dx * dx + dy * dy + dz * dz;
                if (r2 < 4.0 * p.w * p.w) {   // inside the support 2h
                    const double2 k = kern[s];
                    const double w = kernel_w(sqrt(r2) * k.x, k.y);
                    num += ns[s] * w;
                    den += w;
                }
            }
        }
    }
    const double v = den > 0.0 ? num / den : 0.0;
    const int64_t e = (int64_t)ia * sx + (int64_t)ib * sy + ic;
    val[e] = v;
    valf[e] = (float)v;
}

__global__ void __launch_bounds__(kThreads) unpad(int G, int sx, int sy, const double *val, double *out)
{
    const int64_t lin = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (lin >= (int64_t)G * G * G) return;
    const int ia = (int)(lin / ((int64_t)G * G)), ib = (int)((lin / G) % G), ic = (int)(lin % G);
    out[lin] = val[(int64_t)ia * sx + (int64_t)ib * sy + ic];
}

}  // namespace

start_status bin_gas(Ctx *c, const start_box &box, int64_t n, const double *xyz, const double *h,
                     const double *nhi, int grid_log2, GasBins *b)
{
    hipStream_t s = c->stream;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int G = 1 << grid_log2;
    const int64_t ncell = (int64_t)G * G * G;
    *b = GasBins();
    b->box = box;
    b->n = n;
    b->G = G;
    b->delta = box.size / G;
    if (n == 0) return START_OK;
    const int64_t nk = n;
    b->bytes = al(radix_temp_bytes(nk)) + al(nk * sizeof(uint64_t)) + al(nk * sizeof(unsigned)) +
               al((ncell + 1) * sizeof(unsigned)) + al(scan_temp_bytes(ncell + 1)) + al(nk * sizeof(double4)) +
               al(nk * sizeof(double2)) + al(nk * sizeof(double)) + 256;
    if (dmalloc(c, (void **)&b->mem, b->bytes) != hipSuccess) {
        b->mem = nullptr;
        return START_ENOMEM;
    }
    char *q = b->mem;
    auto take = [&](size_t v) { char *r = q; q += al(v); return r; };
    void *radix_tmp = take(radix_temp_bytes(nk));
    uint64_t *keys = (uint64_t *)take(nk * sizeof(uint64_t));
    b->idx = (unsigned *)take(nk * sizeof(unsigned));
    b->start = (unsigned *)take((ncell + 1) * sizeof(unsigned));
    void *scan_tmp = take(scan_temp_bytes(ncell + 1));
    b->pos_h = (double4 *)take(nk * sizeof(double4));
    b->kern = (double2 *)take(nk * sizeof(double2));
    b->ns = (double *)take(nk * sizeof(double));
    unsigned long long *hmax = (unsigned long long *)take(256);

    const double gs = (double)G / box.size;
    unsigned *bflags = c->d_flags + 1;   // build validation word (not the rate calls' one)
    hipMemsetAsync(bflags, 0, sizeof(unsigned), s);
    hipMemsetAsync(hmax, 0, sizeof(unsigned long long), s);
    grid_keys<<<blocks_for(n), kThreads, 0, s>>>(box, gs, G, n, xyz, h, nhi, keys, b->idx, bflags, hmax);
    radix_sort_pairs(keys, b->idx, n, 3 * grid_log2, radix_tmp, s);
    hipMemsetAsync(b->start, 0, (ncell + 1) * sizeof(unsigned), s);
    cell_counts<<<blocks_for(n), kThreads, 0, s>>>(keys, n, b->start);
    exclusive_scan_u32(b->start, ncell + 1, scan_tmp, s);
    gather_particles<<<blocks_for(n), kThreads, 0, s>>>(n, b->idx, xyz, h, nhi, b->pos_h, b->kern, b->ns);
    unsigned flags = 0;
    unsigned long long hbits = 0;
    hipMemcpyAsync(&flags, bflags, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(&hbits, hmax, sizeof(hbits), hipMemcpyDeviceToHost, s);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess || flags) {
        free_bins(c, b);
        if (e != hipSuccess) { c->err = hipGetErrorString(e); return START_EHIP; }
        if (flags & kFlagNonFinite) { c->err = "non-finite gas position, h or n_HI"; return START_ENONFINITE; }
        if (flags & kFlagOutOfBox) { c->err = "gas particle outside the box"; return START_EOUTOFBOX; }
        c->err = "gas h <= 0 or n_HI < 0";
        return START_EINVAL;
    }
    std::memcpy(&b->reach, &hbits, sizeof(double));
    // a particle can reach a centre only from cells within ceil(reach/delta)
    int R = (int)ceil(b->reach / b->delta);
    b->R = R > G ? G : R;
    return START_OK;
}

void free_bins(Ctx *c, GasBins *b)
{
    dfree(c, b->mem, b->bytes);
    b->mem = nullptr;
    b->bytes = 0;
}

void fill_grid(Ctx *c, const GasBins &b, const double *nhi, Grid *g)
{
    hipStream_t s = c->stream;
    const int64_t ncell = (int64_t)g->G * g->G * g->G;
    if (b.n == 0) {
        hipMemsetAsync(g->val, 0, g->span * sizeof(double), s);
        hipMemsetAsync(g->valf, 0, g->span * sizeof(float), s);
        return;
    }
    if (nhi) gather_values<<<blocks_for(b.n), kThreads, 0, s>>>(b.n, b.idx, nhi, b.ns);
    shepard_gather<<<blocks_for(ncell), kThreads, 0, s>>>(b.box, b.delta, b.G, b.R, b.reach, b.start, b.pos_h,
                                                           b.kern, b.ns, g->val, g->valf, g->sx, g->sy);
}

start_status alloc_grid(Ctx *c, const start_box &box, int grid_log2, Grid *g)
{
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    g->box = box;
    g->grid_log2 = grid_log2;
    const int G = 1 << grid_log2;
    g->G = G;
    const int pad = (G >= 64 && G <= 512) ? 16 : 0;
    g->sy = G + pad;
    g->sx = G * g->sy + pad;
    g->span = (int64_t)(G - 1) * g->sx + (int64_t)(G - 1) * g->sy + G;
    size_t persist = al(g->span * sizeof(double)) + al(g->span * sizeof(float));
    char *pm = nullptr;
    if (dmalloc(c, (void **)&pm, persist) != hipSuccess) return START_ENOMEM;
    g->bytes = persist;
    g->val = (double *)pm;
    g->valf = (float *)(pm + al(g->span * sizeof(double)));
    if (pad) hipMemsetAsync(pm, 0, persist, c->stream);   // the padding is never written again
    return START_OK;
}

start_status build_grid(Ctx *c, const start_box &box, int64_t n, const double *xyz, const double *h,
                        const double *nhi, int grid_log2, Grid *g)
{
    start_status st = alloc_grid(c, box, grid_log2, g);
    if (st) return st;
    GasBins b;
    st = bin_gas(c, box, n, xyz, h, nhi, grid_log2, &b);
    if (st) {
        dfree(c, g->val, g->bytes);
        return st;
    }
    fill_grid(c, b, nullptr, g);   // the binning already gathered n_HI
    hipError_t e = hipStreamSynchronize(c->stream);
    free_bins(c, &b);
    if (e != hipSuccess) {
        c->err = hipGetErrorString(e);
        dfree(c, g->val, g->bytes);
        return START_EHIP;
    }
    return START_OK;
}

void launch_grid_unpad(Ctx *c, const Grid &g, double *out)
{
    const int64_t n = (int64_t)g.G * g.G * g.G;
    unpad<<<blocks_for(n), kThreads, 0, c->stream>>>(g.G, g.sx, g.sy, g.val, out);
}

}  // namespace start
