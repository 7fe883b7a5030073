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
                                                             double *ns)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const unsigned o = perm[k];
    pos_h[k] = make_double4(xyz[o], xyz[n + o], xyz[2 * n + o], h[o]);
    ns[k] = nhi[o];
}

// M4 cubic spline of section 2.1 with 3-D normalisation 1/(pi h^3).
__device__ inline double kernel_w(double r, double h)
{
    const double q = r / h;
    double f;
    if (q <= 1.0)
        f = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    else if (q <= 2.0)
        f = 0.25 * (2.0 - q) * (2.0 - q) * (2.0 - q);
    else
        f = 0.0;
    return f / (M_PI * h * h * h);
}

__global__ void __launch_bounds__(kThreads) shepard_gather(start_box box, double delta, int G, int R,
                                                           double reach, const unsigned *start,
                                                           const double4 *pos_h, const double *ns,
                                                           double *val, float *valf)
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
    for (int a = a0; a <= a1; ++a) {
        const int da = a < ia ? ia - a - 1 : (a > ia ? a - ia - 1 : 0);
        for (int b = b0; b <= b1; ++b) {
            const int db = b < ib ? ib - b - 1 : (b > ib ? b - ib - 1 : 0);
            // skip rows of cells entirely beyond the largest kernel reach
            if ((double)(da * da + db * db) * delta * delta > reach * reach) continue;
            const int64_t row = ((int64_t)a * G + b) * G;
            const unsigned s0 = start[row + c0], s1 = start[row + c1 + 1];
            for (unsigned s = s0; s < s1; ++s) {
                const double4 p = pos_h[s];
                const double dx = xc - p.x, dy = yc - p.y, dz = zc - p.z;
                const double r = sqrt(dx * dx + dy * dy + dz * dz);
                if (r < 2.0 * p.w) {
                    const double w = kernel_w(r, p.w);
                    num += ns[s] * w;
                    den += w;
                }
            }
        }
    }
    const double v = den > 0.0 ? num / den : 0.0;
    val[lin] = v;
    valf[lin] = (float)v;
}

}  // namespace

start_status build_grid(Ctx *c, const start_box &box, int64_t n, const double *xyz, const double *h,
                        const double *nhi, int grid_log2, Grid *g)
{
    hipStream_t s = c->stream;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    g->box = box;
    g->grid_log2 = grid_log2;
    const int G = 1 << grid_log2;
    g->G = G;
    const int64_t ncell = (int64_t)G * G * G;
    size_t persist = al(ncell * sizeof(double)) + al(ncell * sizeof(float));
    char *pm = nullptr;
    if (dmalloc(c, (void **)&pm, persist) != hipSuccess) return START_ENOMEM;
    g->bytes = persist;
    g->val = (double *)pm;
    g->valf = (float *)(pm + al(ncell * sizeof(double)));
    if (n == 0) {
        hipMemsetAsync(g->val, 0, ncell * sizeof(double), s);
        hipMemsetAsync(g->valf, 0, ncell * sizeof(float), s);
        hipError_t e = hipStreamSynchronize(s);
        return e == hipSuccess ? START_OK : START_EHIP;
    }
    const int64_t nk = n > 1 ? n : 1;
    size_t tmp_bytes = al(radix_temp_bytes(nk)) + al(nk * sizeof(uint64_t)) + al(nk * sizeof(unsigned)) +
                       al((ncell + 1) * sizeof(unsigned)) + al(scan_temp_bytes(ncell + 1)) +
                       al(nk * sizeof(double4)) + al(nk * sizeof(double)) + 256;
    char *tm = nullptr;
    if (dmalloc(c, (void **)&tm, tmp_bytes) != hipSuccess) {
        dfree(c, pm, persist);
        return START_ENOMEM;
    }
    char *q = tm;
    auto take = [&](size_t b) { char *r = q; q += al(b); return r; };
    void *radix_tmp = take(radix_temp_bytes(nk));
    uint64_t *keys = (uint64_t *)take(nk * sizeof(uint64_t));
    unsigned *idx = (unsigned *)take(nk * sizeof(unsigned));
    unsigned *startv = (unsigned *)take((ncell + 1) * sizeof(unsigned));
    void *scan_tmp = take(scan_temp_bytes(ncell + 1));
    double4 *pos_h = (double4 *)take(nk * sizeof(double4));
    double *ns = (double *)take(nk * sizeof(double));
    unsigned long long *hmax = (unsigned long long *)take(256);

    const double gs = (double)G / box.size;
    unsigned *bflags = c->d_flags + 1;   // build validation word (not the rate calls' one)
    hipMemsetAsync(bflags, 0, sizeof(unsigned), s);
    hipMemsetAsync(hmax, 0, sizeof(unsigned long long), s);
    grid_keys<<<blocks_for(n), kThreads, 0, s>>>(box, gs, G, n, xyz, h, nhi, keys, idx, bflags, hmax);
    radix_sort_pairs(keys, idx, n, 3 * grid_log2, radix_tmp, s);
    hipMemsetAsync(startv, 0, (ncell + 1) * sizeof(unsigned), s);
    cell_counts<<<blocks_for(n), kThreads, 0, s>>>(keys, n, startv);
    exclusive_scan_u32(startv, ncell + 1, scan_tmp, s);
    gather_particles<<<blocks_for(n), kThreads, 0, s>>>(n, idx, xyz, h, nhi, pos_h, ns);
    unsigned flags = 0;
    unsigned long long hbits = 0;
    hipMemcpyAsync(&flags, bflags, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(&hbits, hmax, sizeof(hbits), hipMemcpyDeviceToHost, s);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess || flags) {
        dfree(c, tm, tmp_bytes);
        dfree(c, pm, persist);
        if (e != hipSuccess) { c->err = hipGetErrorString(e); return START_EHIP; }
        if (flags & kFlagNonFinite) { c->err = "non-finite gas position, h or n_HI"; return START_ENONFINITE; }
        if (flags & kFlagOutOfBox) { c->err = "gas particle outside the box"; return START_EOUTOFBOX; }
        c->err = "gas h <= 0 or n_HI < 0";
        return START_EINVAL;
    }
    double reach;
    std::memcpy(&reach, &hbits, sizeof(reach));
    const double delta = box.size / G;
    // a particle can reach a centre only from cells within ceil(reach/delta)
    int R = (int)ceil(reach / delta);
    if (R > G) R = G;
    shepard_gather<<<blocks_for(ncell), kThreads, 0, s>>>(box, delta, G, R, reach, startv, pos_h, ns, g->val,
                                                           g->valf);
    e = hipStreamSynchronize(s);
    dfree(c, tm, tmp_bytes);
    if (e != hipSuccess) {
        c->err = hipGetErrorString(e);
        dfree(c, pm, persist);
        return START_EHIP;
    }
    return START_OK;
}

}  // namespace start
