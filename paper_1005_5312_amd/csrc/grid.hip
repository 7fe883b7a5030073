// Neutral-hydrogen field for the ray integrals, on a G^3 grid over the box.
//
// The paper integrates the optical depth along each light ray through the SPH
// particles (sections 2.2.1-2.2.2).  Here the field is first interpolated to
// the grid cell centres with the SPH kernel of section 2.1 (cubic spline,
// support 2h) in Shepard-normalised form,
//     n_c = sum_k n_k W(|x_c - r_k|, h_k) / sum_k W(|x_c - r_k|, h_k),
// 0 where no kernel reaches, and every ray then integrates the piecewise-
// constant field exactly.  Particles are split into a few classes by their
// support 2h (chosen from a histogram of 2h to minimise the scan work) and
// counting-sorted by (class, cell), stable, so sums run in a fixed order;
// each cell centre gathers, class by class, from the cells within that
// class's largest support.
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>

namespace start {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

constexpr int kBins = 256;   // reach bins of a quarter cell; the last also holds every larger reach

// Quarter-cell bin of a particle's kernel support 2h: ceil(4 * 2h / delta).
__device__ inline int reach_bin(double h, double gs)
{
    const double u = ceil(8.0 * h * gs);
    return u < (double)(kBins - 1) ? (int)u : kBins - 1;
}

__global__ void __launch_bounds__(kThreads) grid_keys(start_box box, double gs, int G, int64_t n,
                                                      const double *xyz, const double *h, const double *nhi,
                                                      uint64_t *keys, unsigned *idx, unsigned *flags,
                                                      unsigned *hist, unsigned long long *hmax_bits)
{
    __shared__ unsigned lh[kBins];
    __shared__ double wmax[kThreads / 64];
    for (int t = threadIdx.x; t < kBins; t += kThreads) lh[t] = 0;
    __syncthreads();
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double reach = 0.0;
    int bin = -1;   // reach bin of a valid particle
    if (k < n) {
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
        if (bad) {
            atomicOr(flags, bad);
        } else {
            reach = 2.0 * hk;
            bin = reach_bin(hk, gs);
        }
        keys[k] = ((uint64_t)c[0] * G + c[1]) * G + c[2];
        idx[k] = (unsigned)k;
    }
    // histogram: one LDS atomic per distinct bin of the wave (most particles
    // share one or two bins, and same-address atomics serialise)
    for (;;) {
        const uint64_t left = __ballot(bin >= 0);
        if (!left) break;
        const int b = __shfl(bin, __ffsll((unsigned long long)left) - 1, 64);
        const uint64_t same = __ballot(bin == b);
        if (bin == b) {
            if ((__lane_id() == __ffsll((unsigned long long)same) - 1)) atomicAdd(&lh[b], (unsigned)__popcll(same));
            bin = -1;
        }
    }
    // largest reach of the block, one atomic per block (positive doubles
    // order like their bit patterns)
    for (int o = 32; o > 0; o >>= 1) reach = fmax(reach, __shfl_xor(reach, o, 64));
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = reach;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = wmax[0];
        for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, wmax[w]);
        if (m > 0.0) atomicMax(hmax_bits, (unsigned long long)__double_as_longlong(m));
    }
    for (int t = threadIdx.x; t < kBins; t += kThreads)
        if (lh[t]) atomicAdd(&hist[t], lh[t]);
}

// The validation word, the reach histogram and the largest reach bits,
// copied by one block into the context's pinned readback words (one host
// wait for all three).
__global__ void grid_readback(const unsigned *bflags, const unsigned *hist, const unsigned long long *hmax,
                              unsigned *rb)
{
    for (int k = threadIdx.x; k < kBins; k += blockDim.x) rb[1 + k] = hist[k];
    if (threadIdx.x == 0) {
        rb[0] = *bflags;
        const unsigned long long v = *hmax;
        rb[1 + kBins] = (unsigned)v;
        rb[2 + kBins] = (unsigned)(v >> 32);
    }
}

// Class-major keys: class * G^3 + cell; top.{x,y,z} are the last bins of
// classes 0..2 (kBins where the class is unused).
__global__ void __launch_bounds__(kThreads) class_keys(int64_t n, const double *h, double gs, int64_t ncell,
                                                       int4 top, uint64_t *keys)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const int bin = reach_bin(h[k], gs);
    const int cls = (bin > top.x) + (bin > top.y) + (bin > top.z);
    keys[k] += (uint64_t)cls * (uint64_t)ncell;
}

__global__ void __launch_bounds__(kThreads) cell_counts(const uint64_t *keys, int64_t n, unsigned *start)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    atomicAdd(&start[keys[k]], 1u);
}

__global__ void __launch_bounds__(kThreads) invert_perm(int64_t n, const unsigned *perm, unsigned *inv)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    inv[perm[k]] = (unsigned)k;
}

// The binned particle arrays, written from the particles in input order
// (reads in order, each particle's three records written to its binned
// place; gathering through the permutation instead reads five scattered
// doubles per particle).
__global__ void __launch_bounds__(kThreads) scatter_particles(int64_t n, const unsigned *inv, const double *xyz,
                                                              const double *h, const double *nhi, double4 *pos_h,
                                                              double2 *kern, double *ns)
{
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o >= n) return;
    const unsigned k = inv[o];
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
// q = r / h and the normalisation, without branches: 0.25 (2 - q)^3 less
// (1 - q)^3 below q = 1 is the inner polynomial 1 - 1.5 q^2 + 0.75 q^3, and
// both cubes vanish from q = 2 on.
__device__ inline double kernel_w(double q, double norm)
{
    const double t2 = fmax(2.0 - q, 0.0), t1 = fmax(1.0 - q, 0.0);
    return (0.25 * (t2 * t2 * t2) - t1 * t1 * t1) * norm;
}

// sqrt(x) for 0 <= x (finite): the hardware reciprocal square root and one
// Newton step on the root, ~1e-15 relative (the library sqrt rounds
// correctly but takes ~4x the instructions).  Below 1e-200 the result is
// ~1e-100 instead of x^(1/2): kernel weights are then W(0) either way.
__device__ inline double sqrt_nr(double x)
{
    const double xm = fmax(x, 1e-200);
    const double y = __builtin_amdgcn_rsq(xm);
    const double r = xm * y;
    return fma(0.5 * y, fma(-r, r, xm), r);
}

constexpr int kCellsZ = 4;   // cell centres per thread, consecutive along z

enum ShepardMode { kGather = 0, kCountPairs = 1, kFillPairs = 2 };
constexpr unsigned long long kMaxPairs = 1ull << 29;   // recorded pairs: at most 6 GiB

// kCellsZ consecutive cell centres of one z row per thread: they share x and
// y, so every particle is loaded once for all of them.  Per reach class, the
// rows of cells within the class reach are scanned: a particle in cell
// (a, b, c) is at least (|a - ia| - 1/2)_+ cells from a centre in cell ia
// along x (likewise y, z), so the stencil is the set of cells whose nearest
// point lies within the reach; the row geometry runs in float on a widened
// reach, so the stencil can only grow.  The support test itself is exact
// (FP64), and every centre sums its particles in (class, row, binned) order.
// kCountPairs counts the (centre, particle) pairs inside the support per
// centre; kFillPairs also records them with their weights, in summation
// order, and the weight sums (for refills with new n_HI at the same
// positions, refill_pairs).  The pairs of 64 consecutive cells are stored
// interleaved (pair q of the group's cell l at q * 64 + l, the group padded
// to its longest list), so that a wave refilling those cells reads
// consecutive addresses at every step.
template <int MODE>
__global__ void __launch_bounds__(kThreads) shepard_gather(start_box box, double delta, int G, ReachClasses cls,
                                                           const unsigned *__restrict__ start,
                                                           const double4 *__restrict__ pos_h,
                                                           const double2 *__restrict__ kern,
                                                           const double *__restrict__ ns, double *val, float *valf,
                                                           int sx, int sy, unsigned *__restrict__ pcount,
                                                           const unsigned *__restrict__ pstart,
                                                           unsigned *__restrict__ pidx, double *__restrict__ pw,
                                                           double *__restrict__ pden)
{
    const int GZ = (G + kCellsZ - 1) / kCellsZ;   // thread groups per z row
    const int64_t lin = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    const int64_t ncell = (int64_t)G * G * G;
    if (lin >= (int64_t)G * G * GZ) return;
    const int ia = (int)(lin / ((int64_t)G * GZ)), ib = (int)((lin / GZ) % G);
    const int ic0 = (int)(lin % GZ) * kCellsZ;
    const int nz = G - ic0 < kCellsZ ? G - ic0 : kCellsZ;
    const int64_t cell0 = ((int64_t)ia * G + ib) * G + ic0;   // unpadded index of the first centre
    const double xc = box.lo[0] + ((double)ia + 0.5) * delta;
    const double yc = box.lo[1] + ((double)ib + 0.5) * delta;
    double zc[kCellsZ], num[kCellsZ], den[kCellsZ];
    unsigned cnt[kCellsZ];
    for (int j = 0; j < kCellsZ; ++j) {
        zc[j] = box.lo[2] + ((double)(ic0 + j) + 0.5) * delta;
        num[j] = 0.0;
        den[j] = 0.0;
        cnt[j] = 0u;
    }
    for (int k = 0; k < cls.K; ++k) {
        const unsigned *st = start + k * ncell;
        const float q2 = cls.q2[k];
        const int R = cls.R[k];
        const int a0 = ia - R < 0 ? 0 : ia - R, a1 = ia + R >= G ? G - 1 : ia + R;
        for (int a = a0; a <= a1; ++a) {
            const float fa = a == ia ? 0.0f : (float)(a < ia ? ia - a : a - ia) - 0.5f;
            const float ra = q2 - fa * fa;
            if (ra < 0.0f) continue;
            const int rb = (int)(sqrtf(ra) + 0.5f);
            const int b0 = ib - rb < 0 ? 0 : ib - rb, b1 = ib + rb >= G ? G - 1 : ib + rb;
            for (int b = b0; b <= b1; ++b) {
                const float fb = b == ib ? 0.0f : (float)(b < ib ? ib - b : b - ib) - 0.5f;
                const float rem = ra - fb * fb;
                const int rz = (int)(sqrtf(rem > 0.0f ? rem : 0.0f) + 0.5f);
                const int z0 = ic0 - rz < 0 ? 0 : ic0 - rz;
                const int z1 = ic0 + nz - 1 + rz >= G ? G - 1 : ic0 + nz - 1 + rz;
                const int64_t row = ((int64_t)a * G + b) * G;
                const unsigned s0 = st[row + z0], s1 = st[row + z1 + 1];
                for (unsigned s = s0; s < s1; ++s) {
                    const double4 p = pos_h[s];
                    const double dx = xc - p.x, dy = yc - p.y;
                    const double dxy2 = dx * dx + dy * dy, h2 = 4.0 * p.w * p.w;
                    if (!(dxy2 < h2)) continue;
                    if (MODE == kCountPairs) {
#pragma unroll
                        for (int j = 0; j < kCellsZ; ++j) {
                            const double dz = zc[j] - p.z;
                            cnt[j] += (j < nz && dxy2 + dz * dz < h2) ? 1u : 0u;
                        }
                        continue;
                    }
                    // the four centres without branches: a centre outside
                    // the support 2h (or past the row's end) adds 0
                    const double2 kk = kern[s];
                    const double nk = ns[s];
#pragma unroll
                    for (int j = 0; j < kCellsZ; ++j) {
                        const double dz = zc[j] - p.z;
                        const double r2 = dxy2 + dz * dz;
                        const bool in = j < nz && r2 < h2;
                        const double w = in ? kernel_w(sqrt_nr(r2) * kk.x, kk.y) : 0.0;
                        num[j] = fma(nk, w, num[j]);
                        den[j] += w;
                        if (MODE == kFillPairs && in) {
                            // pair q of cell c: group c / 64, place q * 64 + c % 64
                            const int64_t c = cell0 + j;
                            const int64_t at = (int64_t)pstart[c >> 6] + (int64_t)cnt[j] * 64 + (c & 63);
                            pidx[at] = s;
                            pw[at] = w;
                            ++cnt[j];
                        }
                    }
                }
            }
        }
    }
    for (int j = 0; j < nz; ++j) {
        if (MODE == kCountPairs) {
            pcount[cell0 + j] = cnt[j];
            continue;
        }
        if (MODE == kFillPairs) pden[cell0 + j] = den[j];
        const double v = den[j] > 0.0 ? num[j] / den[j] : 0.0;
        const int64_t e = (int64_t)ia * sx + (int64_t)ib * sy + ic0 + j;
        val[e] = v;
        valf[e] = (float)v;
    }
}

// Sum of n counts into a 64-bit total (the count scan is 32-bit).
__global__ void __launch_bounds__(kThreads) sum_counts(int64_t n, const unsigned *cnt, unsigned long long *total)
{
    __shared__ unsigned long long part[kThreads / 64];
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    unsigned long long v = i < n ? cnt[i] : 0ull;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kThreads / 64; ++w) t += part[w];
        if (t) atomicAdd(total, t);
    }
}

// The grid from the recorded pairs: the same sums in the same order as
// shepard_gather, so the same values bit for bit, reading each cell's pairs
// instead of searching the stencil.
__global__ void __launch_bounds__(kThreads) refill_pairs(int G, const unsigned *__restrict__ pcount,
                                                         const unsigned *__restrict__ gstart,
                                                         const unsigned *__restrict__ pidx,
                                                         const double *__restrict__ pw,
                                                         const double *__restrict__ pden,
                                                         const double *__restrict__ ns, double *val, float *valf,
                                                         int sx, int sy)
{
    const int64_t lin = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (lin >= (int64_t)G * G * G) return;
    const int ia = (int)(lin / ((int64_t)G * G)), ib = (int)((lin / G) % G), ic = (int)(lin % G);
    const int64_t base = (int64_t)gstart[lin >> 6] + (lin & 63);
    const unsigned nq = pcount[lin];
    double num = 0.0;
    for (unsigned q = 0; q < nq; ++q) {
        const int64_t at = base + (int64_t)q * 64;
        num = fma(ns[pidx[at]], pw[at], num);
    }
    const double den = pden[lin];
    const double v = den > 0.0 ? num / den : 0.0;
    const int64_t e = (int64_t)ia * sx + (int64_t)ib * sy + ic;
    val[e] = v;
    valf[e] = (float)v;
}

// Size of each group of 64 cells in the interleaved pair arrays: 64 times
// its longest list.
__global__ void __launch_bounds__(kThreads) group_sizes(int64_t ncell, int64_t ngroups, const unsigned *pcount,
                                                        unsigned *gsize)
{
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= ngroups) return;
    unsigned m = 0;
    for (int64_t c = g * 64; c < g * 64 + 64 && c < ncell; ++c) m = pcount[c] > m ? pcount[c] : m;
    gsize[g] = 64u * m;
}

__global__ void __launch_bounds__(kThreads) unpad(int G, int sx, int sy, const double *val, double *out)
{
    const int64_t lin = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (lin >= (int64_t)G * G * G) return;
    const int ia = (int)(lin / ((int64_t)G * G)), ib = (int)((lin / G) % G), ic = (int)(lin % G);
    out[lin] = val[(int64_t)ia * sx + (int64_t)ib * sy + ic];
}

}  // namespace

// Splits the non-empty reach bins into at most kmax classes of neighbouring
// bins, minimising an estimate of the gather work per cell centre: for each
// class, the particles it holds per cell times the cells its stencil scans
// (a ball of radius reach + half a cell), plus a fixed cost per row of cells.
// reach_cells is the largest reach in cells; it bounds the last class.
static ReachClasses choose_classes(const unsigned *hist, int64_t n, int64_t ncell, double reach_cells, int kmax,
                                   int4 *top)
{
    constexpr double kRowCost = 3.0;   // one row's set-up, in particle tests
    std::vector<int> bin;
    std::vector<double> pre(1, 0.0);
    for (int u = 0; u < kBins; ++u)
        if (hist[u]) {
            bin.push_back(u);
            pre.push_back(pre.back() + hist[u]);
        }
    const int m = (int)bin.size();
    ReachClasses c;
    *top = make_int4(kBins, kBins, kBins, 0);
    if (m == 0) return c;   // no particle: one empty class
    auto radius = [&](int j) {   // reach in cells of a class ending at bin j
        return bin[j] == kBins - 1 ? reach_cells : std::min(0.25 * bin[j], reach_cells);
    };
    auto cost = [&](int i, int j) {
        const double r = radius(j) + 0.5, rows = M_PI * r * r;
        return (pre[j + 1] - pre[i]) / (double)ncell * (4.0 / 3.0 * M_PI * r * r * r + rows) + kRowCost * rows;
    };
    const double inf = 1e300;
    // best[k][j]: k classes over the first j bins; from[k][j]: first bin of the last class
    std::vector<std::vector<double>> best(kmax + 1, std::vector<double>(m + 1, inf));
    std::vector<std::vector<int>> from(kmax + 1, std::vector<int>(m + 1, 0));
    best[0][0] = 0.0;
    for (int k = 1; k <= kmax; ++k)
        for (int j = 1; j <= m; ++j)
            for (int i = k - 1; i < j; ++i)
                if (best[k - 1][i] < inf) {
                    const double v = best[k - 1][i] + cost(i, j - 1);
                    if (v < best[k][j]) {
                        best[k][j] = v;
                        from[k][j] = i;
                    }
                }
    int K = 1;
    for (int k = 2; k <= kmax && k <= m; ++k)
        if (best[k][m] < best[K][m]) K = k;
    int last[kMaxReachClasses];
    for (int k = K, j = m; k > 0; --k) {
        last[k - 1] = j - 1;
        j = from[k][j];
    }
    c.K = K;
    int t[3] = {kBins, kBins, kBins};
    for (int k = 0; k < K; ++k) {
        const double r = radius(last[k]);
        // a margin far above the rounding of the binning and of the float
        // stencil arithmetic; it only ever adds cells to the scan
        c.q2[k] = (float)(r * r * (1.0 + 1e-4) + 1e-4);
        c.R[k] = (int)floor(0.5 + sqrt((double)c.q2[k]));
        if (k < 3 && k < K - 1) t[k] = bin[last[k]];
    }
    *top = make_int4(t[0], t[1], t[2], 0);
    (void)n;
    return c;
}

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
               al(nk * sizeof(double4)) + al(nk * sizeof(double2)) + al(nk * sizeof(double)) +
               al(kBins * sizeof(unsigned)) + 256;
    if (dmalloc(c, (void **)&b->mem, b->bytes) != hipSuccess) {
        b->mem = nullptr;
        return START_ENOMEM;
    }
    char *q = b->mem;
    auto take = [&](size_t v) { char *r = q; q += al(v); return r; };
    void *radix_tmp = take(radix_temp_bytes(nk));
    uint64_t *keys = (uint64_t *)take(nk * sizeof(uint64_t));
    b->idx = (unsigned *)take(nk * sizeof(unsigned));
    b->pos_h = (double4 *)take(nk * sizeof(double4));
    b->kern = (double2 *)take(nk * sizeof(double2));
    b->ns = (double *)take(nk * sizeof(double));
    unsigned *hist = (unsigned *)take(kBins * sizeof(unsigned));
    unsigned long long *hmax = (unsigned long long *)take(256);

    const double gs = (double)G / box.size;
    unsigned *bflags = c->d_flags + 1;   // build validation word (not the rate calls' one)
    hipMemsetAsync(bflags, 0, sizeof(unsigned), s);
    hipMemsetAsync(hist, 0, kBins * sizeof(unsigned), s);
    hipMemsetAsync(hmax, 0, sizeof(unsigned long long), s);
    grid_keys<<<blocks_for(n), kThreads, 0, s>>>(box, gs, G, n, xyz, h, nhi, keys, b->idx, bflags, hist, hmax);
    unsigned flags = 0;
    unsigned long long hbits = 0;
    unsigned hh[kBins];
    static_assert(kBins + 3 <= kReadbackWords, "readback words");
    if (c->rb) {
        grid_readback<<<1, kBins, 0, s>>>(bflags, hist, hmax, c->rb_dev);
    } else {
        hipMemcpyAsync(&flags, bflags, sizeof(unsigned), hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(hh, hist, sizeof(hh), hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(&hbits, hmax, sizeof(hbits), hipMemcpyDeviceToHost, s);
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess && c->rb) {
        const volatile unsigned *rb = c->rb;
        flags = rb[0];
        for (int k = 0; k < kBins; ++k) hh[k] = rb[1 + k];
        hbits = (unsigned long long)rb[1 + kBins] | ((unsigned long long)rb[2 + kBins] << 32);
    }
    if (e != hipSuccess || flags) {
        free_bins(c, b);
        if (e != hipSuccess) { c->err = hipGetErrorString(e); return START_EHIP; }
        if (flags & kFlagNonFinite) { c->err = "non-finite gas position, h or n_HI"; return START_ENONFINITE; }
        if (flags & kFlagOutOfBox) { c->err = "gas particle outside the box"; return START_EOUTOFBOX; }
        c->err = "gas h <= 0 or n_HI < 0";
        return START_EINVAL;
    }
    std::memcpy(&b->reach, &hbits, sizeof(double));
    int4 top;
    b->cls = choose_classes(hh, n, ncell, b->reach / b->delta, grid_log2 >= 10 ? 2 : kMaxReachClasses, &top);
    const int K = b->cls.K;
    // per (class, cell) starts, allocated once the number of classes is known
    const int64_t nstart = K * ncell + 1;
    b->bytes2 = al(nstart * sizeof(unsigned)) + al(scan_temp_bytes(nstart));
    if (dmalloc(c, (void **)&b->mem2, b->bytes2) != hipSuccess) {
        b->mem2 = nullptr;
        free_bins(c, b);
        c->err = "allocation failed";
        return START_ENOMEM;
    }
    b->start = (unsigned *)b->mem2;
    void *scan_tmp = b->mem2 + al(nstart * sizeof(unsigned));
    if (K > 1) class_keys<<<blocks_for(n), kThreads, 0, s>>>(n, h, gs, ncell, top, keys);
    radix_sort_pairs(keys, b->idx, n, 3 * grid_log2 + (K > 2 ? 2 : K - 1), radix_tmp, s);
    hipMemsetAsync(b->start, 0, nstart * sizeof(unsigned), s);
    cell_counts<<<blocks_for(n), kThreads, 0, s>>>(keys, n, b->start);
    exclusive_scan_u32(b->start, nstart, scan_tmp, s);
    unsigned *inv = (unsigned *)keys;   // the keys are no longer needed
    invert_perm<<<blocks_for(n), kThreads, 0, s>>>(n, b->idx, inv);
    scatter_particles<<<blocks_for(n), kThreads, 0, s>>>(n, inv, xyz, h, nhi, b->pos_h, b->kern, b->ns);
    return START_OK;
}

void free_bins(Ctx *c, GasBins *b)
{
    dfree(c, b->mem, b->bytes);
    dfree(c, b->mem2, b->bytes2);
    dfree(c, b->mem3, b->bytes3);
    dfree(c, b->mem4, b->bytes4);
    b->mem = b->mem2 = b->mem3 = b->mem4 = nullptr;
    b->bytes = b->bytes2 = b->bytes3 = b->bytes4 = 0;
    b->pcount = b->pstart = b->pidx = nullptr;
    b->pw = b->pden = nullptr;
}

namespace {

// Both copies of an empty grid set to 0 by a kernel (fill_grid may be
// captured into a HIP graph, where memset nodes are avoided).
__global__ void __launch_bounds__(256) zero_grid(int64_t span, double *val, float *valf)
{
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= span) return;
    val[k] = 0.0;
    valf[k] = 0.0f;
}

}  // namespace

void fill_grid(Ctx *c, const GasBins &b, const double *nhi, Grid *g)
{
    hipStream_t s = c->stream;
    if (b.n == 0) {
        zero_grid<<<(unsigned)((g->span + 255) / 256), 256, 0, s>>>(g->span, g->val, g->valf);
        return;
    }
    if (nhi) gather_values<<<blocks_for(b.n), kThreads, 0, s>>>(b.n, b.idx, nhi, b.ns);
    if (b.pidx) {
        const int64_t ncell = (int64_t)g->G * g->G * g->G;
        refill_pairs<<<blocks_for(ncell), kThreads, 0, s>>>(g->G, b.pcount, b.pstart, b.pidx, b.pw, b.pden, b.ns,
                                                            g->val, g->valf, g->sx, g->sy);
        return;
    }
    const int64_t groups = (int64_t)g->G * g->G * ((g->G + kCellsZ - 1) / kCellsZ);
    shepard_gather<kGather><<<blocks_for(groups), kThreads, 0, s>>>(
        b.box, b.delta, b.G, b.cls, b.start, b.pos_h, b.kern, b.ns, g->val, g->valf, g->sx, g->sy, nullptr, nullptr,
        nullptr, nullptr, nullptr);
}

start_status record_pairs(Ctx *c, GasBins *b, Grid *g)
{
    if (b->n == 0 || b->pidx) return START_OK;
    hipStream_t s = c->stream;
    auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
    const int64_t ncell = (int64_t)b->G * b->G * b->G;
    const int64_t ngroups = (ncell + 63) / 64;
    const int64_t groups = (int64_t)b->G * b->G * ((b->G + kCellsZ - 1) / kCellsZ);
    // 1. pairs per centre, the padded group sizes and their starts
    b->bytes3 = al(ncell * sizeof(unsigned)) + al((ngroups + 1) * sizeof(unsigned)) +
                al(scan_temp_bytes(ngroups + 1)) + al(ncell * sizeof(double)) + 256;
    if (dmalloc(c, (void **)&b->mem3, b->bytes3) != hipSuccess) {
        b->mem3 = nullptr;
        b->bytes3 = 0;
        return START_ENOMEM;
    }
    char *q = b->mem3;
    auto take = [&](size_t v) { char *r = q; q += al(v); return r; };
    b->pcount = (unsigned *)take(ncell * sizeof(unsigned));
    b->pstart = (unsigned *)take((ngroups + 1) * sizeof(unsigned));
    void *scan_tmp = take(scan_temp_bytes(ngroups + 1));
    b->pden = (double *)take(ncell * sizeof(double));
    unsigned long long *d_total = (unsigned long long *)take(256);
    auto drop = [&]() {
        dfree(c, b->mem3, b->bytes3);
        b->mem3 = nullptr;
        b->bytes3 = 0;
        b->pcount = b->pstart = nullptr;
        b->pden = nullptr;
    };
    hipMemsetAsync(b->pstart + ngroups, 0, sizeof(unsigned), s);
    hipMemsetAsync(d_total, 0, sizeof(unsigned long long), s);
    shepard_gather<kCountPairs><<<blocks_for(groups), kThreads, 0, s>>>(
        b->box, b->delta, b->G, b->cls, b->start, b->pos_h, b->kern, b->ns, nullptr, nullptr, 0, 0, b->pcount,
        nullptr, nullptr, nullptr, nullptr);
    group_sizes<<<blocks_for(ngroups), kThreads, 0, s>>>(ncell, ngroups, b->pcount, b->pstart);
    sum_counts<<<blocks_for(ngroups), kThreads, 0, s>>>(ngroups, b->pstart, d_total);
    unsigned long long total64 = 0;
    hipMemcpyAsync(&total64, d_total, sizeof(total64), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) {
        drop();
        return START_EHIP;
    }
    // the starts are 32-bit, and the pairs (12 B each) must stay modest
    if (total64 > kMaxPairs) {
        drop();
        return START_ENOMEM;
    }
    exclusive_scan_u32(b->pstart, ngroups + 1, scan_tmp, s);
    // 2. the pairs themselves (particle, weight), with the weight sums
    const size_t np = total64 > 0 ? (size_t)total64 : 1;
    b->bytes4 = al(np * sizeof(unsigned)) + al(np * sizeof(double));
    if (dmalloc(c, (void **)&b->mem4, b->bytes4) != hipSuccess) {
        b->mem4 = nullptr;
        b->bytes4 = 0;
        hipStreamSynchronize(s);   // the scan may still run
        drop();
        return START_ENOMEM;
    }
    unsigned *pidx = (unsigned *)b->mem4;
    b->pw = (double *)(b->mem4 + al(np * sizeof(unsigned)));
    shepard_gather<kFillPairs><<<blocks_for(groups), kThreads, 0, s>>>(
        b->box, b->delta, b->G, b->cls, b->start, b->pos_h, b->kern, b->ns, g->val, g->valf, g->sx, g->sy, nullptr,
        b->pstart, pidx, b->pw, b->pden);
    b->pidx = pidx;
    b->n_pairs = (int64_t)total64;
    if (hipStreamSynchronize(s) != hipSuccess) return START_EHIP;
    return START_OK;
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
    g->guard = G <= 512 ? 6 * ((int64_t)g->sx + g->sy + 1) : 0;
    const int64_t held = g->span + 2 * g->guard;
    size_t persist = al(held * sizeof(double)) + al(held * sizeof(float));
    char *pm = nullptr;
    if (dmalloc(c, (void **)&pm, persist) != hipSuccess) return START_ENOMEM;
    g->bytes = persist;
    g->mem = pm;
    g->val = (double *)pm + g->guard;
    g->valf = (float *)(pm + al(held * sizeof(double))) + g->guard;
    // guards and padding are never written again
    if (pad || g->guard) hipMemsetAsync(pm, 0, persist, c->stream);
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
        hipStreamSynchronize(c->stream);   // the padding clear may still run
        dfree(c, g->mem, g->bytes);
        return st;
    }
    fill_grid(c, b, nullptr, g);   // the binning already gathered n_HI
    hipError_t e = hipStreamSynchronize(c->stream);
    free_bins(c, &b);
    if (e != hipSuccess) {
        c->err = hipGetErrorString(e);
        dfree(c, g->mem, g->bytes);
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
