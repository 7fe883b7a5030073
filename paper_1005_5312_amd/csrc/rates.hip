// Photoionization rates of START (Hasegawa & Umemura 2010) on gfx950.
//
// For every target particle i:
//   Gamma_i = sigma / (4 pi) * sum_alpha L_alpha exp(-tau_alpha) / d_alpha^2,
// the monochromatic form of Appendix A eq. (A2) with on-the-spot attenuation
// (eq. 7), summed over the virtual sources the tree walk hands out
// (section 2.2.2, eqs. 12-15) and excluding the target's own emission
// (k_other, eqs. 25-26).  tau_alpha is the optical depth along the straight
// ray between source and target through the gridded n_HI field.
//
// One wavefront owns 64 targets that are adjacent in Morton order and walks
// the depth-first node array with one shared node pointer: a node is visited
// when any lane still needs it.  Each lane applies the FP64 opening test of
// eq. (12) on its own; a lane that uses a cell as a virtual source skips the
// cell's subtree by remembering where the subtree ends.  The lanes that take
// an entry at a node march their rays right away: they share the source, so
// their rays are nearly parallel and read the same grid lines.
//
// Precision: START_FP64 marches and accumulates in FP64.  START_FP32C keeps
// the FP64 opening test (exact lists) and marches in FP32 from the target
// towards the source, with crossings computed from the cell index rather
// than accumulated, and Kahan-compensated sums for tau and Gamma.
#include "internal.h"

#include <cstring>

namespace start {

namespace {

constexpr int kWave = 64;
constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;

enum Mode { kRates = 0, kCount = 1, kList = 2, kStats = 3 };

struct Params {
    // tree
    int64_t n_nodes;
    const int4 *geo;
    const int *skip;
    const int *first;
    const int *count;
    const int *ref;
    const double4 *mom;
    const float4 *momf;
    const double4 *src;
    const float4 *srcf;
    const unsigned *perm;
    // grid
    const double *grid;
    const float *gridf;
    int G;
    double gs;          // G / size
    double lo[3];
    double inv_size;
    double unit_cm;
    double cell_cm;     // size / G * unit_cm
    double theta2;
    double sigma;
    // targets (sorted)
    int64_t n_t;
    const double4 *tgt;      // sorted target positions
    const unsigned *tgt_orig;
    const int64_t *self_src; // original order, may be null
    // outputs
    void *gamma;             // original order
    int64_t *counts;         // kCount: entries per target (original order)
    const int64_t *offsets;  // kList
    int64_t *entries;        // kList
    int64_t *stats;          // kStats: [n_t][4]
};

// Eq. (12): l^2 <= theta^2 d^2 in normalised units, d the distance to the
// closest point of the cube [c 2^-n, (c+1) 2^-n].  Written as the same FP64
// operations as the checker (explicit fma, no contraction) so that the lists
// agree bit for bit.
__device__ inline bool accept(const int4 g, const double u[3], double theta2)
{
    const int level = g.w & 0xFF;
    const double l = ldexp(1.0, -level);
    const int c[3] = {g.x, g.y, g.z};
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double lo = ldexp((double)c[k], -level);
        const double hi = ldexp((double)(c[k] + 1), -level);
        const double a = lo - u[k];
        const double b = u[k] - hi;
        const double m = a > b ? a : b;
        d[k] = m > 0.0 ? m : 0.0;
    }
    const double d2 = fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
    return l * l <= theta2 * d2;
}

__device__ inline int clampi(int v, int G) { return v < 0 ? 0 : (v >= G ? G - 1 : v); }

// Exact column of the piecewise-constant field from a to b (FP64 grid units),
// stepping cell to cell; returns sum n_c dt with t in [0, 1].
__device__ inline double column_fp64(const double *grid, int G, const double A[3], const double B[3],
                                     int &ncell)
{
    int cell[3], step[3];
    double tn[3], dt[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double D = B[k] - A[k];
        cell[k] = clampi((int)floor(A[k]), G);
        if (D > 0.0) {
            const double inv = 1.0 / D;
            step[k] = 1;
            tn[k] = ((double)(cell[k] + 1) - A[k]) * inv;
            dt[k] = inv;
        } else if (D < 0.0) {
            const double inv = 1.0 / D;
            step[k] = -1;
            tn[k] = ((double)cell[k] - A[k]) * inv;
            dt[k] = -inv;
        } else {
            step[k] = 0;
            tn[k] = 2.0;
            dt[k] = 0.0;
        }
    }
    double t = 0.0, sum = 0.0;
    const int max_steps = 3 * G + 3;
    for (int it = 0; it < max_steps; ++it) {
        double tm = fmin(fmin(tn[0], tn[1]), tn[2]);
        const bool last = !(tm < 1.0);
        if (last) tm = 1.0;
        const double len = tm - t;
        if (len > 0.0) {
            sum += grid[((int64_t)cell[0] * G + cell[1]) * G + cell[2]] * len;
            ++ncell;
        }
        if (last) break;
        t = tm;
        int a = (tn[0] <= tn[1] && tn[0] <= tn[2]) ? 0 : (tn[1] <= tn[2] ? 1 : 2);
        cell[a] = clampi(cell[a] + step[a], G);
        tn[a] += dt[a];
    }
    return sum;
}

struct Acc64 {
    double g = 0.0;
};

// FP64 contribution of a (virtual) source at physical position s with
// luminosity L to the target at x.
__device__ inline void contribute_fp64(const Params &P, const double x[3], const double B[3], double sx,
                                       double sy, double sz, double L, Acc64 &acc, int64_t *st)
{
    const double dx = x[0] - sx, dy = x[1] - sy, dz = x[2] - sz;
    const double dist = sqrt(dx * dx + dy * dy + dz * dz);
    if (dist == 0.0) {
        if (st) st[3]++;
        return;
    }
    const double A[3] = {(sx - P.lo[0]) * P.gs, (sy - P.lo[1]) * P.gs, (sz - P.lo[2]) * P.gs};
    int nc = 0;
    const double col = column_fp64(P.grid, P.G, A, B, nc) * dist;
    if (st) st[2] += nc;
    const double tau = P.sigma * col * P.unit_cm;
    const double dcm = dist * P.unit_cm;
    acc.g += L * exp(-tau) / (dcm * dcm);
}

// FP32: the ray is marched from the target (origin, t = 0) to the source
// (t = 1), so the crossings nearest the target -- where the target's own cell
// may be dense -- carry the smallest absolute error.  Crossing parameters come
// from the plane index each time, never by accumulation.
struct Acc32 {
    float g = 0.f, gc = 0.f;   // Kahan sum of L' e^-tau / d^2
};

__device__ inline void contribute_fp32(const Params &P, const int bi[3], const float fb[3], float4 s,
                                       Acc32 &acc, int64_t *st)
{
    const float Gf = (float)P.G;
    int ai[3];
    float D[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float* sp = &s.x;
        const float A = sp[k] * Gf;                 // exact: G is a power of two
        const float fl = floorf(A);
        ai[k] = (int)fl;
        const float fa = A - fl;                     // exact
        D[k] = (float)(ai[k] - bi[k]) + (fa - fb[k]);
    }
    const float d2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
    if (d2 == 0.f) {
        if (st) st[3]++;
        return;
    }
    int cell[3], step[3], plane[3];
    float inv[3], tn[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cell[k] = clampi(bi[k], P.G);
        if (D[k] > 0.f) {
            step[k] = 1;
            plane[k] = bi[k] + 1;
            inv[k] = 1.0f / D[k];
            tn[k] = ((float)(plane[k] - bi[k]) - fb[k]) * inv[k];
        } else if (D[k] < 0.f) {
            step[k] = -1;
            plane[k] = bi[k];
            inv[k] = 1.0f / D[k];
            tn[k] = ((float)(plane[k] - bi[k]) - fb[k]) * inv[k];
        } else {
            step[k] = 0;
            plane[k] = 0;
            inv[k] = 0.f;
            tn[k] = 2.f;
        }
    }
    float t = 0.f, sum = 0.f, comp = 0.f;
    const int max_steps = 3 * P.G + 3;
    int nc = 0;
    for (int it = 0; it < max_steps; ++it) {
        float tm = fminf(fminf(tn[0], tn[1]), tn[2]);
        const bool last = !(tm < 1.f);
        if (last) tm = 1.f;
        const float len = tm - t;
        if (len > 0.f) {
            const float v = P.gridf[((int64_t)cell[0] * P.G + cell[1]) * P.G + cell[2]];
            const float y = fmaf(v, len, -comp);
            const float tt = sum + y;
            comp = (tt - sum) - y;
            sum = tt;
            ++nc;
        }
        if (last) break;
        t = tm;
        const int a = (tn[0] <= tn[1] && tn[0] <= tn[2]) ? 0 : (tn[1] <= tn[2] ? 1 : 2);
        cell[a] = clampi(cell[a] + step[a], P.G);
        plane[a] += step[a];
        tn[a] = ((float)(plane[a] - bi[a]) - fb[a]) * inv[a];
    }
    if (st) st[2] += nc;
    const float dist = sqrtf(d2);                    // grid units
    const float tau = (float)(P.sigma * P.cell_cm) * (sum * dist);
    const float term = s.w * expf(-tau) / d2;
    const float y = term - acc.gc;
    const float tt = acc.g + y;
    acc.gc = (tt - acc.g) - y;
    acc.g = tt;
}

template <int PREC, int MODE>
__global__ void __launch_bounds__(kThreads) walk_kernel(Params P)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t tile = (int64_t)blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    const int64_t it = tile * kWave + lane;
    const bool valid = it < P.n_t;
    if (tile * kWave >= P.n_t) return;   // whole wave past the end

    double x[3] = {0.0, 0.0, 0.0}, u[3] = {0.0, 0.0, 0.0}, B[3] = {0.0, 0.0, 0.0};
    int bi[3] = {0, 0, 0};
    float fb[3] = {0.f, 0.f, 0.f};
    unsigned orig = 0;
    int64_t self = -1;
    if (valid) {
        const double4 p = P.tgt[it];
        x[0] = p.x;
        x[1] = p.y;
        x[2] = p.z;
        orig = P.tgt_orig[it];
        if (P.self_src) self = P.self_src[orig];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double v = (x[k] - P.lo[k]) * P.inv_size;
            u[k] = v > 1.0 ? 1.0 : (v < 0.0 ? 0.0 : v);
            B[k] = (x[k] - P.lo[k]) * P.gs;
            // cell of the target clamped to the grid (a target on the top
            // face sits in the last cell at fraction 1)
            bi[k] = clampi((int)floor(B[k]), P.G);
            fb[k] = (float)(B[k] - (double)bi[k]);
        }
    }
    Acc64 a64;
    Acc32 a32;
    int64_t stv[4] = {0, 0, 0, 0};
    int64_t *st = MODE == kStats ? stv : nullptr;
    int64_t n_entries = 0;
    int64_t out_base = 0;
    if (MODE == kList && valid) out_base = P.offsets[orig];

    auto use = [&](int64_t code, double4 m64, float4 m32) {
        // one interaction-list entry: code >= 0 node index, < 0 -(source)-1
        if (MODE == kCount) {
            ++n_entries;
        } else if (MODE == kList) {
            P.entries[out_base + n_entries] = code;
            ++n_entries;
        } else {
            if (st) st[1]++;
            if (PREC == START_FP64)
                contribute_fp64(P, x, B, m64.x, m64.y, m64.z, m64.w, a64, st);
            else
                contribute_fp32(P, bi, fb, m32, a32, st);
        }
    };

    // Entry filter: sources and cells of zero luminosity contribute nothing
    // and are left out.  The FP32 rate path reads only the FP32 copy.
    constexpr bool kFp32Rates = PREC == START_FP32C && MODE == kRates;
    const double4 z64 = make_double4(0.0, 0.0, 0.0, 0.0);
    const float4 z32 = make_float4(0.f, 0.f, 0.f, 0.f);
    auto use_node = [&](int64_t code, int nd) {
        if (kFp32Rates) {
            const float4 mf = P.momf[nd];
            if (mf.w > 0.f) use(code, z64, mf);
        } else {
            const double4 m = P.mom[nd];
            if (m.w > 0.0) use(code, m, PREC == START_FP32C ? P.momf[nd] : z32);
        }
    };
    auto use_src = [&](int64_t code, int q) {
        if (kFp32Rates) {
            const float4 mf = P.srcf[q];
            if (mf.w > 0.f) use(code, z64, mf);
        } else {
            const double4 m = P.src[q];
            if (m.w > 0.0) use(code, m, PREC == START_FP32C ? P.srcf[q] : z32);
        }
    };

    int resume = 0;
    int node = 0;
    const int n_nodes = (int)P.n_nodes;
    while (node < n_nodes) {
        node = __builtin_amdgcn_readfirstlane(node);
        const int4 g = P.geo[node];
        const int kind = g.w >> 8;
        const bool active = valid && node >= resume;
        if (kind == kKindLeaf) {
            if (active) {
                const int j = P.ref[node];
                if ((int64_t)j != self) use_node(-(int64_t)j - 1, node);
            }
            node += 1;
            continue;
        }
        const int sk = P.skip[node];
        bool acc = false;
        if (active) {
            if (st) st[0]++;
            acc = accept(g, u, P.theta2);
        }
        if (acc) {
            use_node(node, node);
            resume = sk;
        }
        const bool open = active && !acc;
        if (kind == kKindBucket) {
            if (open) {
                const int f = P.first[node], cnt = P.count[node];
                for (int q = f; q < f + cnt; ++q) {
                    const int j = (int)P.perm[q];
                    if ((int64_t)j != self) use_src(-(int64_t)j - 1, q);
                }
            }
            node += 1;
            continue;
        }
        node = __any(open) ? node + 1 : sk;
    }

    if (!valid) return;
    if (MODE == kCount) {
        P.counts[orig] = n_entries;
    } else if (MODE == kStats) {
        for (int k = 0; k < 4; ++k) P.stats[(int64_t)orig * 4 + k] = stv[k];
    } else if (MODE == kRates) {
        const double four_pi = 4.0 * M_PI;
        if (PREC == START_FP64) {
            static_cast<double *>(P.gamma)[orig] = P.sigma / four_pi * a64.g;
        } else {
            // L' = L / L_root and lengths in cells: restore units in FP64
            const double L0 = P.n_nodes > 0 ? P.mom[0].w : 0.0;   // empty tree: no arrays
            const double Lref = L0 > 0.0 ? L0 : 1.0;
            const double sum = (double)a32.g - (double)a32.gc;
            static_cast<float *>(P.gamma)[orig] = (float)(P.sigma / four_pi * sum * Lref / (P.cell_cm * P.cell_cm));
        }
    }
}

__global__ void __launch_bounds__(kThreads) check_self(int64_t n, const int64_t *self_src, int64_t n_src,
                                                       unsigned *flags)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    const int64_t sv = self_src[j];
    if (sv < -1 || sv >= n_src) atomicOr(flags, kFlagBadSelf);
}

__global__ void __launch_bounds__(kThreads) gather_targets(int64_t n, const unsigned *perm, const double *xyz,
                                                           double4 *tgt)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    const unsigned o = perm[j];
    tgt[j] = make_double4(xyz[o], xyz[n + o], xyz[2 * n + o], 0.0);
}

// FP32 copies of the virtual sources: normalised centre in [0, 1] and the
// luminosity relative to the root's (so every L' <= 1).
__global__ void __launch_bounds__(kThreads) make_fp32_nodes(int64_t m, const double4 *mom, start_box box,
                                                            double inv, float4 *momf)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    const double Lref = mom[0].w > 0.0 ? mom[0].w : 1.0;
    const double4 v = mom[p];
    momf[p] = make_float4((float)((v.x - box.lo[0]) * inv), (float)((v.y - box.lo[1]) * inv),
                          (float)((v.z - box.lo[2]) * inv), (float)(v.w / Lref));
}

__global__ void __launch_bounds__(kThreads) make_fp32_src(int64_t n, const double4 *src, const double4 *mom,
                                                          start_box box, double inv, float4 *srcf)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    const double Lref = mom[0].w > 0.0 ? mom[0].w : 1.0;
    const double4 v = src[j];
    srcf[j] = make_float4((float)((v.x - box.lo[0]) * inv), (float)((v.y - box.lo[1]) * inv),
                          (float)((v.z - box.lo[2]) * inv), (float)(v.w / Lref));
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

void make_fp32_tree(Tree *t, hipStream_t s)
{
    if (t->n_nodes == 0) return;
    const double inv = 1.0 / t->box.size;
    make_fp32_nodes<<<blocks_for(t->n_nodes), kThreads, 0, s>>>(t->n_nodes, t->mom, t->box, inv, t->momf);
    make_fp32_src<<<blocks_for(t->n_src), kThreads, 0, s>>>(t->n_src, t->src, t->mom, t->box, inv, t->srcf);
}

struct TargetScratch {
    uint64_t *keys;
    unsigned *idx;
    double4 *tgt;
    void *radix_tmp;
};

size_t target_scratch_bytes(int64_t n)
{
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int64_t nk = n > 1 ? n : 1;
    return al(nk * sizeof(uint64_t)) + al(nk * sizeof(unsigned)) + al(nk * sizeof(double4)) +
           al(radix_temp_bytes(nk)) + 256;
}

static TargetScratch carve(void *base, int64_t n)
{
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int64_t nk = n > 1 ? n : 1;
    char *q = (char *)base;
    TargetScratch ts;
    ts.keys = (uint64_t *)q;
    q += al(nk * sizeof(uint64_t));
    ts.idx = (unsigned *)q;
    q += al(nk * sizeof(unsigned));
    ts.tgt = (double4 *)q;
    q += al(nk * sizeof(double4));
    ts.radix_tmp = q;
    return ts;
}

// Orders the targets by Morton key and gathers their positions (device).
void prepare_targets(Ctx *c, const start_box &box, int64_t n_t, const double *tgt_xyz, const int64_t *self_src,
                     int64_t n_src, void *scratch, hipStream_t s)
{
    TargetScratch ts = carve(scratch, n_t);
    launch_keys(box, n_t, tgt_xyz, nullptr, ts.keys, ts.idx, c->d_flags, s);
    if (self_src) check_self<<<blocks_for(n_t), kThreads, 0, s>>>(n_t, self_src, n_src, c->d_flags);
    radix_sort_pairs(ts.keys, ts.idx, n_t, 63, ts.radix_tmp, s);
    gather_targets<<<blocks_for(n_t), kThreads, 0, s>>>(n_t, ts.idx, tgt_xyz, ts.tgt);
}

static Params make_params(const Tree *t, const Grid *g, int64_t n_t, void *scratch, const int64_t *self_src,
                          double theta, double sigma)
{
    TargetScratch ts = carve(scratch, n_t);
    Params P;
    memset(&P, 0, sizeof(P));
    P.n_nodes = t->n_nodes;
    P.geo = t->geo;
    P.skip = t->skip;
    P.first = t->first;
    P.count = t->count;
    P.ref = t->ref;
    P.mom = t->mom;
    P.momf = t->momf;
    P.src = t->src;
    P.srcf = t->srcf;
    P.perm = t->perm;
    if (g) {
        P.grid = g->val;
        P.gridf = g->valf;
        P.G = g->G;
    } else {
        P.G = 1;
    }
    P.gs = (double)P.G / t->box.size;
    for (int k = 0; k < 3; ++k) P.lo[k] = t->box.lo[k];
    P.inv_size = 1.0 / t->box.size;
    P.unit_cm = t->box.length_unit_cm;
    P.cell_cm = t->box.size / P.G * t->box.length_unit_cm;
    P.theta2 = theta * theta;
    P.sigma = sigma;
    P.n_t = n_t;
    P.tgt = ts.tgt;
    P.tgt_orig = ts.idx;
    P.self_src = self_src;
    return P;
}

static unsigned walk_blocks(int64_t n_t)
{
    const int64_t tiles = (n_t + kWave - 1) / kWave;
    return (unsigned)((tiles + kWavesPerBlock - 1) / kWavesPerBlock);
}

void launch_rates(const Tree *t, const Grid *g, int64_t n_t, void *scratch, const int64_t *self_src,
                  double theta, double sigma, int prec, void *gamma, hipStream_t s)
{
    Params P = make_params(t, g, n_t, scratch, self_src, theta, sigma);
    P.gamma = gamma;
    if (prec == START_FP64) {
        walk_kernel<START_FP64, kRates><<<walk_blocks(n_t), kThreads, 0, s>>>(P);
    } else {
        walk_kernel<START_FP32C, kRates><<<walk_blocks(n_t), kThreads, 0, s>>>(P);
    }
}

void launch_counts(const Tree *t, int64_t n_t, void *scratch, const int64_t *self_src, double theta,
                   int64_t *counts, hipStream_t s)
{
    Params P = make_params(t, nullptr, n_t, scratch, self_src, theta, 0.0);
    P.counts = counts;
    walk_kernel<START_FP64, kCount><<<walk_blocks(n_t), kThreads, 0, s>>>(P);
}

void launch_lists(const Tree *t, int64_t n_t, void *scratch, const int64_t *self_src, double theta,
                  const int64_t *offsets, int64_t *entries, hipStream_t s)
{
    Params P = make_params(t, nullptr, n_t, scratch, self_src, theta, 0.0);
    P.offsets = offsets;
    P.entries = entries;
    walk_kernel<START_FP64, kList><<<walk_blocks(n_t), kThreads, 0, s>>>(P);
}

void launch_stats(const Tree *t, const Grid *g, int64_t n_t, void *scratch, const int64_t *self_src,
                  double theta, int prec, int64_t *stats, hipStream_t s)
{
    Params P = make_params(t, g, n_t, scratch, self_src, theta, 1.0);
    P.stats = stats;
    if (prec == START_FP64)
        walk_kernel<START_FP64, kStats><<<walk_blocks(n_t), kThreads, 0, s>>>(P);
    else
        walk_kernel<START_FP32C, kStats><<<walk_blocks(n_t), kThreads, 0, s>>>(P);
}

}  // namespace start
