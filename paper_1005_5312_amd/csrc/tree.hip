// Source octree of START (Hasegawa & Umemura 2010, section 2.2.2) for gfx950.
//
// The paper splits cubic cells into 8 until every cell holds one source.  On
// the GPU the same cells come out of sorted Morton keys:
//   1. keys: each position is normalised to the box, quantised to 21 bits per
//      axis and bit-interleaved (x most significant), so a key's top 3n bits
//      name its level-n cell;
//   2. a stable radix sort orders the sources by (key, original index);
//   3. a binary radix tree over the sorted keys (one internal node per pair of
//      neighbours, built in parallel); a binary node whose common prefix
//      ends in a deeper octal digit than its parent's is a cell of the
//      octree that splits, and a run of identical keys is a level-21 bucket;
//   4. cells and single-source leaves are sorted by (first source, level),
//      which is the depth-first order of the octree, and every node gets the
//      index of the first node after its subtree (stackless walk);
//   5. the virtual source of each cell, eqs. (14)-(15), is summed bottom-up in
//      FP64, children in depth-first order.
// A cell whose sources all sit in one sub-cube is represented by the deepest
// cube with the same sources: the opening test is monotone from parent to
// child, so testing that cube decides the whole chain.
#include <algorithm>

#include "internal.h"

namespace start {

namespace {

constexpr int kThreads = 256;

__device__ inline uint64_t spread3(uint64_t v)
{
    // 21 bits -> every third bit of 63
    v &= 0x1FFFFFull;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

__device__ inline unsigned compact3(uint64_t v)
{
    v &= 0x1249249249249249ull;
    v = (v ^ (v >> 2)) & 0x10C30C30C30C30C3ull;
    v = (v ^ (v >> 4)) & 0x100F00F00F00F00Full;
    v = (v ^ (v >> 8)) & 0x1F0000FF0000FFull;
    v = (v ^ (v >> 16)) & 0x1F00000000FFFFull;
    v = (v ^ (v >> 32)) & 0x1FFFFFull;
    return (unsigned)v;
}

__global__ void __launch_bounds__(kThreads) keys_kernel(start_box box, double inv, int64_t n, const double *xyz,
                                                        const double *lum, uint64_t *keys, unsigned *idx,
                                                        unsigned *flags)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    unsigned bad = 0;
    uint64_t key = 0;
    for (int k = 0; k < 3; ++k) {
        const double x = xyz[(int64_t)k * n + j];
        double u;
        if (!isfinite(x)) {
            bad |= kFlagNonFinite;
            u = 0.0;
        } else if (x < box.lo[k] || x > box.lo[k] + box.size) {
            bad |= kFlagOutOfBox;
            u = x < box.lo[k] ? 0.0 : 1.0;
        } else {
            u = (x - box.lo[k]) * inv;
            u = u > 1.0 ? 1.0 : u;
        }
        unsigned q = (unsigned)(u * 2097152.0);   // exact scaling by 2^21, truncation = floor
        q = q > 2097151u ? 2097151u : q;
        key |= spread3(q) << (2 - k);
    }
    if (lum) {
        const double L = lum[j];
        if (!isfinite(L)) bad |= kFlagNonFinite;
        else if (L < 0.0) bad |= kFlagNegative;
    }
    if (bad) atomicOr(flags, bad);
    keys[j] = key;
    idx[j] = (unsigned)j;
}

// Common prefix length of keys a and b as 63-bit strings followed by the
// 32-bit index (so identical keys still order); -1 outside [0, n).
__device__ inline int prefix_len(const uint64_t *k, int n, int a, int b)
{
    if (b < 0 || b >= n) return -1;
    const uint64_t x = k[a] ^ k[b];
    if (x) return __clzll((long long)x) - 1;
    return 63 + __clz((int)((unsigned)a ^ (unsigned)b));
}

__device__ inline int oct_level(int delta) { return (delta >= 63 ? 63 : delta) / 3; }

// Binary radix tree over n sorted keys (internal nodes 0..n-2, node 0 the root).
__global__ void __launch_bounds__(kThreads) radix_tree_kernel(const uint64_t *k, int n, int *lo_out, int *hi_out,
                                                              int *delta_out, int *parent_int)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n - 1) return;
    const int d = (prefix_len(k, n, i, i + 1) - prefix_len(k, n, i, i - 1)) >= 0 ? 1 : -1;
    const int dmin = prefix_len(k, n, i, i - d);
    int lmax = 2;
    while (prefix_len(k, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(k, n, i, i + (l + t) * d) > dmin) l += t;
    const int j = i + l * d;
    const int dnode = prefix_len(k, n, i, j);
    int s = 0;
    int t = l;
    do {
        t = (t + 1) >> 1;
        if (prefix_len(k, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int gamma = i + s * d + (d < 0 ? -1 : 0);
    const int lo = i < j ? i : j;
    const int hi = i < j ? j : i;
    lo_out[i] = lo;
    hi_out[i] = hi;
    delta_out[i] = dnode;
    // children: gamma (left) and gamma + 1 (right); leaves are not tracked here
    if (lo != gamma) parent_int[gamma] = i;
    if (hi != gamma + 1) parent_int[gamma + 1] = i;
}

// The counts the host needs mid-build (internal nodes and leaves: the last
// scanned position plus the last flag of each array) and the validation
// word, written by one lane into the context's pinned readback words.
__global__ void tree_readback(int n, const unsigned *pos_int, const unsigned *flag_int, const unsigned *pos_leaf,
                              const unsigned *flag_leaf, const unsigned *bflags, unsigned *rb)
{
    if (threadIdx.x != 0) return;
    rb[0] = n > 1 ? pos_int[n - 2] : 0u;
    rb[1] = n > 1 ? flag_int[n - 2] : 0u;
    rb[2] = pos_leaf[n - 1];
    rb[3] = flag_leaf[n - 1];
    rb[4] = *bflags;
}

// Items of the octree: canonical cells (internal binary nodes whose octal
// level is deeper than their parent's) and single-source leaves.  The sort key
// (first << 5 | level) gives depth-first order; leaves take level 22.
__global__ void __launch_bounds__(kThreads) mark_items(const uint64_t *k, int n, const int *lo, const int *delta,
                                                       const int *parent_int, unsigned *flag_int,
                                                       unsigned *flag_leaf)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n - 1) {
        bool canon = (i == 0) || oct_level(delta[i]) > oct_level(delta[parent_int[i]]);
        flag_int[i] = canon ? 1u : 0u;
    }
    if (i < n) {
        bool single = (i == 0 || k[i - 1] != k[i]) && (i == n - 1 || k[i + 1] != k[i]);
        flag_leaf[i] = single ? 1u : 0u;
    }
}

__global__ void __launch_bounds__(kThreads) emit_items(int n, const int *lo, const int *delta,
                                                       const unsigned *flag_int, const unsigned *pos_int,
                                                       const unsigned *flag_leaf, const unsigned *pos_leaf,
                                                       unsigned n_int_items, uint64_t *item_key,
                                                       unsigned *item_code, unsigned *first_count)
{
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n - 1 && flag_int[i]) {
        const unsigned p = pos_int[i];
        item_key[p] = ((uint64_t)lo[i] << 5) | (uint64_t)oct_level(delta[i]);
        item_code[p] = (unsigned)i;
        atomicAdd(&first_count[lo[i]], 1u);
    }
    if (i < n && flag_leaf[i]) {
        const unsigned p = n_int_items + pos_leaf[i];
        item_key[p] = ((uint64_t)i << 5) | 22ull;
        item_code[p] = (unsigned)(n - 1 + i);
        atomicAdd(&first_count[i], 1u);
    }
}

__global__ void __launch_bounds__(kThreads) fill_nodes(int n, int64_t m, const uint64_t *k, const unsigned *perm,
                                                       const int *lo, const int *hi, const int *delta,
                                                       const unsigned *item_code, const unsigned *pos_start,
                                                       int4 *geo, int *skip, int *first, int *count, int *ref,
                                                       double4 *bnd)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    const unsigned code = item_code[p];
    int f, c, level, kind, r = -1;
    if (code < (unsigned)(n - 1)) {
        const int i = (int)code;
        f = lo[i];
        c = hi[i] - lo[i] + 1;
        level = oct_level(delta[i]);
        kind = delta[i] >= 63 ? kKindBucket : kKindInternal;
    } else {
        f = (int)(code - (unsigned)(n - 1));
        c = 1;
        // a leaf's own cube is one level below the deepest cube it shares
        int dl = f > 0 ? prefix_len(k, n, f, f - 1) : -1;
        int dr = f < n - 1 ? prefix_len(k, n, f, f + 1) : -1;
        int dm = dl > dr ? dl : dr;
        level = dm < 0 ? 0 : oct_level(dm) + 1;
        level = level > kMaxLevel ? kMaxLevel : level;
        kind = kKindLeaf;
        r = (int)perm[f];
    }
    const uint64_t prefix = level > 0 ? (k[f] >> (3 * (kMaxLevel - level))) : 0ull;
    const int cx = (int)compact3(prefix >> 2), cy = (int)compact3(prefix >> 1), cz = (int)compact3(prefix);
    geo[p] = make_int4(cx, cy, cz, level | (kind << 8));
    // the cube's lower corner and side in normalised units (exact: c < 2^21)
    bnd[p] = make_double4(ldexp((double)cx, -level), ldexp((double)cy, -level), ldexp((double)cz, -level),
                          ldexp(1.0, -level));
    skip[p] = (int)pos_start[f + c];
    first[p] = f;
    count[p] = c;
    ref[p] = r;
}

__global__ void __launch_bounds__(kThreads) invert_order(int64_t n, const unsigned *perm, unsigned *inv)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    inv[perm[j]] = (unsigned)j;
}

// The sorted sources, written from the input in order through the inverse
// permutation (a gather through the permutation reads four scattered
// doubles per source).
__global__ void __launch_bounds__(kThreads) scatter_sources(int64_t n, const unsigned *inv, const double *xyz,
                                                            const double *lum, double4 *src)
{
    const int64_t o = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (o >= n) return;
    src[inv[o]] = make_double4(xyz[o], xyz[n + o], xyz[2 * n + o], lum[o]);
}

// Bottom-up sums S = sum L_j r_j and L = sum L_j (eqs. 14-15) for the nodes of
// one level; children are visited in depth-first order.
// One byte per node for the level passes: its level, or 0xFF for a leaf
// (each pass then reads 1 byte per node instead of the 16-byte record).
__global__ void __launch_bounds__(kThreads) node_levels(int64_t m, const int4 *geo, unsigned char *lvl)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    const int w = geo[p].w;
    lvl[p] = (w >> 8) == kKindLeaf ? (unsigned char)0xFF : (unsigned char)(w & 0xFF);
}

__global__ void __launch_bounds__(kThreads) moments_level(int64_t m, int level, const unsigned char *lvl,
                                                          const int4 *geo, const int *skip, const int *first,
                                                          const int *count, const double4 *src, double4 *msum)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    const unsigned char lp = lvl[p];
    if (lp == 0xFF) {
        if (level != 0) return;   // leaves are filled once, in the first launch
        const double4 s = src[first[p]];
        msum[p] = make_double4(s.w * s.x, s.w * s.y, s.w * s.z, s.w);
        return;
    }
    if ((int)lp != kMaxLevel - level) return;
    const int kind = geo[p].w >> 8;
    double sx = 0.0, sy = 0.0, sz = 0.0, L = 0.0;
    if (kind == kKindBucket) {
        for (int q = first[p]; q < first[p] + count[p]; ++q) {
            const double4 s = src[q];
            sx += s.w * s.x;
            sy += s.w * s.y;
            sz += s.w * s.z;
            L += s.w;
        }
    } else {
        const int end = skip[p];
        for (int64_t c = p + 1; c < end; c = skip[c]) {
            const double4 s = msum[c];
            sx += s.x;
            sy += s.y;
            sz += s.z;
            L += s.w;
        }
    }
    msum[p] = make_double4(sx, sy, sz, L);
}

__global__ void __launch_bounds__(kThreads) moments_finish(int64_t m, const int4 *geo, const int *first,
                                                           const double4 *src, const double4 *msum,
                                                           double4 *mom)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    const int kind = geo[p].w >> 8;
    if (kind == kKindLeaf) {
        mom[p] = src[first[p]];
        return;
    }
    const double4 s = msum[p];
    if (s.w > 0.0)
        mom[p] = make_double4(s.x / s.w, s.y / s.w, s.z / s.w, s.w);
    else
        mom[p] = make_double4(0.0, 0.0, 0.0, 0.0);
}

// The luminosity unit of the FP32 copies for a tree of eq. (14): the root's
// luminosity, which no node or source exceeds (1 for a dark tree).
__global__ void root_scale(const double4 *mom, double *lscale)
{
    if (threadIdx.x == 0) lscale[0] = mom[0].w > 0.0 ? mom[0].w : 1.0;
}

// ---- kernel-weighted node luminosities (section 2.2.2) -----------------
// Each node of >= 2 sources gets, at its centre of luminosity r (eq. 15),
//   form 1: L = sum_j L_j W_j / sum_j W_j (0 when every W_j = 0),
//   form 2: L = sum_j V_j L_j W_j,
// W_j = W(|r - r_j|, h_j), the cubic spline of section 2.1.  The members of
// a node are a contiguous run of the sorted sources, so a node is split
// into chunks of kLumChunk members, one wave per chunk (the root alone would
// otherwise hold one wave for the whole source list); the chunks' partial
// sums are added per node in chunk order, so the result does not depend on
// the schedule.
constexpr int kLumChunk = 1024;

__device__ inline double spline_w(double d, double h)
{
    const double q = d / h;
    const double a = fmax(2.0 - q, 0.0), b = fmax(1.0 - q, 0.0);
    return (0.25 * a * a * a - b * b * b) / (M_PI * h * h * h);
}

// (h, V) of every source in sorted order, with the arguments' validation.
__global__ void __launch_bounds__(kThreads) lum_gather(int64_t n, const unsigned *perm, const double *h,
                                                       const double *vol, int form, double2 *hv, unsigned *flags)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const unsigned j = perm[k];
    const double hj = h[j];
    const double vj = form == 2 ? vol[j] : 0.0;
    unsigned bad = 0;
    if (!isfinite(hj) || !isfinite(vj))
        bad = kFlagNonFinite;
    else if (!(hj > 0.0) || vj < 0.0)
        bad = kFlagNegative;
    if (bad) atomicOr(flags, bad);
    hv[k] = make_double2(hj, vj);
}

// Chunks of every node (0 for single sources); element m is 0 so that the
// exclusive scan ends with the total.
__global__ void __launch_bounds__(kThreads) lum_chunks(int64_t m, const int4 *geo, const int *count,
                                                       unsigned *nchunk)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p > m) return;
    unsigned c = 0;
    if (p < m && (geo[p].w >> 8) != kKindLeaf) c = (unsigned)((count[p] + kLumChunk - 1) / kLumChunk);
    nchunk[p] = c;
}

__global__ void __launch_bounds__(kThreads) lum_owner(int64_t m, const unsigned *off, unsigned *owner)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    for (unsigned i = off[p]; i < off[p + 1]; ++i) owner[i] = (unsigned)p;
}

__global__ void __launch_bounds__(kThreads) lum_partial(int64_t n_chunks, const unsigned *owner,
                                                        const unsigned *off, const int *first, const int *count,
                                                        const double4 *mom, const double4 *src, const double2 *hv,
                                                        int form, double2 *part)
{
    const int64_t t = (int64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    const int lane = (int)(threadIdx.x & 63);
    if (t >= n_chunks) return;   // the whole wave
    const unsigned p = owner[t];
    const int64_t beg = (int64_t)first[p] + (t - (int64_t)off[p]) * kLumChunk;
    const int64_t end = min((int64_t)first[p] + count[p], beg + kLumChunk);
    const double4 r = mom[p];
    double num = 0.0, den = 0.0;
    for (int64_t k = beg + lane; k < end; k += 64) {
        const double4 s = src[k];
        const double2 q = hv[k];
        const double dx = r.x - s.x, dy = r.y - s.y, dz = r.z - s.z;
        const double w = spline_w(sqrt(dx * dx + dy * dy + dz * dz), q.x);
        num += (form == 2 ? q.y * s.w : s.w) * w;
        den += w;
    }
    for (int o = 32; o > 0; o >>= 1) {
        num += __shfl_xor(num, o, 64);
        den += __shfl_xor(den, o, 64);
    }
    if (lane == 0) part[t] = make_double2(num, den);
}

__global__ void __launch_bounds__(kThreads) lum_finish(int64_t m, const unsigned *off, const double2 *part,
                                                       int form, double4 *mom)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    const unsigned a = off[p], b = off[p + 1];
    if (a == b) return;   // a single source keeps its own luminosity
    double num = 0.0, den = 0.0;
    for (unsigned i = a; i < b; ++i) {
        num += part[i].x;
        den += part[i].y;
    }
    mom[p].w = form == 1 ? (den > 0.0 ? num / den : 0.0) : num;
}

// Largest luminosity of any node or source (as the bits of a non-negative
// double, which order like the values), one atomic per block.
__global__ void __launch_bounds__(kThreads) lum_max(int64_t m, const double4 *mom, int64_t n, const double4 *src,
                                                    unsigned long long *best)
{
    __shared__ unsigned long long red[kThreads / 64];
    unsigned long long v = 0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < m + n; i += (int64_t)gridDim.x * kThreads) {
        const double L = i < m ? mom[i].w : src[i - m].w;
        const unsigned long long b = (unsigned long long)__double_as_longlong(L);
        v = b > v ? b : v;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long u = __shfl_xor(v, o, 64);
        v = u > v ? u : v;
    }
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kThreads / 64; ++w) v = red[w] > v ? red[w] : v;
        if (v) atomicMax(best, v);
    }
}

__global__ void lum_scale(const unsigned long long *best, double *lscale)
{
    if (threadIdx.x == 0) lscale[0] = *best ? __longlong_as_double((long long)*best) : 1.0;
}

// New luminosities of the same sources, in sorted order (for a refit inside
// the equilibrium loop, whose emission they are); a negative or non-finite
// value raises the equilibrium-input flag of the sticky word.
__global__ void __launch_bounds__(kThreads) set_lum(int64_t n, const unsigned *perm, const double *lum,
                                                    double4 *src, unsigned *flags)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const double L = lum[perm[k]];
    if (!(L >= 0.0) || !isfinite(L)) atomicOr(flags, kFlagEqInput);
    src[k].w = L;
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

// Work arrays of a refit: node levels (computed once) and the moment sums.
size_t refit_bytes(const Tree *t)
{
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return al((size_t)t->n_nodes * sizeof(double4)) + al((size_t)t->n_nodes);
}

void refit_prepare(Ctx *c, const Tree *t, void *work)
{
    const int64_t m = t->n_nodes;
    if (m == 0) return;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    unsigned char *lvl = (unsigned char *)work + al((size_t)m * sizeof(double4));
    node_levels<<<blocks_for(m), kThreads, 0, c->stream>>>(m, t->geo, lvl);
}

// The same tree for new luminosities of the same sources: keys, order and
// nodes depend on the positions only, so only the sorted luminosities, the
// moments of eqs. (14)-(15) (with the build's own kernels, so the result is
// the rebuilt tree bit for bit) and the FP32 unit are redone.  Asynchronous;
// bad luminosities are reported by the next start_synchronize (as an
// equilibrium input).  `work` holds refit_bytes(t) after refit_prepare.
void refit_tree(Ctx *c, Tree *t, const double *lum, void *work)
{
    const int64_t m = t->n_nodes, n = t->n_src;
    if (n == 0) return;
    hipStream_t s = c->stream;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    double4 *msum = (double4 *)work;
    const unsigned char *lvl = (const unsigned char *)work + al((size_t)m * sizeof(double4));
    set_lum<<<blocks_for(n), kThreads, 0, s>>>(n, t->perm, lum, t->src, c->d_flags);
    for (int lv = 0; lv <= kMaxLevel; ++lv)
        moments_level<<<blocks_for(m), kThreads, 0, s>>>(m, lv, lvl, t->geo, t->skip, t->first, t->count, t->src,
                                                         msum);
    moments_finish<<<blocks_for(m), kThreads, 0, s>>>(m, t->geo, t->first, t->src, msum, t->mom);
    root_scale<<<1, 64, 0, s>>>(t->mom, t->lscale);
}

start_status tree_kernel_luminosity(Ctx *c, Tree *t, const double *h, const double *vol, int form)
{
    const int64_t m = t->n_nodes, n = t->n_src;
    if (n == 0) return START_OK;
    hipStream_t s = c->stream;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const size_t b_hv = al(n * sizeof(double2)), b_off = al((m + 1) * sizeof(unsigned));
    const size_t bytes1 = b_hv + b_off + al(scan_temp_bytes(m + 1)) + 256;
    char *t1 = nullptr;
    if (dmalloc(c, (void **)&t1, bytes1) != hipSuccess) return START_ENOMEM;
    double2 *hv = (double2 *)t1;
    unsigned *off = (unsigned *)(t1 + b_hv);
    void *scan_tmp = t1 + b_hv + b_off;
    unsigned long long *best = (unsigned long long *)(t1 + bytes1 - 256);
    unsigned *bflags = c->d_flags + 1;   // build validation word
    hipMemsetAsync(bflags, 0, sizeof(unsigned), s);
    hipMemsetAsync(best, 0, sizeof(*best), s);
    lum_gather<<<blocks_for(n), kThreads, 0, s>>>(n, t->perm, h, vol, form, hv, bflags);
    lum_chunks<<<blocks_for(m + 1), kThreads, 0, s>>>(m, t->geo, t->count, off);
    exclusive_scan_u32(off, m + 1, scan_tmp, s);
    unsigned flags = 0, n_chunks = 0;
    hipMemcpyAsync(&flags, bflags, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    hipMemcpyAsync(&n_chunks, off + m, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    hipError_t e = hipStreamSynchronize(s);
    if (e != hipSuccess || flags) {
        dfree(c, t1, bytes1);
        if (e != hipSuccess) {
            c->err = hipGetErrorString(e);
            return START_EHIP;
        }
        if (flags & kFlagNonFinite) {
            c->err = "non-finite smoothing length or volume";
            return START_ENONFINITE;
        }
        c->err = "smoothing length <= 0 or negative volume";
        return START_EINVAL;
    }
    char *t2 = nullptr;
    const size_t b_part = al((size_t)n_chunks * sizeof(double2));
    const size_t bytes2 = b_part + al((size_t)n_chunks * sizeof(unsigned));
    if (n_chunks > 0 && dmalloc(c, (void **)&t2, bytes2) != hipSuccess) {
        dfree(c, t1, bytes1);
        return START_ENOMEM;
    }
    if (n_chunks > 0) {
        double2 *part = (double2 *)t2;
        unsigned *owner = (unsigned *)(t2 + b_part);
        lum_owner<<<blocks_for(m), kThreads, 0, s>>>(m, off, owner);
        const unsigned waves_per_block = kThreads / 64;
        lum_partial<<<(unsigned)((n_chunks + waves_per_block - 1) / waves_per_block), kThreads, 0, s>>>(
            n_chunks, owner, off, t->first, t->count, t->mom, t->src, hv, form, part);
        lum_finish<<<blocks_for(m), kThreads, 0, s>>>(m, off, part, form, t->mom);
    }
    const int64_t items = m + n;
    const unsigned mb = (unsigned)std::min<int64_t>((items + kThreads - 1) / kThreads, 1024);
    lum_max<<<mb, kThreads, 0, s>>>(m, t->mom, n, t->src, best);
    lum_scale<<<1, 64, 0, s>>>(best, t->lscale);
    e = hipStreamSynchronize(s);
    if (t2) dfree(c, t2, bytes2);
    dfree(c, t1, bytes1);
    if (e != hipSuccess) {
        c->err = hipGetErrorString(e);
        return START_EHIP;
    }
    return START_OK;
}

void launch_keys(const start_box &box, int64_t n, const double *xyz, const double *lum, uint64_t *keys,
                 unsigned *idx, unsigned *flags, hipStream_t s)
{
    if (n <= 0) return;
    const double inv = 1.0 / box.size;
    keys_kernel<<<blocks_for(n), kThreads, 0, s>>>(box, inv, n, xyz, lum, keys, idx, flags);
}

// Builds the octree; all allocations are owned by the tree.  Synchronises once
// (to learn the node count and the validation flags).
start_status build_tree(Ctx *c, const start_box &box, int64_t n, const double *xyz, const double *lum,
                        Tree *t)
{
    hipStream_t s = c->stream;
    t->box = box;
    t->n_src = n;
    t->ctx = c;
    if (n == 0) return START_OK;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int ni = (int)n;
    const int64_t max_items = 2 * n;
    // persistent arrays
    size_t persist = al(n * sizeof(uint64_t)) + al(n * sizeof(unsigned)) + al(n * sizeof(double4)) +
                     al(n * sizeof(uint4)) + al(max_items * sizeof(int4)) + 4 * al(max_items * sizeof(int)) +
                     al(max_items * sizeof(double4)) + al(max_items * sizeof(uint4)) + al(sizeof(double)) +
                     al(max_items * sizeof(double4));
    char *pm = nullptr;
    if (dmalloc(c, (void **)&pm, persist) != hipSuccess) return START_ENOMEM;
    t->bytes = persist;
    char *q = pm;
    auto take = [&](size_t b) { char *r = q; q += al(b); return r; };
    t->keys = (uint64_t *)take(n * sizeof(uint64_t));
    t->perm = (unsigned *)take(n * sizeof(unsigned));
    t->src = (double4 *)take(n * sizeof(double4));
    t->srcq = (uint4 *)take(n * sizeof(uint4));
    t->geo = (int4 *)take(max_items * sizeof(int4));
    t->skip = (int *)take(max_items * sizeof(int));
    t->first = (int *)take(max_items * sizeof(int));
    t->count = (int *)take(max_items * sizeof(int));
    t->ref = (int *)take(max_items * sizeof(int));
    t->mom = (double4 *)take(max_items * sizeof(double4));
    t->momq = (uint4 *)take(max_items * sizeof(uint4));
    t->lscale = (double *)take(sizeof(double));
    t->bnd = (double4 *)take(max_items * sizeof(double4));

    // temporaries
    size_t tmp_bytes = al(radix_temp_bytes(max_items)) + 6 * al(n * sizeof(int)) + 2 * al(n * sizeof(unsigned)) +
                       al((n + 1) * sizeof(unsigned)) + al(max_items * sizeof(uint64_t)) +
                       al(max_items * sizeof(unsigned)) + al(scan_temp_bytes(n + 1)) + al(max_items * sizeof(double4)) +
                       al(max_items) + 256;
    char *tm = nullptr;
    if (dmalloc(c, (void **)&tm, tmp_bytes) != hipSuccess) {
        dfree(c, pm, persist);
        return START_ENOMEM;
    }
    q = tm;
    void *radix_tmp = take(radix_temp_bytes(max_items));
    int *blo = (int *)take(n * sizeof(int));
    int *bhi = (int *)take(n * sizeof(int));
    int *bdelta = (int *)take(n * sizeof(int));
    int *bparent = (int *)take(n * sizeof(int));
    unsigned *flag_int = (unsigned *)take(n * sizeof(int));
    unsigned *flag_leaf = (unsigned *)take(n * sizeof(int));
    unsigned *pos_int = (unsigned *)take(n * sizeof(unsigned));
    unsigned *pos_leaf = (unsigned *)take(n * sizeof(unsigned));
    unsigned *first_count = (unsigned *)take((n + 1) * sizeof(unsigned));
    uint64_t *item_key = (uint64_t *)take(max_items * sizeof(uint64_t));
    unsigned *item_code = (unsigned *)take(max_items * sizeof(unsigned));
    void *scan_tmp = take(scan_temp_bytes(n + 1));
    double4 *msum = (double4 *)take(max_items * sizeof(double4));
    unsigned char *lvl = (unsigned char *)take(max_items);
    unsigned *counts_host_dev = (unsigned *)take(256);

    unsigned *bflags = c->d_flags + 1;   // build validation word (not the rate calls' one)
    hipMemsetAsync(bflags, 0, sizeof(unsigned), s);
    launch_keys(box, n, xyz, lum, t->keys, t->perm, bflags, s);
    radix_sort_pairs(t->keys, t->perm, n, 63, radix_tmp, s);
    invert_order<<<blocks_for(n), kThreads, 0, s>>>(n, t->perm, pos_int);   // pos_int is free until the scans
    scatter_sources<<<blocks_for(n), kThreads, 0, s>>>(n, pos_int, xyz, lum, t->src);

    unsigned n_int = 0, n_leaf = 0;
    if (n > 1) {
        radix_tree_kernel<<<blocks_for(n - 1), kThreads, 0, s>>>(t->keys, ni, blo, bhi, bdelta, bparent);
    }
    mark_items<<<blocks_for(n), kThreads, 0, s>>>(t->keys, ni, blo, bdelta, bparent, flag_int, flag_leaf);
    // positions of the items: scans of the two flag arrays (count through the last element)
    hipMemcpyAsync(pos_int, flag_int, (size_t)n * sizeof(unsigned), hipMemcpyDeviceToDevice, s);
    hipMemcpyAsync(pos_leaf, flag_leaf, (size_t)n * sizeof(unsigned), hipMemcpyDeviceToDevice, s);
    if (n > 1) exclusive_scan_u32(pos_int, n - 1, scan_tmp, s);
    exclusive_scan_u32(pos_leaf, n, scan_tmp, s);
    unsigned h[4] = {0, 0, 0, 0};
    unsigned flags = 0;
    if (c->rb) {
        tree_readback<<<1, 64, 0, s>>>(ni, pos_int, flag_int, pos_leaf, flag_leaf, bflags, c->rb_dev);
    } else {
        if (n > 1) {
            hipMemcpyAsync(&h[0], pos_int + (n - 2), sizeof(unsigned), hipMemcpyDeviceToHost, s);
            hipMemcpyAsync(&h[1], flag_int + (n - 2), sizeof(unsigned), hipMemcpyDeviceToHost, s);
        }
        hipMemcpyAsync(&h[2], pos_leaf + (n - 1), sizeof(unsigned), hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(&h[3], flag_leaf + (n - 1), sizeof(unsigned), hipMemcpyDeviceToHost, s);
        hipMemcpyAsync(&flags, bflags, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess && c->rb) {
        const volatile unsigned *rb = c->rb;
        for (int k = 0; k < 4; ++k) h[k] = rb[k];
        flags = rb[4];
    }
    if (e != hipSuccess) {
        c->err = hipGetErrorString(e);
        dfree(c, tm, tmp_bytes);
        dfree(c, pm, persist);
        return START_EHIP;
    }
    if (flags) {
        dfree(c, tm, tmp_bytes);
        dfree(c, pm, persist);
        if (flags & kFlagNonFinite) { c->err = "non-finite source position or luminosity"; return START_ENONFINITE; }
        if (flags & kFlagOutOfBox) { c->err = "source outside the box"; return START_EOUTOFBOX; }
        c->err = "negative source luminosity";
        return START_EINVAL;
    }
    n_int = n > 1 ? h[0] + h[1] : 0;
    n_leaf = h[2] + h[3];
    const int64_t m = (int64_t)n_int + n_leaf;
    t->n_nodes = m;

    hipMemsetAsync(first_count, 0, (size_t)(n + 1) * sizeof(unsigned), s);
    emit_items<<<blocks_for(n), kThreads, 0, s>>>(ni, blo, bdelta, flag_int, pos_int, flag_leaf, pos_leaf, n_int,
                                                  item_key, item_code, first_count);
    int bits = 5;
    while ((int64_t(1) << (bits - 5)) < n) ++bits;
    radix_sort_pairs(item_key, item_code, m, bits, radix_tmp, s);
    exclusive_scan_u32(first_count, n + 1, scan_tmp, s);   // pos_start[i] = items with first < i
    fill_nodes<<<blocks_for(m), kThreads, 0, s>>>(ni, m, t->keys, t->perm, blo, bhi, bdelta, item_code, first_count,
                                                  t->geo, t->skip, t->first, t->count, t->ref, t->bnd);
    node_levels<<<blocks_for(m), kThreads, 0, s>>>(m, t->geo, lvl);
    for (int lv = 0; lv <= kMaxLevel; ++lv)
        moments_level<<<blocks_for(m), kThreads, 0, s>>>(m, lv, lvl, t->geo, t->skip, t->first, t->count, t->src,
                                                         msum);
    moments_finish<<<blocks_for(m), kThreads, 0, s>>>(m, t->geo, t->first, t->src, msum, t->mom);
    root_scale<<<1, 64, 0, s>>>(t->mom, t->lscale);
    e = hipStreamSynchronize(s);
    dfree(c, tm, tmp_bytes);
    (void)counts_host_dev;
    if (e != hipSuccess) {
        c->err = hipGetErrorString(e);
        return START_EHIP;
    }
    return START_OK;
}

}  // namespace start
