// Optical depths by the upstream-particle chain of section 2.2.1 (eqs. 8-9)
// on the interaction lists of section 2.2.2, with the gas particles as the
// targets.
//
// For a pair p = (particle i, list entry alpha) the upstream particle is the
// neighbour j of i (|r_j - r_i| <= 2 h_i, j != i) that is closer to alpha's
// position, has alpha in its own list, and lies nearest to the ray (largest
// cos phi between r_i - r_alpha and r_j - r_alpha; the lowest j on ties).
// Then tau_p = tau_q + sigma (d_i - d_j) (n_HI,i + n_HI,j) / 2 with q = (j,
// alpha); pairs without an upstream particle (list-boundary particles)
// integrate along the ray.  The paper walks each list in order of distance;
// here every pair finds its upstream pair at once (binary search of alpha in
// the neighbour's sorted list), and the sums along the resulting forest are
// taken by pointer jumping: after round k every pair holds the sum of its
// first 2^k links, so log2(depth) rounds finish all chains.
#include "internal.h"

namespace start {

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// Neighbours within 2 h_i, found through the particles binned by grid cell:
// each neighbour's index and the place of its binned record.
template <bool FILL>
__global__ void __launch_bounds__(kThreads) neighbours(int64_t n, const double *__restrict__ xyz,
                                                       const double *__restrict__ h, start_box box, double delta,
                                                       int G, int K, const unsigned *__restrict__ start,
                                                       const double4 *__restrict__ pos_h,
                                                       const unsigned *__restrict__ idx, unsigned *__restrict__ count,
                                                       const unsigned *__restrict__ nb_off, unsigned *__restrict__ nb,
                                                       unsigned *__restrict__ nbs)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
    const double r = 2.0 * h[i];
    const double r2 = r * r;
    int lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
        // one cell of margin: the binning rounds positions on its own
        const double gl = (x[k] - r - box.lo[k]) / delta, gh = (x[k] + r - box.lo[k]) / delta;
        int a = (int)floor(gl) - 1, b = (int)floor(gh) + 1;
        lo[k] = a < 0 ? 0 : (a > G - 1 ? G - 1 : a);
        hi[k] = b < 0 ? 0 : (b > G - 1 ? G - 1 : b);
    }
    unsigned c = 0;
    const unsigned base = FILL ? nb_off[i] : 0u;
    const int64_t ncell = (int64_t)G * G * G;
    for (int k = 0; k < K; ++k)   // every reach class of the binning
    for (int a = lo[0]; a <= hi[0]; ++a)
        for (int b = lo[1]; b <= hi[1]; ++b) {
            const int64_t row = k * ncell + ((int64_t)a * G + b) * G;
            const unsigned s0 = start[row + lo[2]], s1 = start[row + hi[2] + 1];
            for (unsigned s = s0; s < s1; ++s) {
                const unsigned j = idx[s];
                if (j == (unsigned)i) continue;
                const double4 q = pos_h[s];
                const double ex = q.x - x[0], ey = q.y - x[1], ez = q.z - x[2];
                if (!(ex * ex + ey * ey + ez * ez <= r2)) continue;
                if (FILL) {
                    nb[base + c] = j;
                    nbs[base + c] = s;   // its binned record (x, y, z, h)
                }
                ++c;
            }
        }
    if (!FILL) count[i] = c;
}

__global__ void __launch_bounds__(kThreads) pair_owner(int64_t n, const unsigned *__restrict__ off,
                                                       unsigned *__restrict__ owner)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    for (unsigned p = off[i]; p < off[i + 1]; ++p) owner[p] = (unsigned)i;
}

__device__ inline double dist3(const double x[3], const double4 &a)
{
    const double dx = x[0] - a.x, dy = x[1] - a.y, dz = x[2] - a.z;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// Upstream pair of every pair (or -1) and its step sigma (d_i - d_j) ucm
// (n_i + n_j) / 2; root pairs are appended to `roots`.
__global__ void __launch_bounds__(kThreads) upstream_parent(
    int64_t n_pairs, int64_t n, const double *__restrict__ xyz, const double *__restrict__ nhi,
    const unsigned *__restrict__ off, const uint64_t *__restrict__ keys, const unsigned *__restrict__ owner,
    const unsigned *__restrict__ nb_off, const unsigned *__restrict__ nb, const unsigned *__restrict__ nbs,
    const double4 *__restrict__ pos_h, const double4 *__restrict__ mom,
    const double4 *__restrict__ src, const int *__restrict__ first, double sigma, double ucm,
    int *__restrict__ parent, double *__restrict__ acc, unsigned *__restrict__ roots, unsigned *__restrict__ n_roots)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n_pairs) return;
    const unsigned i = owner[p];
    const uint64_t key = keys[p];
    const unsigned li = off[i], ni = off[i + 1] - li, rank = (unsigned)(p - li);   // alpha's place in i's list
    const double4 a = source_of_key(mom, src, first, key);
    const double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
    const double di = dist3(x, a);
    int best = -1;
    unsigned bj = 0;
    double bc = 0.0, bd = 0.0;
    // the next neighbour's index, list bounds and position are loaded one
    // iteration ahead, so that the loads of successive neighbours overlap;
    // the position comes from the binned record (one line, not three)
    const unsigned t0 = nb_off[i], t1 = nb_off[i + 1];
    unsigned jn = 0, ljn = 0, ljn1 = 0;
    double4 qn = make_double4(0.0, 0.0, 0.0, 0.0);
    if (t0 < t1) {
        jn = nb[t0];
        qn = pos_h[nbs[t0]];
        ljn = off[jn];
        ljn1 = off[jn + 1];
    }
    for (unsigned t = t0; t < t1; ++t) {
        const unsigned j = jn;
        const unsigned lj = ljn, nj = ljn1 - ljn;
        const double y[3] = {qn.x, qn.y, qn.z};
        if (t + 1 < t1) {
            jn = nb[t + 1];
            qn = pos_h[nbs[t + 1]];
            ljn = off[jn];
            ljn1 = off[jn + 1];
        }
        // the geometric conditions first (strictly closer to the source, and
        // closer to the ray than the best so far), so that only a candidate
        // that would be taken is looked up: the same choice as testing them
        // after the search, with far fewer searches
        const double dj = dist3(y, a);
        if (!(dj < di)) continue;
        const double dot = (x[0] - a.x) * (y[0] - a.x) + (x[1] - a.y) * (y[1] - a.y) + (x[2] - a.z) * (y[2] - a.z);
        const double c = dot / (di * dj);
        if (!(best < 0 || c > bc || (c == bc && j < bj))) continue;
        // alpha in j's list (keys ascending).  Neighbours' lists are nearly
        // the same, so the search starts at alpha's place in i's list,
        // scaled to j's length, and gallops to a bracket before bisecting:
        // the same lower bound as a plain bisection of the whole list, with
        // a few nearby loads instead of ~log2(length) scattered ones.
        if (nj == 0) continue;
        const uint64_t *kj = keys + lj;
        unsigned g = ni > 0 ? (unsigned)(((uint64_t)rank * nj) / ni) : 0u;
        g = g < nj ? g : nj - 1;
        unsigned lo, hi;
        if (kj[g] < key) {          // the lower bound is above g
            lo = g + 1;
            unsigned b = 1;
            while (g + b < nj && kj[g + b] < key) {
                lo = g + b + 1;
                b <<= 1;
            }
            hi = g + b < nj ? g + b : nj;
        } else {                    // the lower bound is at most g
            hi = g;
            unsigned b = 1;
            while (b <= g && kj[g - b] >= key) {
                hi = g - b;
                b <<= 1;
            }
            lo = b <= g ? g - b + 1 : 0u;
        }
        while (lo < hi) {
            const unsigned mid = (lo + hi) >> 1;
            if (kj[mid] < key) lo = mid + 1;
            else hi = mid;
        }
        if (lo >= nj || kj[lo] != key) continue;
        best = (int)(lo + lj);
        bj = j;
        bc = c;
        bd = dj;
    }
    parent[p] = best;
    if (best >= 0) {
        acc[p] = sigma * ((di - bd) * ucm) * (0.5 * (nhi[i] + nhi[bj]));
    } else {
        const unsigned r = atomicAdd(n_roots, 1u);
        roots[r] = (unsigned)p;
    }
}

// Pointer jumping on (tau, parent) records of 16 bytes: one round sets
// acc += acc[parent] and parent = parent[parent], reading the parent's two
// values from one cache line (the parents are scattered over the whole pair
// array, so two separate arrays cost two lines per pair).
struct __align__(16) Link {
    double acc;
    int par;
    int pad;
};

__global__ void __launch_bounds__(kThreads) pack_links(int64_t n_pairs, const int *__restrict__ par,
                                                       const double *__restrict__ acc, Link *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n_pairs) return;
    Link l;
    l.acc = acc[p];
    l.par = par[p];
    l.pad = 0;
    out[p] = l;
}

__global__ void __launch_bounds__(kThreads) jump_links(int64_t n_pairs, const Link *__restrict__ in,
                                                       Link *__restrict__ out, unsigned *__restrict__ more)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n_pairs) return;
    const Link a = in[p];
    if (a.par < 0) {
        out[p] = a;
        return;
    }
    const Link b = in[a.par];
    Link l;
    l.acc = a.acc + b.acc;
    l.par = b.par;
    l.pad = 0;
    out[p] = l;
    if (b.par >= 0) *more = 1u;
}

__global__ void __launch_bounds__(kThreads) unpack_acc(int64_t n_pairs, const Link *__restrict__ in,
                                                       double *__restrict__ acc)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n_pairs) return;
    acc[p] = in[p].acc;
}

// Gamma_i = sigma / (4 pi) sum_p L e^-tau / d_cm^2 over the pairs of i in list
// order (eq. A2).
__global__ void __launch_bounds__(kThreads) upstream_gamma(int64_t n, const double *__restrict__ xyz,
                                                           const unsigned *__restrict__ off,
                                                           const uint64_t *__restrict__ keys,
                                                           const double *__restrict__ tau,
                                                           const double4 *__restrict__ mom,
                                                           const double4 *__restrict__ src,
                                                           const int *__restrict__ first, double sigma, double ucm,
                                                           double *__restrict__ gamma)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
    double sum = 0.0;
    for (unsigned p = off[i]; p < off[i + 1]; ++p) {
        const double4 a = source_of_key(mom, src, first, keys[p]);
        const double d = dist3(x, a);
        if (d == 0.0) continue;
        const double dcm = d * ucm;
        sum += a.w * exp(-tau[p]) / (dcm * dcm);
    }
    gamma[i] = sigma / (4.0 * M_PI) * sum;
}

__global__ void __launch_bounds__(kThreads) to_u32(int64_t n, const int64_t *__restrict__ in, unsigned *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) out[i] = (unsigned)in[i];
}

// 64-bit sum of non-negative counts: a block sum (wave reductions, then one
// 64-bit atomic per block)
__global__ void __launch_bounds__(kThreads) sum_i64(int64_t n, const int64_t *__restrict__ in,
                                                    unsigned long long *__restrict__ total)
{
    __shared__ unsigned long long part[kThreads / 64];
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    unsigned long long v = i < n ? (unsigned long long)in[i] : 0ull;
    for (int d = 32; d > 0; d >>= 1) v += __shfl_down(v, d, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long b = 0;
        for (int w = 0; w < kThreads / 64; ++w) b += part[w];
        atomicAdd(total, b);
    }
}

__global__ void __launch_bounds__(kThreads) to_i64(int64_t n, const unsigned *__restrict__ in, int64_t *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) out[i] = (int64_t)in[i];
}

// parent pair -> upstream particle index (or -1), for the export
__global__ void __launch_bounds__(kThreads) parent_particle(int64_t n_pairs, const int *__restrict__ parent,
                                                            const unsigned *__restrict__ owner,
                                                            int64_t *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n_pairs) return;
    const int q = parent[p];
    out[p] = q < 0 ? -1 : (int64_t)owner[q];
}

}  // namespace

void launch_to_u32(Ctx *c, int64_t n, const int64_t *in, unsigned *out)
{
    if (n > 0) to_u32<<<blocks_for(n), kThreads, 0, c->stream>>>(n, in, out);
}

void launch_sum_i64(Ctx *c, int64_t n, const int64_t *in, unsigned long long *total)
{
    if (n > 0) sum_i64<<<blocks_for(n), kThreads, 0, c->stream>>>(n, in, total);
}

void launch_to_i64(Ctx *c, int64_t n, const unsigned *in, int64_t *out)
{
    if (n > 0) to_i64<<<blocks_for(n), kThreads, 0, c->stream>>>(n, in, out);
}

void launch_neighbours(Ctx *c, const GasBins &b, int64_t n, const double *xyz, const double *h, unsigned *count,
                       const unsigned *nb_off, unsigned *nb, unsigned *nbs)
{
    if (n <= 0) return;
    if (!nb_off)
        neighbours<false><<<blocks_for(n), kThreads, 0, c->stream>>>(n, xyz, h, b.box, b.delta, b.G, b.cls.K, b.start, b.pos_h,
                                                                     b.idx, count, nullptr, nullptr, nullptr);
    else
        neighbours<true><<<blocks_for(n), kThreads, 0, c->stream>>>(n, xyz, h, b.box, b.delta, b.G, b.cls.K, b.start, b.pos_h,
                                                                    b.idx, nullptr, nb_off, nb, nbs);
}

void launch_pair_owner(Ctx *c, int64_t n, const unsigned *off, unsigned *owner)
{
    if (n > 0) pair_owner<<<blocks_for(n), kThreads, 0, c->stream>>>(n, off, owner);
}

void launch_upstream_parent(Ctx *c, const Tree *t, int64_t n_pairs, int64_t n, const double *xyz, const double *nhi,
                            const unsigned *off, const uint64_t *keys, const unsigned *owner, const unsigned *nb_off,
                            const unsigned *nb, const unsigned *nbs, const double4 *pos_h, double sigma, int *parent,
                            double *acc, unsigned *roots, unsigned *n_roots)
{
    if (n_pairs <= 0) return;
    upstream_parent<<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(
        n_pairs, n, xyz, nhi, off, keys, owner, nb_off, nb, nbs, pos_h, t->mom, t->src, t->first, sigma,
        t->box.length_unit_cm, parent, acc, roots, n_roots);
}

void launch_pack_links(Ctx *c, int64_t n_pairs, const int *par, const double *acc, void *links)
{
    if (n_pairs > 0) pack_links<<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(n_pairs, par, acc, (Link *)links);
}

void launch_jump_links(Ctx *c, int64_t n_pairs, const void *in, void *out, unsigned *more)
{
    if (n_pairs > 0)
        jump_links<<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(n_pairs, (const Link *)in, (Link *)out, more);
}

void launch_unpack_acc(Ctx *c, int64_t n_pairs, const void *links, double *acc)
{
    if (n_pairs > 0) unpack_acc<<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(n_pairs, (const Link *)links, acc);
}

void launch_upstream_gamma(Ctx *c, const Tree *t, int64_t n, const double *xyz, const unsigned *off,
                           const uint64_t *keys, const double *tau, double sigma, double *gamma)
{
    if (n > 0)
        upstream_gamma<<<blocks_for(n), kThreads, 0, c->stream>>>(n, xyz, off, keys, tau, t->mom, t->src, t->first,
                                                                  sigma, t->box.length_unit_cm, gamma);
}

void launch_parent_particle(Ctx *c, int64_t n_pairs, const int *parent, const unsigned *owner, int64_t *out)
{
    if (n_pairs > 0) parent_particle<<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(n_pairs, parent, owner, out);
}

}  // namespace start
