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

// A neighbour j of a particle as the upstream search reads it: position and
// index (one contiguous 32-byte record per neighbour, so that the search
// streams through them without dependent loads).
struct __align__(16) NbRec {
    double x, y, z;
    unsigned j, pad;
};

// Neighbours within 2 h_i, found through the particles binned by grid cell.
// One wave per particle (the particles taken in Morton order, perm): its
// lanes take one row of cells each (per reach class, x and y of the search
// box), cut to the cells that the sphere of radius 2h reaches, and step
// through their rows' particles together; a ballot of the
// ones within 2h gives each its place, so the records come out in a fixed
// order (row chunk, step, lane).  FILL = false writes the count to count[i];
// FILL = true writes the records from nb_off[i] (the counts scanned).
template <bool FILL>
__global__ void __launch_bounds__(kThreads) neighbours(int64_t n, const unsigned *__restrict__ perm,
                                                       const double *__restrict__ xyz,
                                                       const double *__restrict__ h, start_box box, double delta,
                                                       int G, int K, const unsigned *__restrict__ start,
                                                       const double4 *__restrict__ pos_h,
                                                       const unsigned *__restrict__ idx, unsigned *__restrict__ count,
                                                       const unsigned *__restrict__ nb_off, NbRec *__restrict__ rec)
{
    const int64_t w = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
    const unsigned lane = threadIdx.x & 63u;
    if (w >= n) return;         // whole waves leave together
    const unsigned i = perm[w];
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
    const int nb = hi[1] - lo[1] + 1;
    const int per_class = (hi[0] - lo[0] + 1) * nb;
    const int rows = K * per_class;
    const int64_t ncell = (int64_t)G * G * G;
    const unsigned base = FILL ? nb_off[i] : 0u;
    unsigned total = 0;         // the same in every lane
    for (int r0 = 0; r0 < rows; r0 += 64) {
        const int rw = r0 + (int)lane;
        unsigned s0 = 0, len = 0;
        if (rw < rows) {
            const int k = rw / per_class, rem = rw - k * per_class;
            const int a = lo[0] + rem / nb, b = lo[1] + rem % nb;
            // the row's cells, widened by eps, against the sphere of radius
            // 2h: skip a row that misses it, and keep only the cells of the
            // chord through it (eps = 1e-6 cell covers the rounding of the
            // binning's floor((x - lo) G / size))
            const double eps = 1e-6 * delta;
            const double ax = box.lo[0] + a * delta, by = box.lo[1] + b * delta;
            const double dx = fmax(0.0, fmax(ax - eps - x[0], x[0] - (ax + delta + eps)));
            const double dy = fmax(0.0, fmax(by - eps - x[1], x[1] - (by + delta + eps)));
            const double dxy = dx * dx + dy * dy;
            if (dxy <= r2) {
                const double hz = sqrt(r2 - dxy);
                int z0 = (int)floor((x[2] - hz - eps - box.lo[2]) / delta);
                int z1 = (int)floor((x[2] + hz + eps - box.lo[2]) / delta);
                z0 = z0 < 0 ? 0 : (z0 > G - 1 ? G - 1 : z0);
                z1 = z1 < 0 ? 0 : (z1 > G - 1 ? G - 1 : z1);
                const int64_t row = k * ncell + ((int64_t)a * G + b) * G;
                s0 = start[row + z0];
                len = start[row + z1 + 1] - s0;
            }
        }
        unsigned steps = len;
        for (int d = 32; d > 0; d >>= 1) steps = max(steps, (unsigned)__shfl_xor((int)steps, d, 64));
        for (unsigned t = 0; t < steps; ++t) {
            bool take = false;
            unsigned j = 0;
            double4 q = make_double4(0.0, 0.0, 0.0, 0.0);
            if (t < len) {
                j = idx[s0 + t];
                q = pos_h[s0 + t];
                const double ex = q.x - x[0], ey = q.y - x[1], ez = q.z - x[2];
                take = j != i && ex * ex + ey * ey + ez * ez <= r2;
            }
            const uint64_t m = __ballot(take);
            if (FILL && take) {
                NbRec o;
                o.x = q.x;
                o.y = q.y;
                o.z = q.z;
                o.j = j;
                o.pad = 0u;
                rec[base + total + (unsigned)__popcll(m & ((1ull << lane) - 1ull))] = o;
            }
            total += (unsigned)__popcll(m);
        }
    }
    if (!FILL && lane == 0) count[i] = total;
}

// owner[p] = the particle of pair p; one wave per particle (coalesced writes)
__global__ void __launch_bounds__(kThreads) pair_owner(int64_t n, const uint2 *__restrict__ sl,
                                                       unsigned *__restrict__ owner)
{
    const int64_t i = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
    const unsigned lane = threadIdx.x & 63u;
    if (i >= n) return;
    const uint2 r = sl[i];
    for (unsigned k = lane; k < r.y; k += 64u) owner[r.x + k] = (unsigned)i;
}

// The pairs' layout: each particle's pairs stay contiguous, and the
// particles' runs follow the Morton order of their positions (perm: Morton
// rank -> particle), so that a neighbour's list and a pair's upstream pair
// lie near the pair itself instead of anywhere in the pair arrays.
// lc[r] = pair count of the particle of rank r (then scanned in place).
__global__ void __launch_bounds__(kThreads) layout_counts(int64_t n, const unsigned *__restrict__ perm,
                                                          const int64_t *__restrict__ counts,
                                                          unsigned *__restrict__ lc)
{
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r < n) lc[r] = (unsigned)counts[perm[r]];
}

// Morton keys cut to their top 30 bits (1024 cells per axis): order enough
// for the layout, in four radix passes instead of eight.
__global__ void __launch_bounds__(kThreads) coarse_keys(int64_t n, uint64_t *__restrict__ keys)
{
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r < n) keys[r] >>= 33;
}

// sl[i] = (first pair, pair count) and st[i] = first pair (64-bit, for the
// list writer) of every particle from the scanned counts in Morton order.
__global__ void __launch_bounds__(kThreads) layout_starts(int64_t n, const unsigned *__restrict__ perm,
                                                          const unsigned *__restrict__ lc,
                                                          uint2 *__restrict__ sl, int64_t *__restrict__ st)
{
    const int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (r >= n) return;
    const unsigned i = perm[r];
    sl[i] = make_uint2(lc[r], lc[r + 1] - lc[r]);
    st[i] = (int64_t)lc[r];
}

__device__ inline double dist3(const double x[3], const double4 &a)
{
    const double dx = x[0] - a.x, dy = x[1] - a.y, dz = x[2] - a.z;
    return sqrt(dx * dx + dy * dy + dz * dz);
}

// Place of `key` in the ascending keys kj[0, nj), or -1.  Neighbours' lists
// are nearly the same, so the search starts at guess g (the entry's place in
// the particle's own list, scaled to this list's length) and gallops to a
// bracket before bisecting: the same lower bound as a plain bisection of the
// whole list, with a few nearby loads instead of ~log2(length) scattered ones.
__device__ inline int find_key(const uint64_t *__restrict__ kj, unsigned nj, uint64_t key, unsigned g)
{
    if (nj == 0) return -1;
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
    return (lo < nj && kj[lo] == key) ? (int)lo : -1;
}

// Blocks are dealt round-robin to the 8 XCDs; give each XCD a contiguous run
// of blocks instead, so that the pairs one XCD works on (and the nearby
// pairs their neighbours' lists and parents sit in) share its L2.
__device__ inline int64_t xcd_block()
{
    const int nb = (int)gridDim.x;
    const int per = nb / 8;
    int blk = (int)blockIdx.x;
    if (per > 0 && blk < per * 8) blk = (blk & 7) * per + (blk >> 3);
    return blk;
}

// A pair's (tau, parent) record, 16 bytes.  Pointer jumping sets tau +=
// tau[parent] and parent = parent[parent] each round, reading the parent's
// two values from one cache line (two separate arrays cost two lines per
// scattered parent).
struct __align__(16) Link {
    double acc;
    int par;
    int pad;
};

// Dense index of a list entry: a node as itself, a bucket member as n_nodes
// plus its place in the sorted sources.
__device__ inline uint64_t entry_id(uint64_t key, const int *__restrict__ first, int64_t n_nodes)
{
    const int node = (int)(key >> 32);
    const unsigned m = (unsigned)(key & 0xffffffffu);
    return m == 0 ? (uint64_t)node : (uint64_t)n_nodes + (uint64_t)first[node] + m - 1u;
}

// Membership table: bit entry_id(alpha) of row i is set when alpha is in
// particle i's list (rows of W words).  One wave per particle builds its row
// in LDS (the entries of one list fall in few words, so global atomics from
// neighbouring lanes would wait on each other) and writes it out whole.
constexpr unsigned kRowWordsLds = 2048;     // rows up to 8 KiB per wave in LDS

// LDS writes of a wave's lanes made visible to the wave's other lanes
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ void __launch_bounds__(kThreads) member_rows(int64_t n, const uint64_t *__restrict__ keys,
                                                        const uint2 *__restrict__ sl, const int *__restrict__ first,
                                                        int64_t n_nodes, unsigned W, unsigned *__restrict__ bits)
{
    extern __shared__ unsigned rows[];
    unsigned *row = rows + (threadIdx.x >> 6) * W;
    const int64_t i = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
    const unsigned lane = threadIdx.x & 63u;
    if (i >= n) return;         // whole waves leave together
    for (unsigned w = lane; w < W; w += 64u) row[w] = 0u;
    wave_sync();
    const uint2 r = sl[i];
    for (unsigned p = r.x + lane; p < r.x + r.y; p += 64u) {
        const uint64_t id = entry_id(keys[p], first, n_nodes);
        atomicOr(row + (id >> 5), 1u << (unsigned)(id & 31u));
    }
    wave_sync();
    unsigned *out = bits + (size_t)i * W;
    for (unsigned w = lane; w < W; w += 64u) out[w] = row[w];
}

// The same for rows too long for LDS: one global atomic per pair (the table
// must be zeroed first).
__global__ void __launch_bounds__(kThreads) member_bits(int64_t n_pairs, const uint64_t *__restrict__ keys,
                                                        const unsigned *__restrict__ owner,
                                                        const int *__restrict__ first, int64_t n_nodes, unsigned W,
                                                        unsigned *__restrict__ bits)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n_pairs) return;
    const uint64_t id = entry_id(keys[p], first, n_nodes);
    atomicOr(bits + (size_t)owner[p] * W + (id >> 5), 1u << (unsigned)(id & 31u));
}

// Upstream pair of every pair (or -1) and its step sigma (d_i - d_j) ucm
// (n_i + n_j) / 2; root pairs are appended to `roots`.  sl[i] = (first pair,
// pair count) of particle i.
//
// The choice is the one the definition makes with the rounded values
// d = sqrt(d2) and cos phi = dot / (d_i d_j): among the neighbours with
// d_j < d_i that hold the source in their own list, the largest cos phi, the
// lowest index on ties.  The scan decides both comparisons from d2 and dot
// alone, without a square root or a division, wherever the margin is far
// wider than their rounding (d2_j below d2_i by more than 1e-14 relative;
// dot^2 d2_best against dot_best^2 d2_j by more than 1e-13, both dots
// positive) and falls back to the rounded values themselves otherwise, so
// the choice is the definition's bit for bit.
//
// Membership of the source in a neighbour's list: BITS = false searches the
// neighbour's sorted list for every neighbour that would be taken (the
// lanes of a wave wait for each other's searches); BITS = true reads one bit
// of the membership table per neighbour and searches only the chosen
// neighbour's list, once, at the end.
template <bool BITS>
__global__ void __launch_bounds__(kThreads) upstream_parent(
    int64_t n_pairs, int64_t n, const double *__restrict__ xyz, const double *__restrict__ nhi,
    const uint2 *__restrict__ sl, const uint64_t *__restrict__ keys, const unsigned *__restrict__ owner,
    const unsigned *__restrict__ nb_off, const NbRec *__restrict__ rec, const double4 *__restrict__ mom,
    const double4 *__restrict__ src, const int *__restrict__ first, int64_t n_nodes, const unsigned *__restrict__ bits,
    unsigned W, double sigma, double ucm, Link *__restrict__ links, unsigned *__restrict__ roots,
    unsigned *__restrict__ n_roots)
{
    const int64_t p = xcd_block() * kThreads + threadIdx.x;
    if (p >= n_pairs) return;
    const unsigned i = owner[p];
    const uint64_t key = keys[p];
    const uint2 si = sl[i];
    // alpha's place in i's list as a fraction: the first probe of the search
    // in a neighbour's list (any probe gives the same answer; a near one is
    // quicker)
    const float place = si.y > 0 ? (float)(unsigned)(p - si.x) / (float)si.y : 0.0f;
    const double4 a = source_of_key(mom, src, first, key);
    const double ux = xyz[i] - a.x, uy = xyz[n + i] - a.y, uz = xyz[2 * n + i] - a.z;
    const double d2i = ux * ux + uy * uy + uz * uz;
    const double di = sqrt(d2i);
    const double d2i_lo = d2i * (1.0 - 1e-14);
    unsigned wo = 0, bit = 0;
    if (BITS) {
        const uint64_t id = entry_id(key, first, n_nodes);
        wo = (unsigned)(id >> 5);
        bit = 1u << (unsigned)(id & 31u);
    }
    int best = -1;
    bool have = false;          // a neighbour taken
    unsigned bj = 0;
    double bdot = 0.0, bd2 = 0.0, bdot2 = 0.0;
    // the next neighbour's record is loaded one iteration ahead, so that the
    // loads of successive neighbours overlap; BITS: the neighbour's table
    // word is loaded as its iteration starts and used after the geometric
    // tests (loading it a neighbour ahead as well took more registers than
    // it hid latency)
    const unsigned t0 = nb_off[i], t1 = nb_off[i + 1];
    NbRec qn;
    qn.x = qn.y = qn.z = 0.0;
    qn.j = qn.pad = 0u;
    if (t0 < t1) qn = rec[t0];
    for (unsigned t = t0; t < t1; ++t) {
        const unsigned j = qn.j;
        const double ex = qn.x - a.x, ey = qn.y - a.y, ez = qn.z - a.z;
        const unsigned wc = BITS ? bits[(size_t)j * W + wo] : 0u;
        if (t + 1 < t1) qn = rec[t + 1];
        // strictly closer to the source: d_j < d_i
        const double d2j = ex * ex + ey * ey + ez * ez;
        if (!(d2j < d2i)) continue;
        if (!(d2j < d2i_lo)) {
            // within rounding of d_i: the rounded distances decide (kept a
            // branch of its own, not computed for every neighbour)
            asm volatile("" ::: "memory");
            if (!(sqrt(d2j) < di)) continue;
        }
        // closer to the ray than the best so far (the geometric conditions
        // before the search: only a neighbour that would be taken is looked
        // up in its list)
        const double dot = ux * ex + uy * ey + uz * ez;
        if (have) {
            bool take;
            const double l = (dot * dot) * bd2, r = bdot2 * d2j;
            if (dot > 0.0 && bdot > 0.0 && d2j > 0.0 && l > r * (1.0 + 1e-13)) {
                take = true;
            } else if (dot > 0.0 && bdot > 0.0 && d2j > 0.0 && l < r * (1.0 - 1e-13)) {
                take = false;
            } else {
                const double c = dot / (di * sqrt(d2j)), bc = bdot / (di * sqrt(bd2));
                take = c > bc || (c == bc && j < bj);
            }
            if (!take) continue;
        }
        if (BITS) {
            if (!(wc & bit)) continue;
        } else {
            const uint2 sj = sl[j];
            const int f = find_key(keys + sj.x, sj.y, key, (unsigned)(place * (float)sj.y));
            if (f < 0) continue;
            best = (int)(sj.x + (unsigned)f);
        }
        have = true;
        bj = j;
        bdot = dot;
        bd2 = d2j;
        bdot2 = dot * dot;
    }
    if (BITS && have) {
        // alpha's place in the chosen neighbour's list (present: its bit is set)
        const uint2 bsl = sl[bj];
        const int f = find_key(keys + bsl.x, bsl.y, key, (unsigned)(place * (float)bsl.y));
        best = f >= 0 ? (int)(bsl.x + (unsigned)f) : -1;
    }
    Link l;
    l.par = best;
    l.pad = 0;
    l.acc = 0.0;                // a root's column is set by the root march
    if (best >= 0) {
        l.acc = sigma * ((di - sqrt(bd2)) * ucm) * (0.5 * (nhi[i] + nhi[bj]));
    } else {
        const unsigned r = atomicAdd(n_roots, 1u);
        roots[r] = (unsigned)p;
    }
    links[p] = l;
}

__global__ void __launch_bounds__(kThreads) jump_links(int64_t n_pairs, const Link *__restrict__ in,
                                                       Link *__restrict__ out, unsigned *__restrict__ more)
{
    const int64_t p = xcd_block() * kThreads + threadIdx.x;
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

// Gamma_i = sigma / (4 pi) sum_p L e^-tau / d_cm^2 over the pairs of i
// (eq. A2).  One wave per particle: the lanes take the list's pairs in
// strides of 64 (coalesced reads of the keys and optical depths, where a
// thread per particle touched a line of each per pair) and add their partial
// sums by a butterfly, a fixed order for every call.
__global__ void __launch_bounds__(kThreads) upstream_gamma(int64_t n, const double *__restrict__ xyz,
                                                           const uint2 *__restrict__ sl,
                                                           const uint64_t *__restrict__ keys,
                                                           const Link *__restrict__ tau,
                                                           const double4 *__restrict__ mom,
                                                           const double4 *__restrict__ src,
                                                           const int *__restrict__ first, double sigma, double ucm,
                                                           double *__restrict__ gamma)
{
    const int64_t i = ((int64_t)blockIdx.x * kThreads + threadIdx.x) >> 6;
    const unsigned lane = threadIdx.x & 63u;
    if (i >= n) return;     // whole waves leave together
    const double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
    double sum = 0.0;
    const uint2 r = sl[i];
    for (unsigned p = r.x + lane; p < r.x + r.y; p += 64u) {
        const double4 a = source_of_key(mom, src, first, keys[p]);
        const double d = dist3(x, a);
        if (d == 0.0) continue;
        const double dcm = d * ucm;
        sum += a.w * exp(-tau[p].acc) / (dcm * dcm);
    }
    for (int m = 32; m > 0; m >>= 1) sum += __shfl_xor(sum, m, 64);
    if (lane == 0) gamma[i] = sigma / (4.0 * M_PI) * sum;
}

__global__ void __launch_bounds__(kThreads) to_u32(int64_t n, const int64_t *__restrict__ in, unsigned *__restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) out[i] = (unsigned)in[i];
}

// 64-bit sum of non-negative counts: a block sum (wave reductions, then one
// 64-bit atomic per block)
template <typename T>
__global__ void __launch_bounds__(kThreads) sum_counts(int64_t n, const T *__restrict__ in,
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

// parent pair -> upstream particle index (or -1), for the export, which
// keeps the particles' lists in particle order (offsets `ooff`)
__global__ void __launch_bounds__(kThreads) parent_particle(int64_t n_pairs, const Link *__restrict__ links,
                                                            const unsigned *__restrict__ owner,
                                                            const uint2 *__restrict__ sl,
                                                            const int64_t *__restrict__ ooff,
                                                            int64_t *__restrict__ out)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= n_pairs) return;
    const int q = links[p].par;
    const unsigned i = owner[p];
    out[ooff[i] + (p - (int64_t)sl[i].x)] = q < 0 ? -1 : (int64_t)owner[q];
}

}  // namespace

void launch_to_u32(Ctx *c, int64_t n, const int64_t *in, unsigned *out)
{
    if (n > 0) to_u32<<<blocks_for(n), kThreads, 0, c->stream>>>(n, in, out);
}

void launch_sum_i64(Ctx *c, int64_t n, const int64_t *in, unsigned long long *total)
{
    if (n > 0) sum_counts<int64_t><<<blocks_for(n), kThreads, 0, c->stream>>>(n, in, total);
}

void launch_sum_u32(Ctx *c, int64_t n, const unsigned *in, unsigned long long *total)
{
    if (n > 0) sum_counts<unsigned><<<blocks_for(n), kThreads, 0, c->stream>>>(n, in, total);
}

void launch_to_i64(Ctx *c, int64_t n, const unsigned *in, int64_t *out)
{
    if (n > 0) to_i64<<<blocks_for(n), kThreads, 0, c->stream>>>(n, in, out);
}

size_t neighbour_record_bytes() { return sizeof(NbRec); }

void launch_neighbours(Ctx *c, const GasBins &b, int64_t n, const unsigned *perm, const double *xyz, const double *h,
                       unsigned *count, const unsigned *nb_off, void *rec)
{
    if (n <= 0) return;
    if (!nb_off)
        neighbours<false><<<blocks_for(n * 64), kThreads, 0, c->stream>>>(n, perm, xyz, h, b.box, b.delta, b.G, b.cls.K,
                                                                     b.start, b.pos_h, b.idx, count, nullptr, nullptr);
    else
        neighbours<true><<<blocks_for(n * 64), kThreads, 0, c->stream>>>(n, perm, xyz, h, b.box, b.delta, b.G, b.cls.K,
                                                                    b.start, b.pos_h, b.idx, nullptr, nb_off,
                                                                    (NbRec *)rec);
}

void launch_pair_owner(Ctx *c, int64_t n, const uint2 *sl, unsigned *owner)
{
    if (n > 0) pair_owner<<<blocks_for(n * 64), kThreads, 0, c->stream>>>(n, sl, owner);
}

void launch_coarse_keys(Ctx *c, int64_t n, uint64_t *keys)
{
    if (n > 0) coarse_keys<<<blocks_for(n), kThreads, 0, c->stream>>>(n, keys);
}

void launch_layout_counts(Ctx *c, int64_t n, const unsigned *perm, const int64_t *counts, unsigned *lc)
{
    if (n > 0) layout_counts<<<blocks_for(n), kThreads, 0, c->stream>>>(n, perm, counts, lc);
}

void launch_layout_starts(Ctx *c, int64_t n, const unsigned *perm, const unsigned *lc, uint2 *sl, int64_t *st)
{
    if (n > 0) layout_starts<<<blocks_for(n), kThreads, 0, c->stream>>>(n, perm, lc, sl, st);
}

void launch_upstream_parent(Ctx *c, const Tree *t, int64_t n_pairs, int64_t n, const double *xyz, const double *nhi,
                            const uint2 *sl, const uint64_t *keys, const unsigned *owner, const unsigned *nb_off,
                            const void *rec, const unsigned *bits, unsigned W, double sigma, void *links,
                            unsigned *roots, unsigned *n_roots)
{
    if (n_pairs <= 0) return;
    if (bits)
        upstream_parent<true><<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(
            n_pairs, n, xyz, nhi, sl, keys, owner, nb_off, (const NbRec *)rec, t->mom, t->src, t->first, t->n_nodes,
            bits, W, sigma, t->box.length_unit_cm, (Link *)links, roots, n_roots);
    else
        upstream_parent<false><<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(
            n_pairs, n, xyz, nhi, sl, keys, owner, nb_off, (const NbRec *)rec, t->mom, t->src, t->first, t->n_nodes,
            nullptr, 0u, sigma, t->box.length_unit_cm, (Link *)links, roots, n_roots);
}

void launch_member_bits(Ctx *c, const Tree *t, int64_t n, int64_t n_pairs, const uint64_t *keys, const uint2 *sl,
                        const unsigned *owner, unsigned W, unsigned *bits)
{
    if (n <= 0 || W == 0) return;
    if (W <= kRowWordsLds) {
        member_rows<<<blocks_for(n * 64), kThreads, (kThreads / 64) * W * sizeof(unsigned), c->stream>>>(
            n, keys, sl, t->first, t->n_nodes, W, bits);
    } else {
        hipMemsetAsync(bits, 0, (size_t)n * W * sizeof(unsigned), c->stream);
        if (n_pairs > 0)
            member_bits<<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(n_pairs, keys, owner, t->first, t->n_nodes,
                                                                          W, bits);
    }
}

size_t upstream_link_bytes() { return sizeof(Link); }

void launch_jump_links(Ctx *c, int64_t n_pairs, const void *in, void *out, unsigned *more)
{
    if (n_pairs > 0)
        jump_links<<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(n_pairs, (const Link *)in, (Link *)out, more);
}

void launch_upstream_gamma(Ctx *c, const Tree *t, int64_t n, const double *xyz, const uint2 *sl,
                           const uint64_t *keys, const void *links, double sigma, double *gamma)
{
    if (n > 0)
        upstream_gamma<<<blocks_for(n * 64), kThreads, 0, c->stream>>>(n, xyz, sl, keys, (const Link *)links, t->mom, t->src,
                                                                       t->first, sigma, t->box.length_unit_cm, gamma);
}

void launch_parent_particle(Ctx *c, int64_t n_pairs, const void *links, const unsigned *owner, const uint2 *sl,
                            const int64_t *ooff, int64_t *out)
{
    if (n_pairs > 0)
        parent_particle<<<blocks_for(n_pairs), kThreads, 0, c->stream>>>(n_pairs, (const Link *)links, owner, sl,
                                                                          ooff, out);
}

}  // namespace start
