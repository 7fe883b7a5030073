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
// the FP64 opening test (exact lists) and the FP64 ray geometry, reads the
// FP32 copy of the grid (half the bytes), accumulates each column in FP64
// (one FMA per cell, no dearer than a compensated FP32 sum) and sums the
// terms of Gamma with Kahan compensation in FP32.
#include "internal.h"

#include <cstring>
#include <type_traits>

namespace start {

namespace {

constexpr int kWave = 64;
constexpr int kThreads = 256;
constexpr int kWavesPerBlock = kThreads / kWave;

enum Mode { kRates = 0, kCount = 1, kList = 2, kStats = 3, kKeys = 4 };

// One rate problem: a tree, a grid and a run of targets (the item's segment
// of the batch's sorted target arrays).  Read by the kernels from a device
// table, one entry per item of a batch.
struct Item {
    // tree
    int64_t n_nodes;
    int64_t n_src;
    const int4 *geo;
    const double4 *bnd;
    const int *skip;
    const int *first;
    const int *count;
    const int *ref;
    const double4 *mom;
    const uint4 *momq;
    const double *lscale;   // luminosity unit of the FP32 copies (one value)
    const double4 *src;
    const uint4 *srcq;
    const unsigned *perm;
    // grid
    const double *grid;
    const float *gridf;
    int G;
    int grid_log2;
    int sx, sy;         // element strides of the grid copies (padded rows and planes)
    int64_t guard;      // zeroed elements before cell 0 (and after the last cell)
    double frac_scale;  // 2^-(32 - grid_log2)
    double gs;          // G / size
    double lo[3];
    double size;
    double inv_size;
    double unit_cm;
    double cell_cm;     // size / G * unit_cm
    double theta2;
    double sigma;
    // channel 0: photoionisation, term L exp(-sigma N) / d^2 (eq. A2);
    // channel 1: H2 photodissociation, term L f_sh(N / 1e14) / d^2 (eq. B1)
    int channel;
    double col_scale;   // column in cells x density -> sigma N (0) or N / 1e14 (1)
    double rate_scale;  // sigma / (4 pi) (0) or 1.13e8 / (4 pi) (1)
    // targets: caller's positions, and this item's run of the sorted arrays
    int64_t n_t;
    const double *tgt_xyz;   // [3][n_t], caller order
    const double4 *tgt;      // sorted target positions
    const unsigned *tgt_orig;// caller index of each sorted target
    const int64_t *self_src; // caller order, may be null
    // outputs (caller order)
    void *gamma;
    int64_t *counts;         // list count mode: entries per target
    const int64_t *offsets;  // list mode
    int64_t *entries;        // list mode
    int64_t *stats;          // counter mode: [n_t][4]
};

// A launch covers the tiles (runs of <= 64 targets of one item) of a batch,
// one wave per tile; the item table and the tiles are kernel arguments of
// their own (const, restrict) so their fields are read with scalar loads.

// Eq. (12): l^2 <= theta^2 d^2 in normalised units, d the distance to the
// closest point of the cube [c 2^-n, (c+1) 2^-n].  Written as the same FP64
// operations as the oracle (explicit fma, no contraction) so that the lists
// agree bit for bit.  b = (lo x, lo y, lo z, side): the cube's corner c 2^-n
// and side 2^-n stored at the tree build (exact, c < 2^21), and lo + side =
// (c + 1) 2^-n is exact too.
__device__ inline bool accept_box(const double4 b, const double u[3], double theta2)
{
    const double lo[3] = {b.x, b.y, b.z};
    double d[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double a = lo[k] - u[k];
        const double c = u[k] - (lo[k] + b.w);
        // max(0, a, c) as two v_max_f64 (the operands are finite, so the
        // value is the same as with compares and selects)
        d[k] = fmax(fmax(a, c), 0.0);
    }
    const double d2 = fma(d[2], d[2], fma(d[1], d[1], d[0] * d[0]));
    return b.w * b.w <= theta2 * d2;
}

__device__ inline int clampi(int v, int G) { return v < 0 ? 0 : (v >= G ? G - 1 : v); }

// Tree records at a wave-uniform index, read through the scalar cache (the
// walk's node pointer is the same in every lane, and the tree is read-only
// while a kernel runs): a generic load would take a vector load per lane
// and wait on the LDS counter as well.
using CI = const __attribute__((address_space(4))) int;
using CU = const __attribute__((address_space(4))) unsigned;
using CD = const __attribute__((address_space(4))) double;
__device__ inline int4 uni_int4(const int4 *a, int i)
{
    CI *p = (CI *)a + 4 * (int64_t)i;
    return make_int4(p[0], p[1], p[2], p[3]);
}
__device__ inline int uni_int(const int *a, int64_t i) { return ((CI *)a)[i]; }
__device__ inline unsigned uni_u32(const unsigned *a, int64_t i) { return ((CU *)a)[i]; }
__device__ inline double4 uni_d4(const double4 *a, int i)
{
    CD *p = (CD *)a + 4 * (int64_t)i;
    return make_double4(p[0], p[1], p[2], p[3]);
}
// the luminosity (.w) of a double4 or uint4 record
__device__ inline double uni_w(const double4 *a, int64_t i) { return ((CD *)a)[4 * i + 3]; }
__device__ inline unsigned uni_w(const uint4 *a, int64_t i) { return ((CU *)a)[4 * i + 3]; }

// Orders LDS traffic between the lanes of one wavefront (no block barrier:
// the waves of a block are independent).
__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline int lanes_below(uint64_t m)
{
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// ---------------------------------------------------------------------------
// Ray march through the piecewise-constant grid from its start (t = 0) to
// its end (t = 1); the start is given as its cell (linear index) and its
// fraction fb inside the cell.  The rate kernels start every ray at its
// (virtual) source: the items of one node then leave from one point and fan
// out towards their targets, so the lanes of a gather stay in the same or
// neighbouring cache lines for longer than when each ray starts at its own
// target (~20% fewer L1 accesses per gather on the diffuse benchmark's
// batches).  The geometry (direction D, plane parameters)
// is FP64 in both precisions: an FP32 ray parameter resolves a crossing only
// to ~6e-8 of the ray length (1e-5 cell over 128 cells), which times the
// optical depth of a dense cell (~200 per cell for the 200x clumps) is above
// the 2e-4 target.  TV is the type of the grid values (FP32 or
// FP64); the sum is FP64 in both cases.  Returns sum n_c dt.
//
// The step has no branch: the next crossing is the minimum m of the three
// plane parameters, the first axis whose parameter equals m moves to its next
// plane, and the cell offset moves by that axis's stride (where the ray
// passes exactly through an edge or a corner, the other axes at m follow in
// the next steps with chords of length 0, which add exactly nothing).  The
// cell sequence depends on the geometry only, so the loads run ahead of the
// sum: three cells ahead in the rate kernels, four for FP64 cells (gathers
// in flight per lane hide most of the L1 / L2 latency: three are 7% faster
// in FP32 and 16% in FP64 than one), one ahead in the counter pass, which
// has no registers to spare.
// Cells are addressed by a 32-bit byte offset from the grid base, which the
// hardware adds to the base in the load itself (below 2^32 for FP32 cells at
// G <= 1024 and for FP64 cells at G <= 512, the grids with guard bands;
// FP64 cells of the largest grid take an element index).  The hot loop is
// L1- and VALU-bound: one gather and 14 VALU instructions per step and lane
// in FP32C, 13 in FP64.
//
// The loop ends: each step moves an axis whose parameter equals m, by a_k >=
// 1 / (2 G) (|D| is below 2G for points in the box; the step is exact since
// a_k is far above the spacing of doubles below 1), so after at most
// 3 (2G + 2) steps every parameter is >= 1.  Positions reaching the kernel
// are finite and inside the box (checked on entry), so the parameters are
// finite.  Were m NaN, it would not equal any parameter and z would step
// while t = min(m, 1) is 1 (v_min_f64 returns the non-NaN operand): the
// rate march ends with its turn (three or four steps on) and the counter
// pass at once.  No extra step counter is kept: one costs 4-8% here, as it changes
// how the loop is scheduled.
// ---------------------------------------------------------------------------
// 1 / d for d > 0 to full FP64 precision: hardware reciprocal and two Newton
// steps (the inputs are finite, normal magnitudes: ray components in cells).
__device__ inline double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

// min of two FP64 values in one instruction (fmin() would first quiet
// signalling NaNs of both operands; the plane parameters are never NaN
// signalling, and a quiet NaN loses the comparison either way)
__device__ inline double vmin(double x, double y)
{
    double r;
    asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
    return r;
}

__device__ inline double min3(double x, double y, double z) { return vmin(vmin(x, y), z); }

// H2 self-shielding function of Appendix B: 1 up to x = 1, x^(-3/4) above,
// as (1 / x^(1/4))^3 with two square roots (a few ulp; far lighter than pow)
__device__ inline float fsh(float x)
{
    const float r = 1.0f / sqrtf(sqrtf(x));
    return x <= 1.0f ? 1.0f : r * r * r;
}
__device__ inline double fsh(double x)
{
    const double r = 1.0 / sqrt(sqrt(x));
    return x <= 1.0 ? 1.0 : r * r * r;
}

typedef const __attribute__((address_space(1))) char gchar_t;

// cell value at an offset from the grid base: in bytes (S = 1 byte per unit),
// which the hardware adds to the SGPR base in the load itself, or as an
// element index (S = the cell size, one address computation per load)
template <unsigned S, typename TV>
__device__ inline TV load_cell(const TV *grid, unsigned off)
{
    if constexpr (S == 1)
        return *(const __attribute__((address_space(1))) TV *)((gchar_t *)grid + off);
    else
        return *((const __attribute__((address_space(1))) TV *)grid + off);
}

// One step of the march: the first axis (x, then y, then z) whose plane
// parameter equals the minimum m moves to its next plane, and the cell offset
// by that axis's stride.  Where the ray passes exactly through an edge or a
// corner the other axes at m follow in the next steps, each with a chord of
// length 0 (which adds exactly nothing).  The three moves run under lane
// masks (exec set from the two comparisons), so each is one add per axis
// instead of a select and an add for every axis: 8 vector instructions per
// step for the comparisons and moves against 14.  The masks come from the
// active lanes only and exec is restored at the end of the block.
__device__ inline void step_axis(double tn[3], const double a[3], const int ds[3], double m, unsigned &off)
{
    const uint64_t m0 = __builtin_amdgcn_ballot_w64(tn[0] == m);
    const uint64_t m1 = __builtin_amdgcn_ballot_w64(tn[1] == m);
    uint64_t sv, tmp;
    asm volatile(
        "s_and_saveexec_b64 %[sv], %[m0]\n\t"
        "v_add_f64 %[t0], %[t0], %[a0]\n\t"
        "v_add_u32 %[off], %[off], %[d0]\n\t"
        "s_andn2_b64 exec, %[m1], %[m0]\n\t"
        "v_add_f64 %[t1], %[t1], %[a1]\n\t"
        "v_add_u32 %[off], %[off], %[d1]\n\t"
        "s_or_b64 %[tmp], %[m0], %[m1]\n\t"
        "s_andn2_b64 exec, %[sv], %[tmp]\n\t"
        "v_add_f64 %[t2], %[t2], %[a2]\n\t"
        "v_add_u32 %[off], %[off], %[d2]\n\t"
        "s_mov_b64 exec, %[sv]"
        : [t0] "+v"(tn[0]), [t1] "+v"(tn[1]), [t2] "+v"(tn[2]), [off] "+v"(off), [sv] "=&s"(sv), [tmp] "=&s"(tmp)
        : [m0] "s"(m0), [m1] "s"(m1), [a0] "v"(a[0]), [a1] "v"(a[1]), [a2] "v"(a[2]), [d0] "v"(ds[0]),
          [d1] "v"(ds[1]), [d2] "v"(ds[2]));
}

template <typename TV, bool STATS, bool CLAMP>
__device__ inline TV march(const TV *__restrict__ grid, int sx, int sy, unsigned last, unsigned idx0,
                           const double fb[3], const double D[3], int &ncell)
{
    // Axis k crosses its next plane at tn_k and every 1/|D_k| after it.  In
    // FP64 stepping tn_k by a_k drifts by ~1 ulp per step: over the <= 3G
    // steps of a ray that is ~1e-11 cell, far inside every tolerance.
    // offset units per cell: bytes, except for FP64 cells on a grid without
    // guard bands (G = 1024), whose bytes can pass 2^32
    constexpr unsigned kScale = sizeof(TV) == 8 && CLAMP ? 1u : (unsigned)sizeof(TV);
    constexpr unsigned kUnit = kScale == 1 ? (unsigned)sizeof(TV) : 1u;   // bytes per offset unit
    const int stride[3] = {sx, sy, 1};
    double a[3], tn[3];
    int ds[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (D[k] > 0.0) {
            a[k] = recip(D[k]);
            tn[k] = (1.0 - fb[k]) * a[k];
            ds[k] = stride[k];
        } else if (D[k] < 0.0) {
            a[k] = recip(-D[k]);
            tn[k] = fb[k] * a[k];
            ds[k] = -stride[k];
        } else {
            a[k] = 0.0;
            tn[k] = 2.0;   // never crossed
            ds[k] = 0;
        }
        // a step of 2 carries a parameter past the end (t = 1) whatever it
        // was, so longer steps are cut to 2: every step is then finite
        a[k] = a[k] < 2.0 ? a[k] : 2.0;
        ds[k] *= (int)kScale;
    }
    unsigned off = idx0 * kScale;
    const unsigned off_max = last * kScale;
    double t = 0.0, sum = 0.0;
    auto add = [&](TV v, double len) {
        sum = fma((double)v, len, sum);
        if (STATS) ncell += len > 0.0 ? 1 : 0;
    };
    double m = min3(tn[0], tn[1], tn[2]);
    // leave the current cell (t = m) for the next one and load its value
    auto advance = [&](TV &vnext) {
        t = m;
        step_axis(tn, a, ds, m, off);
        if (CLAMP) off = off > off_max ? off_max : off;   // also catches a step below 0
        vnext = load_cell<kUnit>(grid, off);
        m = min3(tn[0], tn[1], tn[2]);
    };
    if constexpr (!STATS) {
        // Registers take the cells in turn (three for FP32 cells, four for
        // FP64, whose longer gathers gain 2% from the fourth; a fourth for
        // FP32 gains nothing and costs the eighth wave per SIMD); a cell's
        // value is added when the march leaves the cell two (three) places
        // after it, so three (four) loads are in flight.  The march runs in
        // whole turns of three (four) steps with the crossing parameter
        // clamped to 1: once a lane has reached its end its further steps
        // have length 0 and add nothing, so a turn has no exits inside it,
        // and every turn (the first too: the pending registers start as
        // loads of the first cell, added with length 0) enters with the same
        // loads in flight, so no wait for all of them.  Each step is kept in
        // place by a scheduling barrier so that its load is issued within it.
        constexpr bool kFour = sizeof(TV) == 8;
        TV vB = load_cell<kUnit>(grid, off);
        TV vC = load_cell<kUnit>(grid, off);
        TV vD = kFour ? load_cell<kUnit>(grid, off) : TV(0);
        TV vA = load_cell<kUnit>(grid, off);
        double lA = 0.0, lB = 0.0, lC = 0.0, lD = 0.0;
        auto leave = [&](double &len, TV &vnext) {
            const double mc = vmin(m, 1.0);   // a NaN m gives 1: the lane ends
            len = mc - t;
            t = mc;
            step_axis(tn, a, ds, m, off);
            if (CLAMP) off = off > off_max ? off_max : off;   // also catches a step below 0
            vnext = load_cell<kUnit>(grid, off);
            m = min3(tn[0], tn[1], tn[2]);
        };
        for (;;) {
            add(vB, lB);
            leave(lA, vB);
            __builtin_amdgcn_sched_barrier(0);
            add(vC, lC);
            leave(lB, vC);
            __builtin_amdgcn_sched_barrier(0);
            if constexpr (kFour) {
                add(vD, lD);
                leave(lC, vD);
                __builtin_amdgcn_sched_barrier(0);
                add(vA, lA);
                leave(lD, vA);
            } else {
                add(vA, lA);
                leave(lC, vA);
            }
            __builtin_amdgcn_sched_barrier(0);
            if (!(t < 1.0)) break;
        }
        add(vB, lB);
        add(vC, lC);
        if constexpr (kFour) add(vD, lD);
        return (TV)sum;
    } else {
        // the counter pass: one load ahead
        TV v = load_cell<kUnit>(grid, off);
        // two steps per turn (no register copies between them)
        for (;;) {
            if (!(m < 1.0)) break;
            add(v, m - t);
            advance(v);
            if (!(m < 1.0)) break;
            add(v, m - t);
            advance(v);
        }
        add(v, 1.0 - t);
        return sum;
    }
}

// ---------------------------------------------------------------------------
// Walk used by the list export (entries only, no march).
// ---------------------------------------------------------------------------
template <int MODE>
__global__ void __launch_bounds__(kThreads) list_kernel(const Item *__restrict__ items, const int4 *__restrict__ tiles,
                                                        int n_tiles)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int ti = __builtin_amdgcn_readfirstlane((int)blockIdx.x * kWavesPerBlock + (int)(threadIdx.x >> 6));
    if (ti >= n_tiles) return;
    const int4 tile = tiles[ti];
    const Item &P = items[__builtin_amdgcn_readfirstlane(tile.x)];
    const int64_t it = (int64_t)tile.y + lane;
    const bool valid = lane < tile.z;
    double u[3] = {0.0, 0.0, 0.0};
    unsigned orig = 0;
    int64_t self = -1;
    if (valid) {
        const double4 p = P.tgt[it];
        const double x[3] = {p.x, p.y, p.z};
        orig = P.tgt_orig[it];
        if (P.self_src) self = P.self_src[orig];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double v = (x[k] - P.lo[k]) * P.inv_size;
            u[k] = v > 1.0 ? 1.0 : (v < 0.0 ? 0.0 : v);
        }
    }
    int64_t n_entries = 0;
    const int64_t out_base = ((MODE == kList || MODE == kKeys) && valid) ? P.offsets[orig] : 0;
    // kList writes the export code (node index, or -(source index)-1);
    // kKeys writes node << 32 | (bucket member + 1, or 0), which increases
    // along the walk, so each target's keys come out sorted
    auto emit = [&](int64_t code, uint64_t key, double L) {
        if (!(L > 0.0)) return;
        if (MODE == kList) P.entries[out_base + n_entries] = code;
        if (MODE == kKeys) P.entries[out_base + n_entries] = (int64_t)key;
        ++n_entries;
    };
    const int4 *const t_geo = P.geo;
    const double4 *const t_bnd = P.bnd;
    const int *const t_skip = P.skip;
    const int *const t_ref = P.ref;
    const int *const t_first = P.first;
    const int *const t_count = P.count;
    const unsigned *const t_perm = P.perm;
    const double4 *const t_mom = P.mom;
    const double4 *const t_src = P.src;
    const double theta2 = P.theta2;
    int resume = 0, node = 0;
    const int n_nodes = (int)P.n_nodes;
    while (node < n_nodes) {
        node = __builtin_amdgcn_readfirstlane(node);
        const int4 g = uni_int4(t_geo, node);
        const int sk = uni_int(t_skip, node);
        const double lw = uni_w(t_mom, node);
        const int ref = uni_int(t_ref, node);
        const int kind = g.w >> 8;
        const bool active = valid && node >= resume;
        if (kind == kKindLeaf) {
            if (active && (int64_t)ref != self) emit(-(int64_t)ref - 1, (uint64_t)node << 32, lw);
            node += 1;
            continue;
        }
        const bool acc = active && accept_box(uni_d4(t_bnd, node), u, theta2);
        if (acc) {
            emit(node, (uint64_t)node << 32, lw);
            resume = sk;
        }
        const bool open = active && !acc;
        if (kind == kKindBucket) {
            if (__any(open)) {
                const int f = uni_int(t_first, node), cnt = uni_int(t_count, node);
                for (int q = f; q < f + cnt; ++q) {
                    const unsigned pq = uni_u32(t_perm, q);
                    const double lq = uni_w(t_src, q);
                    if (open && (int64_t)pq != self)
                        emit(-(int64_t)pq - 1, (uint64_t)node << 32 | (uint64_t)(q - f + 1), lq);
                }
            }
            node += 1;
            continue;
        }
        node = __any(open) ? node + 1 : sk;
    }
    if (valid) {
        if (MODE == kCount) P.counts[orig] = n_entries;
    }
}

// ---------------------------------------------------------------------------
// Rate kernel.  The wave walks as above, but an entry taken by a lane is not
// marched at once: (entry, lane) items go to a per-wave ring in LDS in node
// order, and as soon as 64 items are pending every lane marches one of them
// -- whichever target it belongs to.  Items of one node share the source and
// sit side by side, so a batch is 1-3 bundles of nearly parallel rays that
// read the same grid lines (sorting a window by ray length instead balanced
// the lanes better but lost this locality and ran 40% slower).  Each node's
// items are recorded as (first slot, lane mask); after a batch every lane
// picks its own terms out of the ring through these records, in node order,
// and adds them to its Kahan (FP32) or plain (FP64) sum.  Results are
// deterministic and every target sums its terms in depth-first order.
// ---------------------------------------------------------------------------
constexpr int kRing = 128;   // items; a node adds <= 64 and a batch drains 64

// 32-bit fixed point of the box: floor(u 2^32) of the normalised coordinate
// u in [0, 1] (1 itself to 2^32 - 1).  The FP32 path encodes the virtual
// sources and the targets alike, so a target at a source's position is at
// distance 0 exactly (both skipped as in the FP64 path); positions closer
// than 2^-32 of the box count as the same.  The top g bits of a coordinate
// are its cell on a 2^g grid, the rest the fraction inside it (exact in FP64).
__device__ inline unsigned fixed32(double x, double lo, double inv)
{
    double u = (x - lo) * inv;
    u = u < 0.0 ? 0.0 : (u > 1.0 ? 1.0 : u);
    const double q = floor(u * 4294967296.0);
    return q >= 4294967295.0 ? 0xFFFFFFFFu : (unsigned)q;
}

// A node's record in the ring: the first slot (absolute) of its items and
// the lanes that took it, side by side so that one LDS read fetches both.
struct __align__(16) NodeRec {
    int start;
    int pad;
    uint64_t mask;
};

// TF: the target's position in cells (FP64) for the FP64 path; for the FP32
// path its 32-bit box fixed-point coordinates (fixed32), kept in the items.
template <typename T, typename TF>
struct WaveLds {
    static constexpr bool kFp64 = sizeof(TF) == 8;
    NodeRec rec[kRing];           // per node: first slot, lanes that took it
    // FP32 path: the item whole (code, then the target's fixed32
    // coordinates), so that a march reads it in one access
    uint4 qitem[kFp64 ? 1 : kRing];
    // FP64 path: the item as code and target lane
    int code[kFp64 ? kRing : 1];  // node index, or -(sorted source index)-1
    T term[kRing];
    TF tpos[kFp64 ? kWave : 1][3];    // FP64 path: target position in cells
    unsigned char lane[kFp64 ? kRing : 1];   // FP64 path: target lane of the item
};


template <int PREC, bool STATS, bool CLAMP, typename T, typename TF>
__device__ __forceinline__ void rates_tile(const Item &P, const int4 tile, WaveLds<T, TF> &L, int *lds_ncell);

template <int PREC, bool STATS, bool CLAMP>
__global__ void __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(PREC == START_FP64 ? 5 : 7))) rates_kernel(const Item *__restrict__ items,
                                                         const int4 *__restrict__ tiles, int n_tiles)
{
    using T = typename std::conditional<PREC == START_FP64, double, float>::type;
    using TF = typename std::conditional<PREC == START_FP64, double, unsigned>::type;
    __shared__ WaveLds<T, TF> lds_all[kWavesPerBlock];
    __shared__ int ncell_all[STATS ? kWavesPerBlock : 1][STATS ? kRing : 1];   // counter mode only
    const int wv = threadIdx.x >> 6;
    // blocks are dealt round-robin to the 8 XCDs: give each XCD a contiguous
    // run of tiles (Morton-adjacent targets share nodes and grid lines in its L2)
    const int nb = (int)gridDim.x;
    const int per_xcd = nb / 8;
    int blk = (int)blockIdx.x;
    if (per_xcd > 0 && blk < per_xcd * 8) blk = (blk & 7) * per_xcd + (blk >> 3);
    // wave-uniform: tile record and item table are read with scalar loads
    const int ti = __builtin_amdgcn_readfirstlane(blk * kWavesPerBlock + wv);
    if (ti >= n_tiles) return;
    const int4 tile = tiles[ti];
    const int item = __builtin_amdgcn_readfirstlane(tile.x);
    rates_tile<PREC, STATS, CLAMP, T, TF>(items[item], tile, lds_all[wv], ncell_all[STATS ? wv : 0]);
}

template <int PREC, bool STATS, bool CLAMP, typename T, typename TF>
__device__ __forceinline__ void rates_tile(const Item &P, const int4 tile, WaveLds<T, TF> &L, int *lds_ncell)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t it = (int64_t)tile.y + lane;
    const bool valid = lane < tile.z;
    wave_sync();   // the previous tile's LDS reads are done

    const int G = P.G;
    const int gl = P.grid_log2;
    // the march addresses the grid from the start of its guard band, which
    // takes the steps past a ray's end (CLAMP: G = 1024, no band, offsets
    // clamped to the last cell's element)
    const int64_t guard = P.guard;
    const int last = (G - 1) * (P.sx + P.sy + 1);
    double u[3] = {0.0, 0.0, 0.0};
    unsigned orig = 0;
    int self = -1;   // source indices fit in 31 bits (n_s <= 2^30)
    unsigned tq[3] = {0u, 0u, 0u};   // FP32 path: this lane's target as fixed32 box coordinates
    {
        double B[3] = {0.0, 0.0, 0.0};
        if (valid) {
            const double4 p = P.tgt[it];
            const double x[3] = {p.x, p.y, p.z};
            orig = P.tgt_orig[it];
            if (P.self_src) self = (int)P.self_src[orig];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const double v = (x[k] - P.lo[k]) * P.inv_size;
                u[k] = v > 1.0 ? 1.0 : (v < 0.0 ? 0.0 : v);
                // the position in cells: its floor (the last cell for a target
                // on the top face) plus the fraction, both exact, sum to it
                B[k] = (x[k] - P.lo[k]) * P.gs;
            }
        }
        if constexpr (PREC == START_FP64) {
            L.tpos[lane][0] = B[0];
            L.tpos[lane][1] = B[1];
            L.tpos[lane][2] = B[2];
        } else {
            const double4 p = valid ? P.tgt[it] : make_double4(P.lo[0], P.lo[1], P.lo[2], 0.0);
            tq[0] = fixed32(p.x, P.lo[0], P.inv_size);
            tq[1] = fixed32(p.y, P.lo[1], P.inv_size);
            tq[2] = fixed32(p.z, P.lo[2], P.inv_size);
        }
    }

    T acc = T(0), accc = T(0);
    int64_t st_test = 0, st_entries = 0, st_cells = 0, st_zero = 0;
    int head = 0, tail = 0, rhead = 0, rtail = 0;   // wave-uniform ring counters
    const T col_scale = (T)P.col_scale;
    const int sh = 32 - gl;

    // the node and source arrays of the item, read once per tile (the item
    // is the same for the whole wave): each march then selects its record's
    // address between two registers instead of loading the array pointer,
    // and reads it as global memory (a generic load would also wait on LDS)
    using GD = const __attribute__((address_space(1))) double;
    using GU = const __attribute__((address_space(1))) unsigned;
    GD *const mom = (GD *)P.mom;
    GD *const src = (GD *)P.src;
    GU *const momq = (GU *)P.momq;
    GU *const srcq = (GU *)P.srcq;
    // the item's scalars, also read once per tile
    const double frac_scale = P.frac_scale, gs = P.gs;
    const double lo[3] = {P.lo[0], P.lo[1], P.lo[2]};
    const int sx = P.sx, sy = P.sy, channel = P.channel;
    const T *const grid_base = (PREC == START_FP64 ? (const T *)P.grid : (const T *)P.gridf) - guard;

    // March one item: the term L e^-tau / d^2 (d in cells) of ring slot `slot`.
    auto march_item = [&](int slot, T &term, int &nc) {
        int code, tl = 0;
        unsigned qt[3] = {0u, 0u, 0u};
        if constexpr (PREC == START_FP64) {
            code = L.code[slot];
            tl = L.lane[slot];
        } else {
            const uint4 q = L.qitem[slot];
            code = (int)q.x;
            qt[0] = q.y;
            qt[1] = q.z;
            qt[2] = q.w;
        }
        double tp[3] = {0.0, 0.0, 0.0};
        if constexpr (PREC == START_FP64) {
#pragma unroll
            for (int k = 0; k < 3; ++k) tp[k] = L.tpos[tl][k];
        }
        // the ray runs from the (virtual) source (t = 0) to the target (t = 1):
        // D = target - source, the march starts in the source's cell
        double D[3], fa[3];
        int ab[3];
        T w;
        if (PREC == START_FP64) {
            GD *const r = code >= 0 ? mom + 4 * (int64_t)code : src + 4 * (int64_t)(-code - 1);
            const double4 m = make_double4(r[0], r[1], r[2], r[3]);
            const double A[3] = {(m.x - lo[0]) * gs, (m.y - lo[1]) * gs, (m.z - lo[2]) * gs};
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                // a source on the top face sits in the last cell at fraction 1
                ab[k] = clampi((int)floor(A[k]), G);
                fa[k] = A[k] - (double)ab[k];
                D[k] = tp[k] - A[k];
            }
            w = (T)m.w;
        } else {
            // centre as 32-bit fixed point of the box: the top g bits are the
            // cell, the rest the fraction inside it (exact in FP64); D is the
            // difference of the two fixed-point coordinates in cells, exact
            // (both below 2^32, scaled by a power of two)
            GU *const r = code >= 0 ? momq + 4 * (int64_t)code : srcq + 4 * (int64_t)(-code - 1);
            const uint4 m = make_uint4(r[0], r[1], r[2], r[3]);
            const unsigned q[3] = {m.x, m.y, m.z};
            const unsigned fmask = (1u << sh) - 1u;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                ab[k] = (int)(q[k] >> sh);
                fa[k] = (double)(q[k] & fmask) * frac_scale;
                D[k] = ((double)qt[k] - (double)q[k]) * frac_scale;
            }
            w = (T)__uint_as_float(m.w);
        }
        const double d2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
        if (d2 > 0.0) {
            const unsigned e0 = (unsigned)(ab[0] * sx + ab[1] * sy + ab[2] + guard);
            const T col = march<T, STATS, CLAMP>(grid_base, sx, sy, (unsigned)(last + guard), e0, fa, D, nc);
            // FP32C: the term from the hardware square root, exp2 and
            // reciprocal (each ~1 ulp; the argument of exp2 is rounded to
            // ~6e-8 relative, i.e. 6e-8 tau of the term), FP64 as written
            const T dist = PREC == START_FP64 ? (T)sqrt(d2) : (T)__builtin_amdgcn_sqrtf((float)d2);   // grid units
            const T c = col_scale * (col * dist);
            if (channel == 0)                                  // c = tau
                term = PREC == START_FP64 ? w * exp(-c) / (T)d2
                                          : (T)(w * __builtin_amdgcn_exp2f((float)c * -1.44269504f) *
                                                __builtin_amdgcn_rcpf((float)d2));
            else
                term = w * fsh(c) / (T)d2;                     // c = N_H2 / 1e14
        } else {
            term = T(0);
            nc = -1;                                           // zero distance: skipped
        }
    };

    // March the next (up to) 64 pending items and hand the terms back.
    auto drain = [&]() {
        const int nb_items = (tail - head) < kWave ? (tail - head) : kWave;
        const int slot = (head + lane) & (kRing - 1);
        T term = T(0);
        int nc = 0;
        if (lane < nb_items) march_item(slot, term, nc);
        L.term[slot] = term;
        if (STATS) lds_ncell[slot] = nc;
        wave_sync();
        const int end = head + nb_items;
        // each record in one read (start in .x, the mask in .z, .w), the next
        // one read while this one's terms are added
        uint4 r = make_uint4(0u, 0u, 0u, 0u);
        if (rhead < rtail) r = *reinterpret_cast<const uint4 *>(&L.rec[rhead & (kRing - 1)]);
        while (rhead < rtail) {
            const int rs = __builtin_amdgcn_readfirstlane((int)r.x);
            const uint64_t m = ((uint64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)r.w) << 32) |
                               (uint64_t)(unsigned)__builtin_amdgcn_readfirstlane((int)r.z);
            if (rs >= end) break;
            if (rhead + 1 < rtail) r = *reinterpret_cast<const uint4 *>(&L.rec[(rhead + 1) & (kRing - 1)]);
            if ((m >> lane) & 1ull) {
                const int s = rs + lanes_below(m);
                if (s >= head && s < end) {
                    const T y = L.term[s & (kRing - 1)] - accc;
                    const T t2 = acc + y;
                    if (sizeof(T) == 4) accc = (t2 - acc) - y;
                    acc = t2;
                    if (STATS) {
                        const int c = lds_ncell[s & (kRing - 1)];
                        if (c < 0) st_zero++;
                        else st_cells += c;
                    }
                }
            }
            if (rs + __popcll(m) <= end) ++rhead;
            else break;
        }
        head = end;
        wave_sync();
    };

    // Queue the entry `code` for the lanes with want == true.
    auto push = [&](bool want, int code) {
        const uint64_t m = __ballot(want);
        if (m == 0) return;
        if (want) {
            const int s = (tail + lanes_below(m)) & (kRing - 1);
            if constexpr (PREC == START_FP64) {
                L.code[s] = code;
                L.lane[s] = (unsigned char)lane;
            } else {
                L.qitem[s] = make_uint4((unsigned)code, tq[0], tq[1], tq[2]);
            }
            if (STATS) st_entries++;
        }
        if (lane == 0) {
            NodeRec r;
            r.start = tail;
            r.pad = 0;
            r.mask = m;
            L.rec[rtail & (kRing - 1)] = r;
        }
        ++rtail;
        tail += __popcll(m);
        wave_sync();
        if (tail - head >= kWave) drain();
    };

    const bool fp32 = PREC == START_FP32C;
    // the tree's arrays and the opening angle, read once per tile
    const int4 *const t_geo = P.geo;
    const double4 *const t_bnd = P.bnd;
    const int *const t_skip = P.skip;
    const int *const t_ref = P.ref;
    const int *const t_first = P.first;
    const int *const t_count = P.count;
    const unsigned *const t_perm = P.perm;
    const double4 *const t_mom = P.mom;
    const double4 *const t_src = P.src;
    const uint4 *const t_momq = P.momq;
    const uint4 *const t_srcq = P.srcq;
    const double theta2 = P.theta2;
    int resume = 0, node = 0;
    const int n_nodes = (int)P.n_nodes;
    while (node < n_nodes) {
        node = __builtin_amdgcn_readfirstlane(node);
        // the node's record, subtree end, luminosity and source index are
        // read together (one wait for all four scalar loads)
        const int4 g = uni_int4(t_geo, node);
        const int sk = uni_int(t_skip, node);
        const float lw = fp32 ? __uint_as_float(uni_w(t_momq, node)) : (float)(uni_w(t_mom, node) > 0.0);
        const int rf = uni_int(t_ref, node);
        const int kind = g.w >> 8;
        const bool active = valid && node >= resume;
        if (kind == kKindLeaf) {
            push(active && rf != self && lw > 0.f, node);
            node += 1;
            continue;
        }
        bool acc_node = false;
        if (active) {
            if (STATS) st_test++;
            acc_node = accept_box(uni_d4(t_bnd, node), u, theta2);
        }
        if (acc_node) resume = sk;
        push(acc_node && lw > 0.f, node);
        const bool open = active && !acc_node;
        if (kind == kKindBucket) {
            if (__any(open)) {
                const int f = uni_int(t_first, node), cnt = uni_int(t_count, node);
                for (int q = f; q < f + cnt; ++q) {
                    const float qw = fp32 ? __uint_as_float(uni_w(t_srcq, q)) : (float)(uni_w(t_src, q) > 0.0);
                    push(open && (int)uni_u32(t_perm, q) != self && qw > 0.f, -q - 1);
                }
            }
            node += 1;
            continue;
        }
        node = __any(open) ? node + 1 : sk;
    }
    while (head < tail) drain();

    if (!valid) return;
    if (STATS) {
        int64_t *o = P.stats + (int64_t)orig * 4;
        o[0] = st_test;
        o[1] = st_entries;
        o[2] = st_cells;
        o[3] = st_zero;
        return;
    }
    if (PREC == START_FP64) {
        // terms are L / d^2 with d in cells: restore cm
        static_cast<double *>(P.gamma)[orig] = P.rate_scale * (double)acc / (P.cell_cm * P.cell_cm);
    } else {
        // L' = L / *lscale and lengths in cells: restore units in FP64
        const double Lref = P.n_nodes > 0 ? *P.lscale : 1.0;   // empty tree: no arrays
        const double sum = (double)acc - (double)accc;
        static_cast<float *>(P.gamma)[orig] = (float)(P.rate_scale * sum * Lref / (P.cell_cm * P.cell_cm));
    }
}

// Batched target preparation: every target of every item gets the key
// (item << 30 | 30-bit Morton key of its 1024^3 cell), so one radix sort
// groups the targets by item and orders each item's targets along the Morton
// curve (the order only affects speed: no target's result depends on its
// neighbours).  Positions and self indices are validated on the way.
__device__ inline unsigned spread10(unsigned v)
{
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__device__ inline int item_of(int64_t g, int n_items, const int64_t *offsets)
{
    int lo = 0, hi = n_items - 1;   // last item with offsets[item] <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

__global__ void __launch_bounds__(kThreads) batch_keys(int64_t n, int n_items, const int64_t *offsets,
                                                       const Item *__restrict__ items, uint64_t *keys,
                                                       unsigned *vals, unsigned *flags)
{
    const int64_t g = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (g >= n) return;
    const int item = item_of(g, n_items, offsets);
    const Item &I = items[item];
    const int64_t j = g - offsets[item];
    unsigned bad = 0, code = 0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double x = I.tgt_xyz[(int64_t)k * I.n_t + j];
        double u = 0.0;
        if (!isfinite(x)) {
            bad |= kFlagNonFinite;
        } else if (x < I.lo[k] || x > I.lo[k] + I.size) {
            bad |= kFlagOutOfBox;
        } else {
            u = (x - I.lo[k]) * I.inv_size;
            u = u > 1.0 ? 1.0 : u;
        }
        unsigned q = (unsigned)(u * 1024.0);
        q = q > 1023u ? 1023u : q;
        code |= spread10(q) << (2 - k);
    }
    if (I.self_src) {
        const int64_t sv = I.self_src[j];
        if (sv < -1 || sv >= I.n_src) bad |= kFlagBadSelf;
    }
    if (bad) atomicOr(flags, bad);
    keys[g] = ((uint64_t)item << 30) | code;
    vals[g] = (unsigned)g;
}

__global__ void __launch_bounds__(kThreads) batch_gather(int64_t n, const int64_t *offsets,
                                                         const Item *__restrict__ items, const uint64_t *keys,
                                                         const unsigned *vals, double4 *tgt, unsigned *tgt_orig)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const int item = (int)(keys[k] >> 30);
    const Item &I = items[item];
    const int64_t j = (int64_t)vals[k] - offsets[item];
    tgt[k] = make_double4(I.tgt_xyz[j], I.tgt_xyz[I.n_t + j], I.tgt_xyz[2 * I.n_t + j], 0.0);
    tgt_orig[k] = (unsigned)j;
}


// FP32-path copies of the virtual sources (fixed32 above, with the targets'
// encoding): the centre as 32-bit fixed-point coordinates of the box and the
// luminosity relative to the root's (every L' <= 1).
__global__ void __launch_bounds__(kThreads) make_fp32_nodes(int64_t m, const double4 *mom, const double *lscale,
                                                            start_box box, double inv, uint4 *momq)
{
    const int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (p >= m) return;
    const double Lref = *lscale;
    const double4 v = mom[p];
    momq[p] = make_uint4(fixed32(v.x, box.lo[0], inv), fixed32(v.y, box.lo[1], inv), fixed32(v.z, box.lo[2], inv),
                         __float_as_uint((float)(v.w / Lref)));
}

__global__ void __launch_bounds__(kThreads) make_fp32_src(int64_t n, const double4 *src, const double *lscale,
                                                          start_box box, double inv, uint4 *srcq)
{
    const int64_t j = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    const double Lref = *lscale;
    const double4 v = src[j];
    srcq[j] = make_uint4(fixed32(v.x, box.lo[0], inv), fixed32(v.y, box.lo[1], inv), fixed32(v.z, box.lo[2], inv),
                         __float_as_uint((float)(v.w / Lref)));
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

void make_fp32_tree(Tree *t, hipStream_t s)
{
    if (t->n_nodes == 0) return;
    const double inv = 1.0 / t->box.size;
    make_fp32_nodes<<<blocks_for(t->n_nodes), kThreads, 0, s>>>(t->n_nodes, t->mom, t->lscale, t->box, inv,
                                                                 t->momq);
    make_fp32_src<<<blocks_for(t->n_src), kThreads, 0, s>>>(t->n_src, t->src, t->lscale, t->box, inv, t->srcq);
}

// ------------------------------------------------------------------------
// Batch launcher.  All items of a call share one sort of their targets and
// one persistent launch per precision; a single start_compute_rates is a
// batch of one item.
// ------------------------------------------------------------------------
namespace {

struct BatchScratch {
    uint64_t *keys;
    unsigned *vals;
    double4 *tgt;
    unsigned *tgt_orig;
    Item *items;
    int64_t *offsets;
    int4 *tiles;
    void *radix_tmp;
};

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

size_t stage_bytes(int n_items, int64_t n_tiles)
{
    return al256((size_t)n_items * sizeof(Item)) + al256((size_t)(n_items + 1) * sizeof(int64_t)) +
           al256((size_t)n_tiles * sizeof(int4));
}

BatchScratch carve_batch(void *base, int64_t n, int n_items, int64_t n_tiles)
{
    const int64_t nk = n > 1 ? n : 1;
    char *q = (char *)base;
    BatchScratch b;
    b.items = (Item *)q;   // the staged block first: items, offsets, tiles
    q += al256((size_t)n_items * sizeof(Item));
    b.offsets = (int64_t *)q;
    q += al256((size_t)(n_items + 1) * sizeof(int64_t));
    b.tiles = (int4 *)q;
    q += al256((size_t)n_tiles * sizeof(int4));
    b.keys = (uint64_t *)q;
    q += al256((size_t)nk * sizeof(uint64_t));
    b.vals = (unsigned *)q;
    q += al256((size_t)nk * sizeof(unsigned));
    b.tgt = (double4 *)q;
    q += al256((size_t)nk * sizeof(double4));
    b.tgt_orig = (unsigned *)q;
    q += al256((size_t)nk * sizeof(unsigned));
    b.radix_tmp = q;
    return b;
}

template <int PREC, bool STATS>
void launch_tiles(const Item *items, const int4 *tiles, int64_t n_tiles, bool clamp, hipStream_t s)
{
    int64_t blocks = (n_tiles + kWavesPerBlock - 1) / kWavesPerBlock;
    if (blocks >= 64) blocks = (blocks + 7) / 8 * 8;   // whole rounds over the 8 XCDs
    if (clamp) rates_kernel<PREC, STATS, true><<<(unsigned)blocks, kThreads, 0, s>>>(items, tiles, (int)n_tiles);
    else rates_kernel<PREC, STATS, false><<<(unsigned)blocks, kThreads, 0, s>>>(items, tiles, (int)n_tiles);
}

// Whether any item's grid has no guard band (G = 1024): the launch then
// clamps every march step.
bool needs_clamp(const RateSpec *specs, int n)
{
    for (int i = 0; i < n; ++i)
        if (specs[i].grid && specs[i].grid->guard == 0) return true;
    return false;
}

}  // namespace

size_t batch_stage_bytes(int n_items, int64_t n_tiles) { return stage_bytes(n_items, n_tiles); }

size_t batch_scratch_bytes(int64_t n, int n_items, int64_t n_tiles)
{
    const int64_t nk = n > 1 ? n : 1;
    return stage_bytes(n_items, n_tiles) + al256((size_t)nk * sizeof(uint64_t)) +
           al256((size_t)nk * sizeof(unsigned)) + al256((size_t)nk * sizeof(double4)) +
           al256((size_t)nk * sizeof(unsigned)) + al256(radix_temp_bytes(nk)) + 256;
}

int64_t batch_tiles(const RateSpec *specs, int n, int tile)
{
    int64_t t = 0;
    for (int i = 0; i < n; ++i) t += (specs[i].n_t + tile - 1) / tile;
    return t;
}

namespace {

// The table entry of one rate problem; its targets are the run [off, off +
// n_t) of the batch's sorted target arrays in bs.
Item make_item(const RateSpec &r, const BatchScratch &bs, int64_t off)
{
    const Tree *t = r.tree;
    const Grid *g = r.grid;
    Item I;
    memset(&I, 0, sizeof(I));
    I.n_nodes = t->n_nodes;
    I.n_src = t->n_src;
    I.geo = t->geo;
    I.bnd = t->bnd;
    I.skip = t->skip;
    I.first = t->first;
    I.count = t->count;
    I.ref = t->ref;
    I.mom = t->mom;
    I.momq = t->momq;
    I.lscale = t->lscale;
    I.src = t->src;
    I.srcq = t->srcq;
    I.perm = t->perm;
    if (g) {
        I.grid = g->val;
        I.gridf = g->valf;
        I.G = g->G;
        I.grid_log2 = g->grid_log2;
        I.sx = g->sx;
        I.sy = g->sy;
        I.guard = g->guard;
    } else {
        I.G = 1;
        I.grid_log2 = 0;
        I.sx = I.sy = 1;
    }
    I.frac_scale = ldexp(1.0, -(32 - I.grid_log2));
    I.gs = (double)I.G / t->box.size;
    for (int k = 0; k < 3; ++k) I.lo[k] = t->box.lo[k];
    I.size = t->box.size;
    I.inv_size = 1.0 / t->box.size;
    I.unit_cm = t->box.length_unit_cm;
    I.cell_cm = t->box.size / I.G * t->box.length_unit_cm;
    I.theta2 = r.theta * r.theta;
    I.sigma = r.sigma;
    I.channel = r.channel;
    I.col_scale = r.channel == 0 ? r.sigma * I.cell_cm : I.cell_cm * 1e-14;
    I.rate_scale = (r.channel == 0 ? r.sigma : 1.13e8) / (4.0 * M_PI);
    I.n_t = r.n_t;
    I.tgt_xyz = r.tgt_xyz;
    I.tgt = bs.tgt + off;
    I.tgt_orig = bs.tgt_orig + off;
    I.self_src = r.self_src;
    I.gamma = r.gamma;
    I.counts = r.counts;
    I.offsets = r.offsets;
    I.entries = r.entries;
    I.stats = r.stats;
    return I;
}

// Device part of a batch whose tables are in place: target keys, sort and
// gather, then the kernels of the mode.
void launch_staged(const BatchScratch &bs, int64_t N, int n, int64_t n_tiles, int64_t n64, int mode, bool clamp,
                   unsigned *flags, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1, BatchLaunch *launch)
{
    if (N == 0) return;
    const unsigned nb = (unsigned)((N + kThreads - 1) / kThreads);
    batch_keys<<<nb, kThreads, 0, s>>>(N, n, bs.offsets, bs.items, bs.keys, bs.vals, flags);
    int bits = 30;
    while ((1 << (bits - 30)) < n) ++bits;
    radix_sort_pairs(bs.keys, bs.vals, N, bits, bs.radix_tmp, s);
    batch_gather<<<nb, kThreads, 0, s>>>(N, bs.offsets, bs.items, bs.keys, bs.vals, bs.tgt, bs.tgt_orig);

    if (mode == 2 || mode == 3 || mode == 4) {
        const unsigned lb = (unsigned)((n_tiles + kWavesPerBlock - 1) / kWavesPerBlock);
        if (mode == 2) list_kernel<kCount><<<lb, kThreads, 0, s>>>(bs.items, bs.tiles, (int)n_tiles);
        else if (mode == 3) list_kernel<kList><<<lb, kThreads, 0, s>>>(bs.items, bs.tiles, (int)n_tiles);
        else list_kernel<kKeys><<<lb, kThreads, 0, s>>>(bs.items, bs.tiles, (int)n_tiles);
        return;
    }
    BatchLaunch bl{bs.items, bs.tiles, n_tiles, n64, mode, clamp};
    if (launch) *launch = bl;
    if (ev0) hipEventRecord(ev0, s);
    relaunch_batch(bl, s);
    if (ev1) hipEventRecord(ev1, s);
}

static_assert(sizeof(Item) <= 1024, "the item table entry is passed as a kernel argument");

// The tables of a one-item batch written on the device from the kernel
// argument (no host staging): the item, its offsets (0, n_t) and its tiles.
__global__ void __launch_bounds__(kThreads) single_tables(Item I, int tile, int64_t n_tiles, Item *items,
                                                          int64_t *offsets, int4 *tiles)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k == 0) {
        *items = I;
        offsets[0] = 0;
        offsets[1] = I.n_t;
    }
    if (k < n_tiles) {
        const int64_t f = k * tile;
        tiles[k] = make_int4(0, (int)f, (int)(I.n_t - f < tile ? I.n_t - f : tile), 0);
    }
}

}  // namespace

// Enqueues a batch (the scratch and the pinned staging area must be large
// enough: batch_scratch_bytes / stage_bytes).  mode: 0 rates, 1 counters,
// 2 list counts, 3 lists.  ev0/ev1 (may be null) bracket the rate kernels.
void run_batch(Ctx *c, const RateSpec *specs, int n, int mode, int tile, void *scratch, hipEvent_t ev0,
               hipEvent_t ev1, BatchLaunch *launch)
{
    hipStream_t s = c->stream;
    int64_t N = 0;
    for (int i = 0; i < n; ++i) N += specs[i].n_t;
    const int64_t n_tiles = batch_tiles(specs, n, tile);
    BatchScratch bs = carve_batch(scratch, N, n, n_tiles);

    // host side: item table, offsets, tiles (FP64 items' tiles first)
    hipEventSynchronize(c->stage_ev);   // the previous upload has been read
    char *h = (char *)c->host_stage;
    Item *hi = (Item *)h;
    int64_t *ho = (int64_t *)(h + al256((size_t)n * sizeof(Item)));
    int4 *ht = (int4 *)(h + al256((size_t)n * sizeof(Item)) + al256((size_t)(n + 1) * sizeof(int64_t)));
    int64_t off = 0;
    for (int i = 0; i < n; ++i) {
        hi[i] = make_item(specs[i], bs, off);
        ho[i] = off;
        off += specs[i].n_t;
    }
    ho[n] = off;
    int64_t t64 = 0;
    for (int pass = 0; pass < 2; ++pass)   // FP64 items, then FP32C items
        for (int i = 0; i < n; ++i) {
            if ((specs[i].prec == START_FP64) != (pass == 0)) continue;
            for (int64_t f = 0; f < specs[i].n_t; f += tile)
                ht[t64++] = make_int4(i, (int)f, (int)(specs[i].n_t - f < tile ? specs[i].n_t - f : tile), 0);
        }
    int64_t n64 = 0;
    for (int i = 0; i < n; ++i)
        if (specs[i].prec == START_FP64) n64 += (specs[i].n_t + tile - 1) / tile;
    hipMemcpyAsync(bs.items, h, stage_bytes(n, n_tiles), hipMemcpyHostToDevice, s);
    hipEventRecord(c->stage_ev, s);
    launch_staged(bs, N, n, n_tiles, n64, mode, needs_clamp(specs, n), c->d_flags, s, ev0, ev1, launch);
}

void run_single_fixed(Ctx *c, const RateSpec &r, int tile, void *scratch)
{
    hipStream_t s = c->stream;
    const int64_t n_tiles = batch_tiles(&r, 1, tile);
    BatchScratch bs = carve_batch(scratch, r.n_t, 1, n_tiles);
    const Item I = make_item(r, bs, 0);
    const int64_t nb = (n_tiles + kThreads - 1) / kThreads;
    single_tables<<<(unsigned)(nb > 0 ? nb : 1), kThreads, 0, s>>>(I, tile, n_tiles, bs.items, bs.offsets, bs.tiles);
    launch_staged(bs, r.n_t, 1, n_tiles, r.prec == START_FP64 ? n_tiles : 0, 0, needs_clamp(&r, 1), c->d_flags, s,
                  nullptr, nullptr, nullptr);
}

void relaunch_batch(const BatchLaunch &b, hipStream_t s)
{
    const Item *items = static_cast<const Item *>(b.items);
    if (b.n64 > 0) {
        if (b.mode == 1) launch_tiles<START_FP64, true>(items, b.tiles, b.n64, b.clamp, s);
        else launch_tiles<START_FP64, false>(items, b.tiles, b.n64, b.clamp, s);
    }
    if (b.n_tiles - b.n64 > 0) {
        if (b.mode == 1) launch_tiles<START_FP32C, true>(items, b.tiles + b.n64, b.n_tiles - b.n64, b.clamp, s);
        else launch_tiles<START_FP32C, false>(items, b.tiles + b.n64, b.n_tiles - b.n64, b.clamp, s);
    }
}

// ---------------------------------------------------------------------------
// Upstream-particle chain: optical depth of the pairs (particle, source) that
// have no upstream particle, integrated along the ray as in the rate kernel
// (FP64).  key: node << 32 | (bucket member + 1, or 0).
// ---------------------------------------------------------------------------
namespace {

template <bool CLAMP>
__global__ void __launch_bounds__(256) upstream_roots(int64_t n_roots, const unsigned *__restrict__ roots,
                                                      const uint64_t *__restrict__ keys,
                                                      const unsigned *__restrict__ owner, const double *__restrict__ xyz,
                                                      int64_t n, const double4 *__restrict__ mom,
                                                      const double4 *__restrict__ src, const int *__restrict__ first,
                                                      const double *__restrict__ grid, int64_t guard, int G, int sx,
                                                      int sy, double lo0,
                                                      double lo1, double lo2, double gs, double tau_scale,
                                                      double *__restrict__ acc, int acc_stride)
{
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n_roots) return;
    const unsigned p = roots[r];
    const unsigned i = owner[p];
    const double4 a = source_of_key(mom, src, first, keys[p]);
    const double lo[3] = {lo0, lo1, lo2};
    const double x[3] = {xyz[i], xyz[n + i], xyz[2 * n + i]};
    const double A[3] = {(a.x - lo[0]) * gs, (a.y - lo[1]) * gs, (a.z - lo[2]) * gs};
    int tb[3];
    double fb[3], D[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double B = (x[k] - lo[k]) * gs;
        int b = (int)floor(B);
        b = b < 0 ? 0 : (b > G - 1 ? G - 1 : b);
        tb[k] = b;
        fb[k] = B - (double)b;
        D[k] = A[k] - ((double)tb[k] + fb[k]);
    }
    const double d2 = D[0] * D[0] + D[1] * D[1] + D[2] * D[2];
    if (!(d2 > 0.0)) {
        acc[(int64_t)p * acc_stride] = 0.0;
        return;
    }
    int nc = 0;
    const unsigned e0 = (unsigned)(tb[0] * sx + tb[1] * sy + tb[2] + guard);
    const double col = march<double, false, CLAMP>(grid - guard, sx, sy, (unsigned)((G - 1) * (sx + sy + 1) + guard),
                                                   e0, fb, D, nc);
    acc[(int64_t)p * acc_stride] = tau_scale * (col * sqrt(d2));
}

}  // namespace

void launch_upstream_roots(Ctx *c, const Tree *t, const Grid *g, int64_t n_roots, const unsigned *roots,
                           const uint64_t *keys, const unsigned *owner, const double *xyz, int64_t n, double sigma,
                           double *acc, int acc_stride)
{
    if (n_roots <= 0) return;
    const double gs = (double)g->G / t->box.size;
    const double tau_scale = sigma * (t->box.size / g->G * t->box.length_unit_cm);
    const unsigned nb = (unsigned)((n_roots + 255) / 256);
    if (g->guard == 0)
        upstream_roots<true><<<nb, 256, 0, c->stream>>>(n_roots, roots, keys, owner, xyz, n, t->mom, t->src, t->first,
                                                        g->val, g->guard, g->G, g->sx, g->sy, t->box.lo[0],
                                                        t->box.lo[1], t->box.lo[2], gs, tau_scale, acc, acc_stride);
    else
        upstream_roots<false><<<nb, 256, 0, c->stream>>>(n_roots, roots, keys, owner, xyz, n, t->mom, t->src,
                                                         t->first, g->val, g->guard, g->G, g->sx, g->sy, t->box.lo[0],
                                                         t->box.lo[1], t->box.lo[2], gs, tau_scale, acc, acc_stride);
}

}  // namespace start
