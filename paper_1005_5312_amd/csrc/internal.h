// Internal declarations of libstart (HIP, gfx950).  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/start.h"
#include "limits.h"

namespace start {

constexpr int kMaxLevel = 21;            // 63-bit Morton keys: 21 levels below the root
constexpr int kKindInternal = 0;         // cell that splits into >= 2 sub-cubes
constexpr int kKindBucket = 1;           // level-21 cell with >= 2 coincident sources
constexpr int kKindLeaf = 2;             // single source

// Error flags raised by validation kernels (bit set in a device word).
constexpr unsigned kFlagNonFinite = 1u;
constexpr unsigned kFlagOutOfBox = 2u;
constexpr unsigned kFlagNegative = 4u;
constexpr unsigned kFlagBadSelf = 8u;
constexpr unsigned kFlagEqInput = 16u;    // equilibrium: n_H, Gamma or x out of range

constexpr size_t kPoolMaxBytes = (size_t)8 << 30;

constexpr int kReadbackWords = 512;   // per build: flags, counts, the 256-bin reach histogram

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    size_t budget = 0;        // 0 = unlimited
    size_t in_use = 0;
    unsigned *d_flags = nullptr;   // sticky validation flags (device)
    std::string err;
    // scratch reused by compute_rates (grown on demand)
    void *scratch = nullptr;
    size_t scratch_bytes = 0;
    // pinned staging of batch tables (item descriptors, offsets, tiles) and
    // the event after its last upload
    void *host_stage = nullptr;
    size_t host_stage_bytes = 0;
    hipEvent_t stage_ev = nullptr;
    // targets per wave of the rate kernels: fixed (1..64), or 0 = from the
    // autotuned table by size class (ceil(log2) of the total targets and of
    // the largest tree's sources; 0 entries: chosen from the size)
    int tile_fixed = 0;
    int tile_by_class[40][32] = {};
    // replay repeated kernel sequences (the equilibrium iterations) from a
    // captured HIP graph
    bool graphs = true;
    // refill the equilibrium loops' grids from recorded (cell, particle) pairs
    bool grid_pairs = true;
    // freed device blocks kept for reuse (dmalloc / dfree), at most
    // kPoolMaxBytes in total; guarded by mem_mu
    std::vector<std::pair<void *, size_t>> pool;
    size_t pooled = 0;
    std::mutex mem_mu;
    // a helper context (the second build of start_build_scene) allocates
    // through its owner: one budget, one pool
    Ctx *mem_owner = nullptr;
    // pinned, device-visible words that the builds' own kernels fill with the
    // counts and flags the host reads back mid-build (one host wait, no copy
    // call): kReadbackWords per build, the owner's first, a helper's second
    unsigned *rb = nullptr;       // host address
    unsigned *rb_dev = nullptr;   // the same words as the device sees them
    // second stream and its event, for the concurrent scene builds
    hipStream_t stream2 = nullptr;
    hipEvent_t ev2 = nullptr;
    // walk-kernel timing (start_profile_enable)
    bool profile = false;
    std::vector<hipEvent_t> ev_pool;   // pairs (start, stop)
    size_t ev_used = 0;
};

// Device-resident octree in depth-first (Morton) order.  Arrays of n_nodes.
struct Tree {
    start_box box;
    int64_t n_src = 0;
    int64_t n_nodes = 0;
    int4 *geo = nullptr;       // (cx, cy, cz, level | kind << 8)
    double4 *bnd = nullptr;    // the cube in normalised units: lower corner (c 2^-level) and side 2^-level
    int *skip = nullptr;       // index of the first node after the subtree
    int *first = nullptr;      // range of the cell in sorted source order
    int *count = nullptr;
    int *ref = nullptr;        // leaf: original source index
    double4 *mom = nullptr;    // (centre of luminosity x, y, z; luminosity)
    uint4 *momq = nullptr;     // FP32 path: centre as 32-bit fixed-point box
                               // coordinates, L / *lscale as float bits
    uint64_t *keys = nullptr;  // sorted source keys
    unsigned *perm = nullptr;  // sorted position -> original source index
    double4 *src = nullptr;    // sorted sources (x, y, z, L)
    uint4 *srcq = nullptr;     // same for the sorted sources (bucket members)
    double *lscale = nullptr;  // L_root of the FP32 copies (device, one value > 0):
                               // the root's luminosity, or after kernel weighting
                               // the largest luminosity of any node or source
    size_t bytes = 0;
    Ctx *ctx = nullptr;
};

// Cell (ix, iy, iz) is element ix*sx + iy*sy + iz of both copies.  Rows and
// planes are padded by 16 elements for 64 <= G <= 512: with power-of-two
// strides the lanes of a gather that sit in neighbouring rows or planes hit
// the same L1 tag banks, and the padded grid marches ~5% faster (FP32
// offsets stay below 2^32 up to G = 512; G = 1024 is left unpadded).
//
// Each copy also has `guard` zeroed elements before its first and after its
// last cell (G <= 512): a march may step up to 4 cells per axis past its
// target before it stops (its last turn runs to the end), and those reads
// land in the guard band instead of needing a clamp on every step.  G = 1024
// has no guard (its FP32 byte offsets already use all 32 bits) and its
// marches clamp the offset.
struct Grid {
    start_box box;
    int grid_log2 = 0;
    int G = 1;
    int sx = 1, sy = 1;        // element strides of x and y
    int64_t span = 1;          // elements of the cells (padding included, zeroed)
    int64_t guard = 0;         // zeroed elements before and after the cells
    void *mem = nullptr;       // the allocation (both copies with their guards)
    double *val = nullptr;     // FP64 values (cell 0)
    float *valf = nullptr;     // FP32 copy (cell 0)
    size_t bytes = 0;
};

// Gas particles counting-sorted into the cells of a G^3 grid, kept so that
// the grid can be refilled for new n_HI values at the same positions.
// The particles are split into at most kMaxReachClasses classes by their
// kernel support 2h, so that each cell centre scans, per class, only the
// cells that class can reach; the binned order is class-major, then cell.
constexpr int kMaxReachClasses = 4;
struct ReachClasses {
    int K = 1;
    int R[kMaxReachClasses] = {};      // loop half-width in cells
    float q2[kMaxReachClasses] = {};   // (reach / delta)^2 with a small safety margin
};

struct GasBins {
    start_box box;
    int64_t n = 0;
    int G = 1;
    double reach = 0.0;        // largest kernel support 2h
    double delta = 0.0;        // cell side
    ReachClasses cls;
    char *mem = nullptr;       // particle arrays
    size_t bytes = 0;
    char *mem2 = nullptr;      // starts
    size_t bytes2 = 0;
    unsigned *idx = nullptr;   // binned order -> particle index
    unsigned *start = nullptr; // first binned particle of each (class, cell) [K G^3 + 1]
    double4 *pos_h = nullptr;  // binned (x, y, z, h)
    double2 *kern = nullptr;   // binned (1/h, 1/(pi h^3))
    double *ns = nullptr;      // binned n_HI
    // optional (record_pairs): every (cell centre, particle) pair inside the
    // support, in summation order, for refills at the same positions
    char *mem3 = nullptr, *mem4 = nullptr;
    size_t bytes3 = 0, bytes4 = 0;
    unsigned *pcount = nullptr;  // pairs of each cell [G^3] (unpadded order)
    unsigned *pstart = nullptr;  // first pair of each group of 64 cells [G^3 / 64 + 1]; a group's
                                 // pairs are interleaved: pair q of its cell l at q * 64 + l
    unsigned *pidx = nullptr;    // binned particle of each pair
    double *pw = nullptr;        // kernel weight of each pair
    double *pden = nullptr;      // weight sum of each cell
    int64_t n_pairs = 0;
};

// ---- gas grid (grid.hip) ----
start_status alloc_grid(Ctx *c, const start_box &box, int grid_log2, Grid *g);
// Validates and bins the particles (synchronises); n_HI is gathered too.
start_status bin_gas(Ctx *c, const start_box &box, int64_t n, const double *xyz, const double *h,
                     const double *nhi, int grid_log2, GasBins *b);
void free_bins(Ctx *c, GasBins *b);
// Enqueues the grid values from the binned particles; nhi (particle order,
// not validated) replaces the binned n_HI first when non-null.
void fill_grid(Ctx *c, const GasBins &b, const double *nhi, Grid *g);
// Records the pairs (and fills g from the binned n_HI) so that later
// fill_grid calls read them instead of searching the stencil; synchronises.
// START_ENOMEM leaves the bins as they were (fill_grid then gathers).
start_status record_pairs(Ctx *c, GasBins *b, Grid *g);

// ---- memory helpers (count against the context budget) ----
hipError_t dmalloc(Ctx *c, void **p, size_t bytes);
void dfree(Ctx *c, void *p, size_t bytes);
void release_pool(Ctx *c);

// ---- primitives (sort.hip) ----
// Exclusive scan of n unsigned ints in place; returns total through *d_total
// when non-null (device pointer).  temp must hold scan_temp_bytes(n).
size_t scan_temp_bytes(int64_t n);
void exclusive_scan_u32(unsigned *d_data, int64_t n, void *temp, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on the low `bits` bits of the
// keys.  Buffers are ping-ponged; the result ends in keys/vals.
size_t radix_temp_bytes(int64_t n);
void radix_sort_pairs(uint64_t *keys, unsigned *vals, int64_t n, int bits, void *temp,
                      hipStream_t s);

// ---- rate batches (rates.hip) ----
// One rate problem as given to the library.
struct RateSpec {
    const Tree *tree;
    const Grid *grid;
    int64_t n_t;
    const double *tgt_xyz;
    const int64_t *self_src;
    double theta;
    double sigma;
    int prec;
    int channel;               // 0 photoionisation (eq. A2), 1 H2 photodissociation (eq. B1)
    void *gamma;               // rates
    int64_t *stats;            // counters [n_t][4]
    int64_t *counts;           // list counts [n_t]
    const int64_t *offsets;    // list offsets [n_t + 1]
    int64_t *entries;          // list entries
};
size_t batch_scratch_bytes(int64_t n_targets, int n_items, int64_t n_tiles);
size_t batch_stage_bytes(int n_items, int64_t n_tiles);
// Tiles of at most `tile` targets (1..64) of one item, one wave each.
int64_t batch_tiles(const RateSpec *specs, int n, int tile);
// The rate kernels of a staged batch: item and tile tables and the sorted
// targets already in the scratch (rates and counter modes only).  They can
// be launched again while the scratch, the trees and the grids are
// unchanged, and contain no host work, so they can be captured in a graph.
struct BatchLaunch {
    const void *items;
    const int4 *tiles;
    int64_t n_tiles;
    int64_t n64;     // tiles of FP64 items (first)
    int mode;
    bool clamp;      // some grid has no guard band: clamp the march offsets
};
// Stages a batch (host tables, upload, target sort) and launches it; the
// launch is described in *launch when non-null.
void run_batch(Ctx *c, const RateSpec *specs, int n, int mode, int tile, void *scratch, hipEvent_t ev0,
               hipEvent_t ev1, BatchLaunch *launch = nullptr);
void relaunch_batch(const BatchLaunch &b, hipStream_t s);
// One rate problem (mode 0) on a caller-provided device scratch of at least
// batch_scratch_bytes(r.n_t, 1, batch_tiles(&r, 1, tile)) bytes: its tables
// are written by a kernel, so nothing is allocated or staged on the host.
void run_single_fixed(Ctx *c, const RateSpec &r, int tile, void *scratch);

// ---- fixed device scratch of start_compute_rates_noalloc (noalloc.hip) ----
// Looks up this device's copy of the library's static scratch array (the
// device must be current); returns false if the runtime refuses.
bool noalloc_init(int device);
// One rate call (mode 0) on that array: START_ECAPACITY (with *err) when the
// call needs more than it holds, START_EHIP when it was not looked up.
start_status noalloc_rates(Ctx *c, const RateSpec &r, int tile, const char **err);

// ---- photoionisation equilibrium (equilibrium.hip) ----
// x <- equilibrium neutral fraction for gamma (double or float by
// gamma_prec); nhi (may be null) <- x n_H; max |change| folded into
// *max_change (bits of a non-negative double; may be null).  Bad inputs set
// kFlagEqInput in the context's flags word.
void launch_eq_update(Ctx *c, int64_t n, const double *n_h, const void *gamma, int gamma_prec, double alpha,
                      double *x, double *nhi, unsigned long long *max_change);
// *w = 0 by a one-thread kernel (graph-safe, unlike a memset node).
void launch_clear_word(Ctx *c, unsigned long long *w);
void launch_iota(Ctx *c, int64_t n, int64_t *out);
// The equilibrium update with the transfer of recombination photons:
// alpha_eff = alpha_A - alpha_1 (1 - exp(-tau_self(x_old))) per particle.
void launch_eq_update_diffuse(Ctx *c, int64_t n, const double *n_h, const void *gamma, int gamma_prec,
                              const double *vol, double sigma, double alpha_a, double alpha_1, double *x, double *nhi,
                              unsigned long long *max_change);
// nhi <- x n_H after checking n_H >= 0 and x in [0, 1].
void launch_eq_prepare(Ctx *c, int64_t n, const double *n_h, const double *x, double *nhi);
// Recombination emission alpha_1 n_e n_p V and k_self per particle (either
// output may be null).
void launch_recomb_terms(Ctx *c, int64_t n, const double *n_h, const double *x, const double *vol, double sigma,
                         double alpha_1, double *lum, double *kself);
// k_ion = x n_H gamma + k_self (k_self may be null).
void launch_total_rate(Ctx *c, int64_t n, const double *n_h, const double *x, const void *gamma, int gamma_prec,
                       const double *kself, double *kion);

// ---- upstream-particle chain (upstream.hip, rates.hip) ----
// A list entry as a sortable key: node << 32 | (bucket member + 1, or 0);
// the (virtual) source it stands for: the node's centre and luminosity, or
// the bucket member's position and luminosity.
__device__ inline double4 source_of_key(const double4 *__restrict__ mom, const double4 *__restrict__ src,
                                        const int *__restrict__ first, uint64_t key)
{
    const int node = (int)(key >> 32);
    const unsigned m = (unsigned)(key & 0xffffffffu);
    return m == 0 ? mom[node] : src[first[node] + (int)m - 1];
}
// Grid values in linear order (ix*G + iy)*G + iz (the export layout).
void launch_grid_unpad(Ctx *c, const Grid &g, double *out);
// acc[p * acc_stride] = optical depth along the ray of each root pair p
// (FP64 march).
void launch_upstream_roots(Ctx *c, const Tree *t, const Grid *g, int64_t n_roots, const unsigned *roots,
                           const uint64_t *keys, const unsigned *owner, const double *xyz, int64_t n, double sigma,
                           double *acc, int acc_stride);

void launch_to_u32(Ctx *c, int64_t n, const int64_t *in, unsigned *out);
// *total += sum of n non-negative int64 values (64-bit accumulation)
void launch_sum_i64(Ctx *c, int64_t n, const int64_t *in, unsigned long long *total);
void launch_sum_u32(Ctx *c, int64_t n, const unsigned *in, unsigned long long *total);
void launch_to_i64(Ctx *c, int64_t n, const unsigned *in, int64_t *out);
// Neighbours within 2 h_i (one wave per particle, the particles taken in the
// Morton order perm): counts (nb_off null) into count[n], or, with nb_off =
// the exclusive scan of those counts (n + 1 entries), one record per
// neighbour (position and index) of neighbour_record_bytes() bytes.
size_t neighbour_record_bytes();
void launch_neighbours(Ctx *c, const GasBins &b, int64_t n, const unsigned *perm, const double *xyz, const double *h,
                       unsigned *count, const unsigned *nb_off, void *rec);
// The pairs' layout: each particle's list contiguous, the lists in the
// Morton order of their particles (perm: rank -> particle).  lc[r] = pair
// count of rank r (to be scanned); sl[i] = (first pair, count), st[i] = first
// pair of particle i.
void launch_coarse_keys(Ctx *c, int64_t n, uint64_t *keys);   // keys >>= 33 (top 30 bits)
void launch_layout_counts(Ctx *c, int64_t n, const unsigned *perm, const int64_t *counts, unsigned *lc);
void launch_layout_starts(Ctx *c, int64_t n, const unsigned *perm, const unsigned *lc, uint2 *sl, int64_t *st);
void launch_pair_owner(Ctx *c, int64_t n, const uint2 *sl, unsigned *owner);
void launch_upstream_parent(Ctx *c, const Tree *t, int64_t n_pairs, int64_t n, const double *xyz, const double *nhi,
                            const uint2 *sl, const uint64_t *keys, const unsigned *owner, const unsigned *nb_off,
                            const void *rec, const unsigned *bits, unsigned W, double sigma, void *links,
                            unsigned *roots, unsigned *n_roots);
// Membership table of the lists: row i (W 32-bit words) has bit id(alpha)
// set for every entry alpha of particle i's list, id = node, or n_nodes +
// sorted source index for a bucket member; every word of the table is written.
void launch_member_bits(Ctx *c, const Tree *t, int64_t n, int64_t n_pairs, const uint64_t *keys, const uint2 *sl,
                        const unsigned *owner, unsigned W, unsigned *bits);
// The pairs' 16-byte (tau, parent) records (upstream_link_bytes() each; tau
// at double index 2p): written by the upstream search (tau = the step to the
// parent, or left for the root march), then pointer jumping, one round from
// `in` to `out` (sets *more when a parent still has a parent).
size_t upstream_link_bytes();
void launch_jump_links(Ctx *c, int64_t n_pairs, const void *in, void *out, unsigned *more);
void launch_upstream_gamma(Ctx *c, const Tree *t, int64_t n, const double *xyz, const uint2 *sl,
                           const uint64_t *keys, const void *links, double sigma, double *gamma);
// parent pair -> upstream particle (or -1) at the pair's place in the
// particle-order export (offsets ooff), from the search's records
void launch_parent_particle(Ctx *c, int64_t n_pairs, const void *links, const unsigned *owner, const uint2 *sl,
                            const int64_t *ooff, int64_t *out);

// ---- Morton keys (tree.hip) ----
void launch_keys(const start_box &box, int64_t n, const double *xyz, const double *lum,
                 uint64_t *keys, unsigned *idx, unsigned *flags, hipStream_t s);

// ---- kernel-weighted node luminosities (tree.hip) ----
// Replaces the luminosity of every node of >= 2 sources by form 1 (kernel-
// weighted mean) or form 2 (volume-weighted SPH sum) at its centre of
// luminosity and sets t->lscale; the FP32 copies are left to the caller.
// h, vol: device arrays in caller order.  Synchronises (validation).
start_status tree_kernel_luminosity(Ctx *c, Tree *t, const double *h, const double *vol, int form);

}  // namespace start
