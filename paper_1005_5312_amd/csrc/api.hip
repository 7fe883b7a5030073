// C-ABI entry points of libstart (declared in include/start.h).
#include <cmath>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "internal.h"

namespace start {

start_status build_tree(Ctx *c, const start_box &box, int64_t n, const double *xyz, const double *lum, Tree *t);
start_status build_grid(Ctx *c, const start_box &box, int64_t n, const double *xyz, const double *h,
                        const double *nhi, int grid_log2, Grid *g);
void make_fp32_tree(Tree *t, hipStream_t s);
size_t refit_bytes(const Tree *t);
void refit_prepare(Ctx *c, const Tree *t, void *work);
void refit_tree(Ctx *c, Tree *t, const double *lum, void *work);

// Freed blocks stay with the context and are handed out again for a request
// of the same size: the builds ask for the same sizes at every step, and a
// hipMalloc / hipFree pair costs ~0.3 ms (hipFree waits for the device).  A
// block is released only once the work that used it is done or is ordered
// before any later use: the work of a context runs on its stream, and the
// second stream of start_build_scene only starts after the first is idle and
// releases blocks only after waiting for its own work.  The pool is returned
// to the device when an allocation would fail without it, and when the
// context ends.  A helper context allocates through its owner.
static void release_pool_locked(Ctx *c)
{
    for (auto &b : c->pool) hipFree(b.first);
    c->pool.clear();
    c->pooled = 0;
}

void release_pool(Ctx *c)
{
    if (c->mem_owner) c = c->mem_owner;
    std::lock_guard<std::mutex> lock(c->mem_mu);
    release_pool_locked(c);
}

hipError_t dmalloc(Ctx *c, void **p, size_t bytes)
{
    *p = nullptr;
    if (bytes == 0) bytes = 256;
    if (c->mem_owner) c = c->mem_owner;
    std::lock_guard<std::mutex> lock(c->mem_mu);
    if (c->budget && c->in_use + bytes > c->budget) return hipErrorOutOfMemory;
    for (size_t i = c->pool.size(); i-- > 0;)
        if (c->pool[i].second == bytes) {
            *p = c->pool[i].first;
            c->pool.erase(c->pool.begin() + (std::ptrdiff_t)i);
            c->pooled -= bytes;
            c->in_use += bytes;
            return hipSuccess;
        }
    if (c->budget && c->in_use + c->pooled + bytes > c->budget) release_pool_locked(c);
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess && !c->pool.empty()) {
        (void)hipGetLastError();
        release_pool_locked(c);
        e = hipMalloc(p, bytes);
    }
    if (e == hipSuccess) c->in_use += bytes;
    else *p = nullptr;
    return e;
}

void dfree(Ctx *c, void *p, size_t bytes)
{
    if (!p) return;
    if (bytes == 0) bytes = 256;
    if (c->mem_owner) c = c->mem_owner;
    std::lock_guard<std::mutex> lock(c->mem_mu);
    c->in_use -= bytes < c->in_use ? bytes : c->in_use;
    c->pool.emplace_back(p, bytes);
    c->pooled += bytes;
    // keep the pool bounded: the oldest blocks go back first
    while (c->pooled > kPoolMaxBytes && !c->pool.empty()) {
        hipFree(c->pool.front().first);
        c->pooled -= c->pool.front().second;
        c->pool.erase(c->pool.begin());
    }
}

}  // namespace start

struct start_ctx {
    start::Ctx c;
};
struct start_tree {
    start::Tree t;
};
struct start_grid {
    start::Grid g;
};
// A staged rate batch and the HIP graph of its rate kernels.
struct start_plan {
    start::Ctx *c = nullptr;
    void *scratch = nullptr;     // item and tile tables, sorted targets
    size_t bytes = 0;
    start::BatchLaunch bl{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

using namespace start;

namespace {

start_status fail(start_ctx *ctx, start_status st, const char *msg)
{
    if (ctx) ctx->c.err = msg;
    return st;
}

start_status check_box(start_ctx *ctx, const start_box *box)
{
    if (!box) return fail(ctx, START_EINVAL, "box is NULL");
    for (int k = 0; k < 3; ++k)
        if (!std::isfinite(box->lo[k])) return fail(ctx, START_ENONFINITE, "box corner is not finite");
    if (!std::isfinite(box->size) || !std::isfinite(box->length_unit_cm))
        return fail(ctx, START_ENONFINITE, "box size or unit is not finite");
    if (!(box->size > 0.0) || !(box->length_unit_cm > 0.0))
        return fail(ctx, START_EINVAL, "box size and length unit must be > 0");
    return START_OK;
}

bool same_box(const start_box &a, const start_box &b)
{
    return a.lo[0] == b.lo[0] && a.lo[1] == b.lo[1] && a.lo[2] == b.lo[2] && a.size == b.size &&
           a.length_unit_cm == b.length_unit_cm;
}

start_status ensure_scratch(start_ctx *ctx, size_t bytes)
{
    Ctx &c = ctx->c;
    if (c.scratch_bytes >= bytes) return START_OK;
    hipStreamSynchronize(c.stream);
    dfree(&c, c.scratch, c.scratch_bytes);
    c.scratch = nullptr;
    c.scratch_bytes = 0;
    size_t want = bytes + bytes / 4;
    hipError_t e = dmalloc(&c, &c.scratch, want);
    if (e != hipSuccess) {
        if (c.budget && c.in_use + want > c.budget) return fail(ctx, START_EBUDGET, "HBM budget exceeded");
        return fail(ctx, START_ENOMEM, "device allocation failed");
    }
    c.scratch_bytes = want;
    return START_OK;
}

start_status ensure_stage(start_ctx *ctx, size_t bytes)
{
    Ctx &c = ctx->c;
    if (c.host_stage_bytes >= bytes) return START_OK;
    hipEventSynchronize(c.stage_ev);
    if (c.host_stage) hipHostFree(c.host_stage);
    c.host_stage = nullptr;
    c.host_stage_bytes = 0;
    const size_t want = bytes + bytes / 2 + 4096;
    if (hipHostMalloc(&c.host_stage, want, hipHostMallocDefault) != hipSuccess)
        return fail(ctx, START_ENOMEM, "pinned host allocation failed");
    c.host_stage_bytes = want;
    return START_OK;
}

// Enqueues a batch of rate problems (mode 0 rates, 1 counters, 2 list
// counts, 3 lists), growing scratch and staging when needed.
int size_class(int64_t v, int top)
{
    int k = 0;
    while (k < top && ((int64_t)1 << k) < v) ++k;
    return k;
}

// Total targets and largest source count of a batch (the autotuning key).
void batch_size(const RateSpec *specs, int n, int64_t *total, int64_t *max_src)
{
    *total = 0;
    *max_src = 0;
    for (int i = 0; i < n; ++i) {
        *total += specs[i].n_t;
        if (specs[i].tree->n_src > *max_src) *max_src = specs[i].tree->n_src;
    }
}

// About total / 4096 targets per wave (a power of two in [1, 64]), which
// keeps ~4096 waves in flight for small calls (measured on MI355X: 2^12
// targets run 3x faster with one target per wave than with 64, 2^14 2.4x
// with 4, 2^16 1.7x with 16; from 2^18 on, 64 is as fast as any).
int tile_from_size(int64_t total)
{
    int h = 1;
    while (h < 64 && (int64_t)h * 2 * 4096 <= total) h *= 2;
    return h;
}

// Targets per wavefront: the fixed choice, else the autotuned one for the
// size class, else from the size.
int tile_for(const Ctx &c, int64_t total, int64_t max_src)
{
    if (c.tile_fixed > 0) return c.tile_fixed;
    const int t = c.tile_by_class[size_class(total, 39)][size_class(max_src, 31)];
    return t > 0 ? t : tile_from_size(total);
}

start_status enqueue(start_ctx *ctx, const RateSpec *specs, int n, int mode, int tile_override = 0,
                     BatchLaunch *launch = nullptr)
{
    Ctx &c = ctx->c;
    int64_t total = 0, max_src = 0;
    batch_size(specs, n, &total, &max_src);
    const int tile = tile_override > 0 ? tile_override : tile_for(c, total, max_src);
    const int64_t tiles = batch_tiles(specs, n, tile);
    start_status st = ensure_scratch(ctx, batch_scratch_bytes(total, n, tiles));
    if (st) return st;
    st = ensure_stage(ctx, batch_stage_bytes(n, tiles));
    if (st) return st;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (c.profile && mode == 0) {
        if (c.ev_used + 2 > c.ev_pool.size()) {
            hipEvent_t a = nullptr, b = nullptr;
            if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess)
                return fail(ctx, START_EHIP, "hipEventCreate failed");
            c.ev_pool.push_back(a);
            c.ev_pool.push_back(b);
        }
        ev0 = c.ev_pool[c.ev_used];
        ev1 = c.ev_pool[c.ev_used + 1];
        c.ev_used += 2;
    }
    run_batch(&c, specs, n, mode, tile, c.scratch, ev0, ev1, launch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    return START_OK;
}

RateSpec spec_of(const start_tree *tree, const start_grid *grid, int64_t n_t, const double *tgt_xyz,
                 const int64_t *self_src, double theta, double sigma, int prec)
{
    RateSpec r;
    memset(&r, 0, sizeof(r));
    r.tree = &tree->t;
    r.grid = grid ? &grid->g : nullptr;
    r.n_t = n_t;
    r.tgt_xyz = tgt_xyz;
    r.self_src = self_src;
    r.theta = theta;
    r.sigma = sigma;
    r.prec = prec;
    return r;
}

start_status check_rate_args(start_ctx *ctx, const start_tree *tree, const start_grid *grid, int64_t n_t,
                             const double *tgt, double theta, double sigma, int prec, bool need_grid)
{
    if (!ctx) return START_EINVAL;
    if (!tree) return fail(ctx, START_EINVAL, "tree is NULL");
    if (need_grid && !grid) return fail(ctx, START_EINVAL, "grid is NULL");
    if (n_t < 0) return fail(ctx, START_EINVAL, "n_t < 0");
    if (n_t > 0 && !tgt) return fail(ctx, START_EINVAL, "target positions are NULL");
    if (n_t > ((int64_t)1 << 31) - 1) return fail(ctx, START_EINVAL, "n_t too large");
    if (!std::isfinite(theta) || !std::isfinite(sigma)) return fail(ctx, START_ENONFINITE, "theta or sigma not finite");
    if (theta < 0.0 || sigma < 0.0) return fail(ctx, START_EINVAL, "theta and sigma must be >= 0");
    if (prec != START_FP64 && prec != START_FP32C) return fail(ctx, START_EINVAL, "unknown precision");
    if (need_grid && !same_box(tree->t.box, grid->g.box))
        return fail(ctx, START_EINVAL, "tree and grid were built on different boxes");
    return START_OK;
}

}  // namespace

extern "C" {

start_status start_ctx_create(int device, void *hip_stream, size_t hbm_budget_bytes, start_ctx **out)
{
    if (!out) return START_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return START_EINVAL;
    if (hipSetDevice(device) != hipSuccess) return START_EHIP;
    start_ctx *ctx = new (std::nothrow) start_ctx;
    if (!ctx) return START_ENOMEM;
    ctx->c.device = device;
    ctx->c.budget = hbm_budget_bytes;
    if (hip_stream) {
        ctx->c.stream = (hipStream_t)hip_stream;
    } else {
        if (hipStreamCreateWithFlags(&ctx->c.stream, hipStreamNonBlocking) != hipSuccess) {
            delete ctx;
            return START_EHIP;
        }
        ctx->c.own_stream = true;
    }
    if (hipMalloc((void **)&ctx->c.d_flags, 256) != hipSuccess) {
        if (ctx->c.own_stream) hipStreamDestroy(ctx->c.stream);
        delete ctx;
        return START_ENOMEM;
    }
    hipMemset(ctx->c.d_flags, 0, 256);
    // the builds' readback words (two builds: start_build_scene runs the grid
    // on a helper context beside the tree); without them the builds copy
    // their counts back one by one
    if (hipHostMalloc((void **)&ctx->c.rb, 2 * kReadbackWords * sizeof(unsigned),
                      hipHostMallocMapped | hipHostMallocCoherent) == hipSuccess) {
        if (hipHostGetDevicePointer((void **)&ctx->c.rb_dev, ctx->c.rb, 0) != hipSuccess) {
            hipHostFree(ctx->c.rb);
            ctx->c.rb = nullptr;
            ctx->c.rb_dev = nullptr;
        }
    } else {
        ctx->c.rb = nullptr;
    }
    // this device's address of the fixed scratch of start_compute_rates_noalloc
    // (a failed lookup only disables that entry point, which then says so)
    (void)noalloc_init(device);
    if (hipEventCreateWithFlags(&ctx->c.stage_ev, hipEventDisableTiming) != hipSuccess) {
        hipFree(ctx->c.d_flags);
        if (ctx->c.own_stream) hipStreamDestroy(ctx->c.stream);
        delete ctx;
        return START_EHIP;
    }
    *out = ctx;
    return START_OK;
}

void start_ctx_destroy(start_ctx *ctx)
{
    if (!ctx) return;
    hipSetDevice(ctx->c.device);
    hipStreamSynchronize(ctx->c.stream);
    dfree(&ctx->c, ctx->c.scratch, ctx->c.scratch_bytes);
    release_pool(&ctx->c);
    if (ctx->c.stream2) hipStreamDestroy(ctx->c.stream2);
    if (ctx->c.ev2) hipEventDestroy(ctx->c.ev2);
    for (hipEvent_t ev : ctx->c.ev_pool) hipEventDestroy(ev);
    if (ctx->c.stage_ev) hipEventDestroy(ctx->c.stage_ev);
    if (ctx->c.host_stage) hipHostFree(ctx->c.host_stage);
    if (ctx->c.rb) hipHostFree(ctx->c.rb);
    hipFree(ctx->c.d_flags);
    if (ctx->c.own_stream) hipStreamDestroy(ctx->c.stream);
    delete ctx;
}

const char *start_last_error(const start_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "no context"; }

size_t start_bytes_in_use(const start_ctx *ctx) { return ctx ? ctx->c.in_use : 0; }

start_status start_synchronize(start_ctx *ctx)
{
    if (!ctx) return START_EINVAL;
    hipSetDevice(ctx->c.device);
    hipError_t e = hipStreamSynchronize(ctx->c.stream);
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    unsigned flags = 0;
    e = hipMemcpy(&flags, ctx->c.d_flags, sizeof(unsigned), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    if (!flags) return START_OK;
    hipMemset(ctx->c.d_flags, 0, sizeof(unsigned));
    if (flags & kFlagEqInput)
        return fail(ctx, START_EINVAL, "equilibrium input: n_H or Gamma negative or not finite, or x outside [0, 1]");
    if (flags & kFlagNonFinite) return fail(ctx, START_ENONFINITE, "non-finite target position");
    if (flags & kFlagOutOfBox) return fail(ctx, START_EOUTOFBOX, "target outside the box");
    return fail(ctx, START_EINVAL, "self_src index out of range");
}

start_status start_build_source_tree(start_ctx *ctx, const start_box *box, int64_t n_s, const double *src_xyz,
                                     const double *src_lum, start_tree **out)
{
    if (!ctx || !out) return START_EINVAL;
    *out = nullptr;
    start_status st = check_box(ctx, box);
    if (st) return st;
    if (n_s < 0) return fail(ctx, START_EINVAL, "n_s < 0");
    if (n_s > ((int64_t)1 << 30)) return fail(ctx, START_EINVAL, "n_s too large");
    if (n_s > 0 && (!src_xyz || !src_lum)) return fail(ctx, START_EINVAL, "source arrays are NULL");
    hipSetDevice(ctx->c.device);
    // the flags word is shared with asynchronous rate calls: report theirs first
    st = start_synchronize(ctx);
    if (st) return st;
    start_tree *t = new (std::nothrow) start_tree;
    if (!t) return START_ENOMEM;
    st = build_tree(&ctx->c, *box, n_s, src_xyz, src_lum, &t->t);
    if (st == START_ENOMEM && ctx->c.budget) st = START_EBUDGET;
    if (st) {
        if (ctx->c.err.empty()) ctx->c.err = "tree build failed";
        delete t;
        return st;
    }
    make_fp32_tree(&t->t, ctx->c.stream);
    hipError_t e = hipStreamSynchronize(ctx->c.stream);
    if (e != hipSuccess) {
        start_tree_free(ctx, t);
        return fail(ctx, START_EHIP, hipGetErrorString(e));
    }
    *out = t;
    return START_OK;
}

start_status start_tree_kernel_luminosity(start_ctx *ctx, start_tree *tree, start_lum_form form, const double *src_h,
                                          const double *src_vol)
{
    if (!ctx || !tree) return START_EINVAL;
    if (form != START_LUM_KERNEL_MEAN && form != START_LUM_KERNEL_VOLUME)
        return fail(ctx, START_EINVAL, "unknown luminosity form");
    if (tree->t.n_src > 0 && (!src_h || (form == START_LUM_KERNEL_VOLUME && !src_vol)))
        return fail(ctx, START_EINVAL, "smoothing length or volume array is NULL");
    hipSetDevice(ctx->c.device);
    start_status st = start_synchronize(ctx);
    if (st) return st;
    st = tree_kernel_luminosity(&ctx->c, &tree->t, src_h, src_vol, (int)form);
    if (st == START_ENOMEM && ctx->c.budget) st = START_EBUDGET;
    if (st) {
        if (ctx->c.err.empty()) ctx->c.err = "kernel luminosity failed";
        return st;
    }
    make_fp32_tree(&tree->t, ctx->c.stream);
    hipError_t e = hipStreamSynchronize(ctx->c.stream);
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    return START_OK;
}

start_status start_tree_free(start_ctx *ctx, start_tree *tree)
{
    if (!ctx) return START_EINVAL;
    if (!tree) return START_OK;
    hipSetDevice(ctx->c.device);
    hipStreamSynchronize(ctx->c.stream);
    // all persistent arrays live in one allocation starting at keys
    dfree(&ctx->c, tree->t.keys, tree->t.bytes);
    delete tree;
    return START_OK;
}

// Host-side checks of the grid build's arguments; resolves grid_log2 = 0.
static start_status check_grid_args(start_ctx *ctx, const start_box *box, int64_t n_gas, const double *gas_xyz,
                                    const double *gas_h, const double *gas_nhi, int *grid_log2)
{
    start_status st = check_box(ctx, box);
    if (st) return st;
    if (n_gas < 0) return fail(ctx, START_EINVAL, "n_gas < 0");
    if (n_gas > ((int64_t)1 << 31) - 1) return fail(ctx, START_EINVAL, "n_gas too large");
    if (n_gas > 0 && (!gas_xyz || !gas_h || !gas_nhi)) return fail(ctx, START_EINVAL, "gas arrays are NULL");
    if (*grid_log2 == 0) {
        int gl = 1;
        while (gl < 10 && (double)(1 << gl) < std::cbrt((double)n_gas) - 1e-9) ++gl;
        *grid_log2 = gl;
    }
    if (*grid_log2 < 1 || *grid_log2 > 10) return fail(ctx, START_EINVAL, "grid_log2 must be in [1, 10]");
    return START_OK;
}

start_status start_build_gas_grid(start_ctx *ctx, const start_box *box, int64_t n_gas, const double *gas_xyz,
                                  const double *gas_h, const double *gas_nhi, int grid_log2, start_grid **out)
{
    if (!ctx || !out) return START_EINVAL;
    *out = nullptr;
    start_status st = check_grid_args(ctx, box, n_gas, gas_xyz, gas_h, gas_nhi, &grid_log2);
    if (st) return st;
    hipSetDevice(ctx->c.device);
    st = start_synchronize(ctx);
    if (st) return st;
    start_grid *g = new (std::nothrow) start_grid;
    if (!g) return START_ENOMEM;
    st = build_grid(&ctx->c, *box, n_gas, gas_xyz, gas_h, gas_nhi, grid_log2, &g->g);
    if (st == START_ENOMEM && ctx->c.budget) st = START_EBUDGET;
    if (st) {
        if (ctx->c.err.empty()) ctx->c.err = "grid build failed";
        delete g;
        return st;
    }
    *out = g;
    return START_OK;
}

start_status start_build_scene(start_ctx *ctx, const start_box *box, int64_t n_s, const double *src_xyz,
                               const double *src_lum, int64_t n_gas, const double *gas_xyz, const double *gas_h,
                               const double *gas_nhi, int grid_log2, start_tree **tree_out, start_grid **grid_out)
{
    if (!ctx || !tree_out || !grid_out) return START_EINVAL;
    *tree_out = nullptr;
    *grid_out = nullptr;
    start_status st = check_box(ctx, box);
    if (st) return st;
    if (n_s < 0) return fail(ctx, START_EINVAL, "n_s < 0");
    if (n_s > ((int64_t)1 << 30)) return fail(ctx, START_EINVAL, "n_s too large");
    if (n_s > 0 && (!src_xyz || !src_lum)) return fail(ctx, START_EINVAL, "source arrays are NULL");
    st = check_grid_args(ctx, box, n_gas, gas_xyz, gas_h, gas_nhi, &grid_log2);
    if (st) return st;
    Ctx &c = ctx->c;
    hipSetDevice(c.device);
    st = start_synchronize(ctx);   // also: every pooled block is idle from here on
    if (st) return st;
    if (!c.stream2) {
        if (hipStreamCreateWithFlags(&c.stream2, hipStreamNonBlocking) != hipSuccess) {
            c.stream2 = nullptr;
            return fail(ctx, START_EHIP, "second stream");
        }
        if (hipEventCreateWithFlags(&c.ev2, hipEventDisableTiming) != hipSuccess) {
            c.ev2 = nullptr;
            return fail(ctx, START_EHIP, "second stream event");
        }
    }
    // the grid's stream starts after all work before it on the context's
    hipEventRecord(c.ev2, c.stream);
    hipStreamWaitEvent(c.stream2, c.ev2, 0);
    start_tree *t = new (std::nothrow) start_tree;
    start_grid *g = new (std::nothrow) start_grid;
    if (!t || !g) {
        delete t;
        delete g;
        return START_ENOMEM;
    }
    // the grid is built from a second host thread on the second stream, by
    // a helper context with its own validation word that allocates through
    // this one; build_grid waits for its stream before it returns
    Ctx side;
    side.device = c.device;
    side.stream = c.stream2;
    side.d_flags = c.d_flags + 2;
    side.mem_owner = &c;
    if (c.rb) {
        side.rb = c.rb + kReadbackWords;
        side.rb_dev = c.rb_dev + kReadbackWords;
    }
    start_status gst = START_OK;
    std::thread worker([&]() {
        // no exception may leave the thread (it would end the process)
        try {
            hipSetDevice(side.device);
            gst = build_grid(&side, *box, n_gas, gas_xyz, gas_h, gas_nhi, grid_log2, &g->g);
        } catch (...) {
            side.err = "grid build: host allocation failed";
            gst = START_ENOMEM;
        }
    });
    start_status tst = build_tree(&c, *box, n_s, src_xyz, src_lum, &t->t);
    bool have_tree = tst == START_OK;
    if (have_tree) {
        make_fp32_tree(&t->t, c.stream);
        hipError_t e = hipStreamSynchronize(c.stream);
        if (e != hipSuccess) {
            c.err = hipGetErrorString(e);
            tst = START_EHIP;
        }
    }
    worker.join();
    if (tst == START_ENOMEM && c.budget) tst = START_EBUDGET;
    if (gst == START_ENOMEM && c.budget) gst = START_EBUDGET;
    if (tst || gst) {
        if (have_tree) dfree(&c, t->t.keys, t->t.bytes);
        if (!gst) dfree(&c, g->g.mem, g->g.bytes);
        delete t;
        delete g;
        if (tst) {
            if (c.err.empty()) c.err = "tree build failed";
            return tst;
        }
        c.err = side.err.empty() ? "grid build failed" : side.err;
        return gst;
    }
    *tree_out = t;
    *grid_out = g;
    return START_OK;
}

start_status start_grid_free(start_ctx *ctx, start_grid *grid)
{
    if (!ctx) return START_EINVAL;
    if (!grid) return START_OK;
    hipSetDevice(ctx->c.device);
    hipStreamSynchronize(ctx->c.stream);
    dfree(&ctx->c, grid->g.mem, grid->g.bytes);
    delete grid;
    return START_OK;
}

int start_grid_size(const start_grid *grid) { return grid ? grid->g.G : 0; }

start_status start_compute_rates(start_ctx *ctx, const start_tree *tree, const start_grid *grid, int64_t n_t,
                                 const double *tgt_xyz, const int64_t *self_src, double theta_crit,
                                 double sigma_cm2, start_precision prec, void *gamma_out)
{
    start_status st = check_rate_args(ctx, tree, grid, n_t, tgt_xyz, theta_crit, sigma_cm2, prec, true);
    if (st) return st;
    if (n_t == 0) return START_OK;
    if (!gamma_out) return fail(ctx, START_EINVAL, "gamma_out is NULL");
    hipSetDevice(ctx->c.device);
    RateSpec r = spec_of(tree, grid, n_t, tgt_xyz, self_src, theta_crit, sigma_cm2, prec);
    r.gamma = gamma_out;
    return enqueue(ctx, &r, 1, 0);
}

start_status start_compute_rates_noalloc(start_ctx *ctx, const start_tree *tree, const start_grid *grid,
                                         int64_t n_t, const double *tgt_xyz, const int64_t *self_src,
                                         double theta_crit, double sigma_cm2, start_precision prec, void *gamma_out)
{
    start_status st = check_rate_args(ctx, tree, grid, n_t, tgt_xyz, theta_crit, sigma_cm2, prec, true);
    if (st) return st;
    if (n_t == 0) return START_OK;
    if (!gamma_out) return fail(ctx, START_EINVAL, "gamma_out is NULL");
    hipSetDevice(ctx->c.device);
    RateSpec r = spec_of(tree, grid, n_t, tgt_xyz, self_src, theta_crit, sigma_cm2, prec);
    r.gamma = gamma_out;
    const char *err = nullptr;
    st = noalloc_rates(&ctx->c, r, tile_for(ctx->c, n_t, tree->t.n_src), &err);
    if (st) return fail(ctx, st, err ? err : "start_compute_rates_noalloc failed");
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    return START_OK;
}

start_status start_compute_dissociation_rates(start_ctx *ctx, const start_tree *tree, const start_grid *grid,
                                              int64_t n_t, const double *tgt_xyz, const int64_t *self_src,
                                              double theta_crit, start_precision prec, void *kdis_out)
{
    start_status st = check_rate_args(ctx, tree, grid, n_t, tgt_xyz, theta_crit, 0.0, prec, true);
    if (st) return st;
    if (n_t == 0) return START_OK;
    if (!kdis_out) return fail(ctx, START_EINVAL, "kdis_out is NULL");
    hipSetDevice(ctx->c.device);
    RateSpec r = spec_of(tree, grid, n_t, tgt_xyz, self_src, theta_crit, 0.0, prec);
    r.channel = 1;
    r.gamma = kdis_out;
    return enqueue(ctx, &r, 1, 0);
}

start_status start_compute_rates_upstream(start_ctx *ctx, const start_tree *tree, const start_grid *grid,
                                          int64_t n_gas, const double *gas_xyz, const double *gas_h,
                                          const double *gas_nhi, const int64_t *self_src, double theta_crit,
                                          double sigma_cm2, double *gamma_out, int64_t *offsets_out,
                                          int64_t *parents_out, int64_t capacity, int64_t *n_roots_out)
{
    if (n_roots_out) *n_roots_out = 0;
    start_status st = check_rate_args(ctx, tree, grid, n_gas, gas_xyz, theta_crit, sigma_cm2, START_FP64, true);
    if (st) return st;
    if (n_gas > 0 && (!gas_h || !gas_nhi || !gamma_out)) return fail(ctx, START_EINVAL, "gas arrays are NULL");
    hipSetDevice(ctx->c.device);
    Ctx &c = ctx->c;
    hipStream_t s = c.stream;
    if (n_gas == 0) {
        const int64_t z = 0;
        if (offsets_out && hipMemcpy(offsets_out, &z, sizeof(z), hipMemcpyDefault) != hipSuccess)
            return fail(ctx, START_EHIP, "copy failed");
        return START_OK;
    }
    st = start_synchronize(ctx);
    if (st) return st;
    // every buffer of the call, freed at the end
    std::vector<std::pair<void *, size_t>> bufs;
    auto alloc = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (dmalloc(&c, &p, bytes) != hipSuccess) return nullptr;
        bufs.push_back({p, bytes});
        return p;
    };
    GasBins bins;
    bool have_bins = false;
    auto done = [&](start_status code) {
        hipStreamSynchronize(s);
        if (have_bins) free_bins(&c, &bins);
        for (auto &b : bufs) dfree(&c, b.first, b.second);
        return code;
    };
    auto nomem = [&]() { return done(fail(ctx, c.budget ? START_EBUDGET : START_ENOMEM, "device allocation failed")); };
    const int64_t n = n_gas;
    // 1. list sizes and offsets.  The pairs are indexed with 32-bit offsets:
    // the sizes are first summed in 64 bits and the call is refused before
    // anything is narrowed if the total does not fit.
    int64_t *off64 = (int64_t *)alloc((size_t)(n + 1) * sizeof(int64_t));
    unsigned *off = (unsigned *)alloc((size_t)(n + 1) * sizeof(unsigned));
    void *scan_tmp = alloc(scan_temp_bytes(n + 1) + (size_t)(n + 1) * sizeof(unsigned));
    unsigned long long *total64 = (unsigned long long *)alloc(256);
    if (!off64 || !off || !scan_tmp || !total64) return nomem();
    RateSpec r = spec_of(tree, grid, n, gas_xyz, self_src, theta_crit, sigma_cm2, START_FP64);
    r.counts = off64;
    st = enqueue(ctx, &r, 1, 2);
    if (st) return done(st);
    hipMemsetAsync(total64, 0, sizeof(unsigned long long), s);
    launch_sum_i64(&c, n, off64, total64);
    unsigned long long total = 0;
    hipMemcpyAsync(&total, total64, sizeof(total), hipMemcpyDeviceToHost, s);
    st = start_synchronize(ctx);
    if (st) return done(st);
    if (!upstream_pairs_fit(total)) return done(fail(ctx, START_ECAPACITY, "more than 2^31 - 1 list entries"));
    const int64_t E = (int64_t)total;
    // the pairs' layout: each particle's list contiguous, the lists in the
    // Morton order of the particles, so that the lists of neighbours (searched
    // for each pair) and a pair's upstream pair (read in every jumping round)
    // lie close to the pair; sl[i] = (first pair, count)
    uint64_t *mk = (uint64_t *)alloc((size_t)n * sizeof(uint64_t));
    unsigned *perm = (unsigned *)alloc((size_t)n * sizeof(unsigned));
    void *radix_tmp = alloc(radix_temp_bytes(n));
    unsigned *lc = (unsigned *)alloc((size_t)(n + 1) * sizeof(unsigned));
    uint2 *sl = (uint2 *)alloc((size_t)n * sizeof(uint2));
    int64_t *first_pair = (int64_t *)alloc((size_t)n * sizeof(int64_t));
    unsigned *kflags = (unsigned *)alloc(256);
    if (!mk || !perm || !radix_tmp || !lc || !sl || !first_pair || !kflags) return nomem();
    hipMemsetAsync(kflags, 0, sizeof(unsigned), s);
    launch_keys(tree->t.box, n, gas_xyz, nullptr, mk, perm, kflags, s);
    launch_coarse_keys(&c, n, mk);
    radix_sort_pairs(mk, perm, n, 30, radix_tmp, s);
    launch_layout_counts(&c, n, perm, off64, lc);
    hipMemsetAsync(lc + n, 0, sizeof(unsigned), s);
    exclusive_scan_u32(lc, n + 1, scan_tmp, s);
    launch_layout_starts(&c, n, perm, lc, sl, first_pair);
    // the offsets of the export (lists in particle order)
    launch_to_u32(&c, n, off64, off);
    hipMemsetAsync(off + n, 0, sizeof(unsigned), s);
    exclusive_scan_u32(off, n + 1, scan_tmp, s);
    launch_to_i64(&c, n + 1, off, off64);
    const size_t Eb = (size_t)(E > 0 ? E : 1);
    uint64_t *keys = (uint64_t *)alloc(Eb * sizeof(uint64_t));
    unsigned *owner = (unsigned *)alloc(Eb * sizeof(unsigned));
    // two arrays of 16-byte (tau, parent) records: the search writes the
    // first, pointer jumping alternates between the two
    const size_t lb_bytes = Eb * upstream_link_bytes();
    char *links = (char *)alloc(2 * lb_bytes);
    unsigned *roots = (unsigned *)alloc(Eb * sizeof(unsigned));
    unsigned *words = (unsigned *)alloc(256);   // [0] root count, [1] "more" flag
    const int64_t nslots = n;   // one neighbour count per particle
    unsigned *nbc = (unsigned *)alloc((size_t)(nslots + 1) * sizeof(unsigned));
    void *nb_scan_tmp = alloc(scan_temp_bytes(nslots + 1));
    if (!keys || !owner || !links || !roots || !words || !nbc || !nb_scan_tmp) return nomem();
    // 2. the lists as sorted keys, and the owner of every pair
    r.counts = nullptr;
    r.offsets = first_pair;
    r.entries = (int64_t *)keys;
    st = enqueue(ctx, &r, 1, 4);
    if (st) return done(st);
    launch_pair_owner(&c, n, sl, owner);
    // 3. neighbours within 2h (particles binned on the grid's cells)
    st = bin_gas(&c, tree->t.box, n, gas_xyz, gas_h, gas_nhi, grid->g.grid_log2, &bins);
    if (st) return done(st == START_ENOMEM && c.budget ? START_EBUDGET : st);
    have_bins = true;
    launch_neighbours(&c, bins, n, perm, gas_xyz, gas_h, nbc, nullptr, nullptr);
    // their total in 64 bits, checked before the 32-bit scan is used
    hipMemsetAsync(total64, 0, sizeof(unsigned long long), s);
    launch_sum_u32(&c, nslots, nbc, total64);
    unsigned long long nb_total = 0;
    hipMemcpyAsync(&nb_total, total64, sizeof(nb_total), hipMemcpyDeviceToHost, s);
    hipMemsetAsync(nbc + nslots, 0, sizeof(unsigned), s);
    exclusive_scan_u32(nbc, nslots + 1, nb_scan_tmp, s);
    if (hipStreamSynchronize(s) != hipSuccess) return done(fail(ctx, START_EHIP, "neighbour count failed"));
    if (!neighbour_pairs_fit(nb_total))
        return done(fail(ctx, START_ECAPACITY, "more than 2^31 - 1 neighbour pairs"));
    const unsigned n_nb = (unsigned)nb_total;
    void *nrec = alloc((size_t)(n_nb > 0 ? n_nb : 1) * neighbour_record_bytes());
    if (!nrec) return nomem();
    launch_neighbours(&c, bins, n, perm, gas_xyz, gas_h, nullptr, nbc, nrec);
    // 4. upstream pair of every pair, its step, and the roots.  Membership of
    // a source in a neighbour's list comes from a bit table (one row of
    // n_nodes + n_src bits per particle) where that table is small beside
    // the pair arrays (at most 8 bytes per pair, or 64 MiB); otherwise, or
    // if it cannot be allocated, from searches of the sorted lists.
    unsigned *bits = nullptr;
    unsigned W = 0;
    {
        const int64_t ids = tree->t.n_nodes + tree->t.n_src;
        const int64_t w = (ids + 31) / 32;
        const double table = (double)n * (double)w * 4.0;
        if (table <= std::max(8.0 * (double)E, 64.0 * 1048576.0) && table <= 4.0 * 1073741824.0) {
            bits = (unsigned *)alloc((size_t)n * (size_t)w * sizeof(unsigned));
            if (bits) {
                W = (unsigned)w;
                launch_member_bits(&c, &tree->t, n, E, keys, sl, owner, W, bits);
            }
        }
    }
    hipMemsetAsync(words, 0, 256, s);
    launch_upstream_parent(&c, &tree->t, E, n, gas_xyz, gas_nhi, sl, keys, owner, nbc, nrec, bits, W, sigma_cm2, links,
                           roots, words);
    unsigned n_roots = 0;
    hipMemcpyAsync(&n_roots, words, sizeof(unsigned), hipMemcpyDeviceToHost, s);
    if (hipStreamSynchronize(s) != hipSuccess) return done(fail(ctx, START_EHIP, "upstream search failed"));
    if (n_roots_out) *n_roots_out = n_roots;
    // 5. roots: the column along the ray
    launch_upstream_roots(&c, &tree->t, &grid->g, n_roots, roots, keys, owner, gas_xyz, n, sigma_cm2, (double *)links,
                          (int)(upstream_link_bytes() / sizeof(double)));
    // 6. sums along the chains by pointer jumping
    void *fin = links;
    {
        void *la = links, *lb = links + lb_bytes;
        for (int round = 0;; ++round) {
            if (round > 40) return done(fail(ctx, START_EHIP, "upstream chains did not resolve"));
            hipMemsetAsync(words + 1, 0, sizeof(unsigned), s);
            launch_jump_links(&c, E, la, lb, words + 1);
            std::swap(la, lb);
            unsigned more = 0;
            hipMemcpyAsync(&more, words + 1, sizeof(unsigned), hipMemcpyDeviceToHost, s);
            if (hipStreamSynchronize(s) != hipSuccess) return done(fail(ctx, START_EHIP, "pointer jumping failed"));
            if (!more) break;
        }
        fin = la;
    }
    // 7. the rates
    launch_upstream_gamma(&c, &tree->t, n, gas_xyz, sl, keys, fin, sigma_cm2, gamma_out);
    // exports
    hipError_t e = hipSuccess;
    if (offsets_out) e = hipMemcpyAsync(offsets_out, off64, (size_t)(n + 1) * sizeof(int64_t), hipMemcpyDefault, s);
    if (e == hipSuccess && parents_out) {
        if (E > capacity) return done(fail(ctx, START_ECAPACITY, "parents capacity too small"));
        int64_t *pp = (int64_t *)alloc(Eb * sizeof(int64_t));
        if (!pp) return nomem();
        // the pair-level parent is lost to the jumping; search again, into
        // the record array the rates do not read
        char *spare = (char *)fin == links ? links + lb_bytes : links;
        hipMemsetAsync(words, 0, 256, s);
        launch_upstream_parent(&c, &tree->t, E, n, gas_xyz, gas_nhi, sl, keys, owner, nbc, nrec, bits, W, sigma_cm2,
                               spare, roots, words);
        launch_parent_particle(&c, E, spare, owner, sl, off64, pp);
        if (E > 0) e = hipMemcpyAsync(parents_out, pp, (size_t)E * sizeof(int64_t), hipMemcpyDefault, s);
    }
    if (e != hipSuccess) return done(fail(ctx, START_EHIP, hipGetErrorString(e)));
    st = start_synchronize(ctx);
    return done(st);
}

// Checks the items of a batch and turns the non-empty ones into specs.
static start_status batch_specs(start_ctx *ctx, int n_items, const start_item *items, std::vector<RateSpec> *specs)
{
    if (!ctx) return START_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, START_EINVAL, "bad item array");
    for (int i = 0; i < n_items; ++i) {
        const start_item &it = items[i];
        start_status st = check_rate_args(ctx, it.tree, it.grid, it.n_t, it.tgt_xyz, it.theta_crit, it.sigma_cm2,
                                          it.prec, true);
        if (st) return st;
        if (it.n_t > 0 && !it.gamma_out) return fail(ctx, START_EINVAL, "gamma_out is NULL");
    }
    specs->reserve((size_t)n_items);
    for (int i = 0; i < n_items; ++i) {
        const start_item &it = items[i];
        if (it.n_t == 0) continue;
        RateSpec r = spec_of(it.tree, it.grid, it.n_t, it.tgt_xyz, it.self_src, it.theta_crit, it.sigma_cm2, it.prec);
        r.gamma = it.gamma_out;
        specs->push_back(r);
    }
    return START_OK;
}

start_status start_compute_rates_batched(start_ctx *ctx, int n_items, const start_item *items)
{
    std::vector<RateSpec> specs;
    start_status st = batch_specs(ctx, n_items, items, &specs);
    if (st || specs.empty()) return st;
    hipSetDevice(ctx->c.device);
    return enqueue(ctx, specs.data(), (int)specs.size(), 0);
}

start_status start_rates_plan_create(start_ctx *ctx, int n_items, const start_item *items, start_plan **out)
{
    if (!out) return ctx ? fail(ctx, START_EINVAL, "out is NULL") : START_EINVAL;
    *out = nullptr;
    std::vector<RateSpec> specs;
    start_status st = batch_specs(ctx, n_items, items, &specs);
    if (st) return st;
    Ctx &c = ctx->c;
    hipSetDevice(c.device);
    st = start_synchronize(ctx);
    if (st) return st;
    start_plan *pl = new (std::nothrow) start_plan;
    if (!pl) return START_ENOMEM;
    pl->c = &c;
    if (specs.empty()) {   // nothing to compute: an empty plan
        *out = pl;
        return START_OK;
    }
    const int n = (int)specs.size();
    int64_t total = 0, max_src = 0;
    batch_size(specs.data(), n, &total, &max_src);
    const int tile = tile_for(c, total, max_src);
    const int64_t tiles = batch_tiles(specs.data(), n, tile);
    pl->bytes = batch_scratch_bytes(total, n, tiles);
    st = ensure_stage(ctx, batch_stage_bytes(n, tiles));
    if (st || dmalloc(&c, &pl->scratch, pl->bytes) != hipSuccess) {
        delete pl;
        return st ? st : fail(ctx, c.budget ? START_EBUDGET : START_ENOMEM, "plan allocation failed");
    }
    // stage and run once (this computes the outputs), then capture the rate
    // kernels of the staged batch
    run_batch(&c, specs.data(), n, 0, tile, pl->scratch, nullptr, nullptr, &pl->bl);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        relaunch_batch(pl->bl, c.stream);
        e = hipStreamEndCapture(c.stream, &pl->graph);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipStreamSynchronize(c.stream);
        if (pl->graph) hipGraphDestroy(pl->graph);
        dfree(&c, pl->scratch, pl->bytes);
        delete pl;
        return fail(ctx, START_EHIP, hipGetErrorString(e));
    }
    *out = pl;
    return START_OK;
}

start_status start_rates_plan_launch(start_ctx *ctx, start_plan *plan)
{
    if (!ctx || !plan) return ctx ? fail(ctx, START_EINVAL, "plan is NULL") : START_EINVAL;
    if (plan->c != &ctx->c) return fail(ctx, START_EINVAL, "plan belongs to another context");
    if (!plan->exec) return START_OK;
    hipSetDevice(ctx->c.device);
    const hipError_t e = hipGraphLaunch(plan->exec, ctx->c.stream);
    return e == hipSuccess ? START_OK : fail(ctx, START_EHIP, hipGetErrorString(e));
}

start_status start_rates_plan_free(start_ctx *ctx, start_plan *plan)
{
    if (!ctx) return START_EINVAL;
    if (!plan) return START_OK;
    if (plan->c != &ctx->c) return fail(ctx, START_EINVAL, "plan belongs to another context");
    hipSetDevice(ctx->c.device);
    hipStreamSynchronize(ctx->c.stream);
    if (plan->exec) hipGraphExecDestroy(plan->exec);
    if (plan->graph) hipGraphDestroy(plan->graph);
    dfree(&ctx->c, plan->scratch, plan->bytes);
    delete plan;
    return START_OK;
}

start_status start_equilibrium_update(start_ctx *ctx, int64_t n, const double *n_h, const void *gamma,
                                      start_precision gamma_prec, double alpha, double *x_hi, double *n_hi,
                                      double *max_change)
{
    if (!ctx) return START_EINVAL;
    if (n < 0) return fail(ctx, START_EINVAL, "n < 0");
    if (n > ((int64_t)1 << 31) - 1) return fail(ctx, START_EINVAL, "n too large");
    if (!std::isfinite(alpha)) return fail(ctx, START_ENONFINITE, "alpha not finite");
    if (!(alpha > 0.0)) return fail(ctx, START_EINVAL, "alpha must be > 0");
    if (gamma_prec != START_FP64 && gamma_prec != START_FP32C) return fail(ctx, START_EINVAL, "unknown precision");
    if (n > 0 && (!n_h || !gamma || !x_hi)) return fail(ctx, START_EINVAL, "equilibrium arrays are NULL");
    if (max_change) *max_change = 0.0;
    if (n == 0) return START_OK;
    hipSetDevice(ctx->c.device);
    Ctx &c = ctx->c;
    unsigned long long *word = nullptr;
    if (max_change) {
        start_status st = ensure_scratch(ctx, 256);
        if (st) return st;
        word = (unsigned long long *)c.scratch;
        hipMemsetAsync(word, 0, sizeof(*word), c.stream);
    }
    launch_eq_update(&c, n, n_h, gamma, gamma_prec, alpha, x_hi, n_hi, word);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    if (!max_change) return START_OK;
    unsigned long long bits = 0;
    e = hipMemcpyAsync(&bits, word, sizeof(bits), hipMemcpyDeviceToHost, c.stream);
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    start_status st = start_synchronize(ctx);
    if (st) return st;
    std::memcpy(max_change, &bits, sizeof(double));
    return START_OK;
}

start_status start_recombination_emission(start_ctx *ctx, int64_t n, const double *n_h, const double *x_hi,
                                          const double *volume_cm3, double sigma_cm2, double alpha_1,
                                          double *lum_out, double *k_self_out)
{
    if (!ctx) return START_EINVAL;
    if (n < 0) return fail(ctx, START_EINVAL, "n < 0");
    if (n > ((int64_t)1 << 31) - 1) return fail(ctx, START_EINVAL, "n too large");
    if (!std::isfinite(sigma_cm2) || !std::isfinite(alpha_1)) return fail(ctx, START_ENONFINITE, "sigma or alpha_1 not finite");
    if (sigma_cm2 < 0.0 || alpha_1 < 0.0) return fail(ctx, START_EINVAL, "sigma and alpha_1 must be >= 0");
    if (n > 0 && (!n_h || !x_hi || !volume_cm3)) return fail(ctx, START_EINVAL, "input arrays are NULL");
    if (n == 0 || (!lum_out && !k_self_out)) return START_OK;
    hipSetDevice(ctx->c.device);
    launch_recomb_terms(&ctx->c, n, n_h, x_hi, volume_cm3, sigma_cm2, alpha_1, lum_out, k_self_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    return START_OK;
}

start_status start_total_ionization(start_ctx *ctx, int64_t n, const double *n_h, const double *x_hi,
                                    const void *gamma, start_precision gamma_prec, const double *k_self,
                                    double *k_ion_out)
{
    if (!ctx) return START_EINVAL;
    if (n < 0) return fail(ctx, START_EINVAL, "n < 0");
    if (n > ((int64_t)1 << 31) - 1) return fail(ctx, START_EINVAL, "n too large");
    if (gamma_prec != START_FP64 && gamma_prec != START_FP32C) return fail(ctx, START_EINVAL, "unknown precision");
    if (n > 0 && (!n_h || !x_hi || !gamma || !k_ion_out)) return fail(ctx, START_EINVAL, "input arrays are NULL");
    if (n == 0) return START_OK;
    hipSetDevice(ctx->c.device);
    launch_total_rate(&ctx->c, n, n_h, x_hi, gamma, gamma_prec, k_self, k_ion_out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    return START_OK;
}

start_status start_ionization_equilibrium(start_ctx *ctx, const start_tree *tree, int64_t n_gas,
                                          const double *gas_xyz, const double *gas_h, const double *n_h,
                                          int grid_log2, double theta_crit, double sigma_cm2, double alpha,
                                          start_precision prec, int max_iter, double tol, double *x_hi,
                                          void *gamma_out, int *iterations, double *last_change)
{
    if (iterations) *iterations = 0;
    if (last_change) *last_change = 0.0;
    if (!ctx) return START_EINVAL;
    if (!tree) return fail(ctx, START_EINVAL, "tree is NULL");
    if (n_gas < 0) return fail(ctx, START_EINVAL, "n_gas < 0");
    if (n_gas > ((int64_t)1 << 31) - 1) return fail(ctx, START_EINVAL, "n_gas too large");
    if (n_gas > 0 && (!gas_xyz || !gas_h || !n_h || !x_hi || !gamma_out))
        return fail(ctx, START_EINVAL, "equilibrium arrays are NULL");
    if (!std::isfinite(theta_crit) || !std::isfinite(sigma_cm2) || !std::isfinite(alpha) || !std::isfinite(tol))
        return fail(ctx, START_ENONFINITE, "theta, sigma, alpha or tol not finite");
    if (theta_crit < 0.0 || sigma_cm2 < 0.0 || !(alpha > 0.0) || tol < 0.0)
        return fail(ctx, START_EINVAL, "theta, sigma and tol must be >= 0 and alpha > 0");
    if (prec != START_FP64 && prec != START_FP32C) return fail(ctx, START_EINVAL, "unknown precision");
    if (max_iter < 1) return fail(ctx, START_EINVAL, "max_iter must be >= 1");
    if (grid_log2 < 1 || grid_log2 > 10) return fail(ctx, START_EINVAL, "grid_log2 must be in [1, 10]");
    if (n_gas == 0) return START_OK;
    hipSetDevice(ctx->c.device);
    start_status st = start_synchronize(ctx);
    if (st) return st;
    Ctx &c = ctx->c;
    const start_box box = tree->t.box;
    double *nhi = nullptr;
    const size_t nhi_bytes = (size_t)n_gas * sizeof(double) + 256;
    if (dmalloc(&c, (void **)&nhi, nhi_bytes) != hipSuccess)
        return fail(ctx, c.budget ? START_EBUDGET : START_ENOMEM, "equilibrium buffer allocation failed");
    unsigned long long *word = (unsigned long long *)((char *)nhi + (size_t)n_gas * sizeof(double));
    GasBins bins;
    Grid grid;
    bool have_grid = false, have_bins = false;
    auto cleanup = [&](start_status code) {
        hipStreamSynchronize(c.stream);
        if (have_bins) free_bins(&c, &bins);
        if (have_grid) dfree(&c, grid.mem, grid.bytes);
        dfree(&c, nhi, nhi_bytes);
        return code;
    };
    launch_eq_prepare(&c, n_gas, n_h, x_hi, nhi);
    st = start_synchronize(ctx);
    if (st) return cleanup(st);
    c.err.clear();
    st = bin_gas(&c, box, n_gas, gas_xyz, gas_h, nhi, grid_log2, &bins);
    if (st == START_ENOMEM && c.budget) st = START_EBUDGET;
    if (st) return cleanup(st);
    have_bins = true;
    st = alloc_grid(&c, box, grid_log2, &grid);
    if (st) return cleanup(fail(ctx, c.budget ? START_EBUDGET : START_ENOMEM, "grid allocation failed"));
    have_grid = true;
    start_grid gh;
    gh.g = grid;
    RateSpec r = spec_of(tree, &gh, n_gas, gas_xyz, nullptr, theta_crit, sigma_cm2, prec);
    r.gamma = gamma_out;
    // The first iteration stages the rate call (tables, target sort); the
    // later ones repeat the same kernels on the same buffers (grid refill,
    // rate kernels, equilibrium update), replayed from a HIP graph when
    // graphs are on.
    BatchLaunch bl{};
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
    auto iteration_kernels = [&]() {
        fill_grid(&c, bins, nhi, &grid);
        relaunch_batch(bl, c.stream);
        launch_clear_word(&c, word);
        launch_eq_update(&c, n_gas, n_h, gamma_out, prec, alpha, x_hi, nhi, word);
    };
    auto drop_graph = [&]() {
        if (gexec) hipGraphExecDestroy(gexec);
        if (graph) hipGraphDestroy(graph);
        gexec = nullptr;
        graph = nullptr;
    };
    for (int it = 1; it <= max_iter; ++it) {
        if (it == 1) {
            fill_grid(&c, bins, nullptr, &grid);
            st = enqueue(ctx, &r, 1, 0, 0, &bl);
            if (st) return cleanup(st);
            launch_clear_word(&c, word);
            launch_eq_update(&c, n_gas, n_h, gamma_out, prec, alpha, x_hi, nhi, word);
        } else if (c.graphs) {
            if (!gexec) {
                hipError_t e = hipStreamBeginCapture(c.stream, hipStreamCaptureModeThreadLocal);
                if (e == hipSuccess) {
                    iteration_kernels();
                    e = hipStreamEndCapture(c.stream, &graph);
                }
                if (e == hipSuccess) e = hipGraphInstantiate(&gexec, graph, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    drop_graph();
                    return cleanup(fail(ctx, START_EHIP, hipGetErrorString(e)));
                }
            }
            hipError_t e = hipGraphLaunch(gexec, c.stream);
            if (e != hipSuccess) {
                drop_graph();
                return cleanup(fail(ctx, START_EHIP, hipGetErrorString(e)));
            }
        } else {
            iteration_kernels();
        }
        unsigned long long bits = 0;
        hipError_t e = hipMemcpyAsync(&bits, word, sizeof(bits), hipMemcpyDeviceToHost, c.stream);
        if (e != hipSuccess) {
            drop_graph();
            return cleanup(fail(ctx, START_EHIP, hipGetErrorString(e)));
        }
        st = start_synchronize(ctx);
        if (st) {
            drop_graph();
            return cleanup(st);
        }
        double change;
        std::memcpy(&change, &bits, sizeof(double));
        if (it == 1 && it < max_iter && !(change <= tol) && c.grid_pairs) {
            // later refills read the recorded (centre, particle) pairs; without
            // the memory for them they search the stencil as before
            const start_status pst = record_pairs(&c, &bins, &grid);
            if (pst != START_OK && pst != START_ENOMEM) {
                drop_graph();
                return cleanup(fail(ctx, pst, "grid pair recording failed"));
            }
        }
        if (iterations) *iterations = it;
        if (last_change) *last_change = change;
        if (change <= tol) break;
    }
    drop_graph();
    return cleanup(START_OK);
}

start_status start_diffuse_equilibrium(start_ctx *ctx, const start_box *box, int64_t n_gas, const double *gas_xyz,
                                       const double *gas_h, const double *n_h, const double *volume_cm3,
                                       int64_t n_star, const double *star_xyz, const double *star_lum, int grid_log2,
                                       double theta_crit, double sigma_cm2, double alpha_a, double alpha_1,
                                       start_precision prec, int max_iter, double tol, double *x_hi, void *gamma_out,
                                       int *iterations, double *last_change)
{
    if (iterations) *iterations = 0;
    if (last_change) *last_change = 0.0;
    if (!ctx) return START_EINVAL;
    start_status st = check_box(ctx, box);
    if (st) return st;
    if (n_gas < 0 || n_star < 0) return fail(ctx, START_EINVAL, "n_gas or n_star < 0");
    if (n_gas + n_star > ((int64_t)1 << 30)) return fail(ctx, START_EINVAL, "too many particles and stars");
    if (n_gas > 0 && (!gas_xyz || !gas_h || !n_h || !volume_cm3 || !x_hi || !gamma_out))
        return fail(ctx, START_EINVAL, "equilibrium arrays are NULL");
    if (n_star > 0 && (!star_xyz || !star_lum)) return fail(ctx, START_EINVAL, "star arrays are NULL");
    if (!std::isfinite(theta_crit) || !std::isfinite(sigma_cm2) || !std::isfinite(alpha_a) || !std::isfinite(alpha_1) ||
        !std::isfinite(tol))
        return fail(ctx, START_ENONFINITE, "theta, sigma, alpha or tol not finite");
    if (theta_crit < 0.0 || sigma_cm2 < 0.0 || alpha_1 < 0.0 || !(alpha_a > alpha_1) || tol < 0.0)
        return fail(ctx, START_EINVAL, "need theta, sigma, tol >= 0 and alpha_A > alpha_1 >= 0");
    if (prec != START_FP64 && prec != START_FP32C) return fail(ctx, START_EINVAL, "unknown precision");
    if (max_iter < 1) return fail(ctx, START_EINVAL, "max_iter must be >= 1");
    if (grid_log2 < 1 || grid_log2 > 10) return fail(ctx, START_EINVAL, "grid_log2 must be in [1, 10]");
    if (n_gas == 0) return START_OK;
    hipSetDevice(ctx->c.device);
    st = start_synchronize(ctx);
    if (st) return st;
    Ctx &c = ctx->c;
    hipStream_t s = c.stream;
    const int64_t n = n_gas, ns = n + n_star;
    std::vector<std::pair<void *, size_t>> bufs;
    auto alloc = [&](size_t bytes) -> void * {
        void *p = nullptr;
        if (dmalloc(&c, &p, bytes) != hipSuccess) return nullptr;
        bufs.push_back({p, bytes});
        return p;
    };
    GasBins bins;
    Grid grid;
    Tree tree;
    bool have_bins = false, have_grid = false, have_tree = false;
    auto free_tree = [&]() {
        if (have_tree) dfree(&c, tree.keys, tree.bytes);
        have_tree = false;
    };
    auto done = [&](start_status code) {
        hipStreamSynchronize(s);
        free_tree();
        if (have_bins) free_bins(&c, &bins);
        if (have_grid) dfree(&c, grid.mem, grid.bytes);
        for (auto &b : bufs) dfree(&c, b.first, b.second);
        return code;
    };
    auto nomem = [&]() { return done(fail(ctx, c.budget ? START_EBUDGET : START_ENOMEM, "device allocation failed")); };
    double *src = (double *)alloc((size_t)ns * 3 * sizeof(double));
    double *lum = (double *)alloc((size_t)ns * sizeof(double));
    int64_t *self = (int64_t *)alloc((size_t)n * sizeof(int64_t));
    double *nhi = (double *)alloc((size_t)n * sizeof(double));
    unsigned long long *word = (unsigned long long *)alloc(256);
    if (!src || !lum || !self || !nhi || !word) return nomem();
    // sources: the particles, then the stars (positions fixed)
    for (int k = 0; k < 3; ++k) {
        hipMemcpyAsync(src + (size_t)k * ns, gas_xyz + (size_t)k * n, (size_t)n * sizeof(double),
                       hipMemcpyDeviceToDevice, s);
        if (n_star > 0)
            hipMemcpyAsync(src + (size_t)k * ns + n, star_xyz + (size_t)k * n_star, (size_t)n_star * sizeof(double),
                           hipMemcpyDeviceToDevice, s);
    }
    if (n_star > 0)
        hipMemcpyAsync(lum + n, star_lum, (size_t)n_star * sizeof(double), hipMemcpyDeviceToDevice, s);
    launch_iota(&c, n, self);
    launch_eq_prepare(&c, n, n_h, x_hi, nhi);
    st = start_synchronize(ctx);
    if (st) return done(st);
    c.err.clear();
    st = bin_gas(&c, *box, n, gas_xyz, gas_h, nhi, grid_log2, &bins);
    if (st) return done(st == START_ENOMEM && c.budget ? START_EBUDGET : st);
    have_bins = true;
    if (alloc_grid(&c, *box, grid_log2, &grid)) return nomem();
    have_grid = true;
    start_grid gh;
    start_tree th;
    void *refit_work = nullptr;
    for (int it = 1; it <= max_iter; ++it) {
        // emitters: alpha_1 n_e n_p V of the current x (eq. 19)
        launch_recomb_terms(&c, n, n_h, x_hi, volume_cm3, sigma_cm2, alpha_1, lum, nullptr);
        if (it == 1) {
            st = start_synchronize(ctx);
            if (st) return done(st);
            st = build_tree(&c, *box, ns, src, lum, &tree);
            if (st) return done(st == START_ENOMEM && c.budget ? START_EBUDGET : st);
            have_tree = true;
            refit_work = alloc(refit_bytes(&tree));
            if (!refit_work) return nomem();
            refit_prepare(&c, &tree, refit_work);
        } else {
            // the emitters do not move: the same tree with new luminosities
            refit_tree(&c, &tree, lum, refit_work);
        }
        make_fp32_tree(&tree, s);
        fill_grid(&c, bins, it == 1 ? nullptr : nhi, &grid);
        gh.g = grid;
        th.t = tree;
        RateSpec r = spec_of(&th, &gh, n, gas_xyz, self, theta_crit, sigma_cm2, prec);
        r.gamma = gamma_out;
        st = enqueue(ctx, &r, 1, 0);
        if (st) return done(st);
        launch_clear_word(&c, word);
        launch_eq_update_diffuse(&c, n, n_h, gamma_out, prec, volume_cm3, sigma_cm2, alpha_a, alpha_1, x_hi, nhi,
                                 word);
        unsigned long long bits = 0;
        hipError_t e = hipMemcpyAsync(&bits, word, sizeof(bits), hipMemcpyDeviceToHost, s);
        if (e != hipSuccess) return done(fail(ctx, START_EHIP, hipGetErrorString(e)));
        st = start_synchronize(ctx);
        if (st) return done(st);
        double change;
        std::memcpy(&change, &bits, sizeof(double));
        if (it == 1 && it < max_iter && !(change <= tol) && c.grid_pairs) {
            const start_status pst = record_pairs(&c, &bins, &grid);   // as in the on-the-spot loop
            if (pst != START_OK && pst != START_ENOMEM) return done(fail(ctx, pst, "grid pair recording failed"));
        }
        if (iterations) *iterations = it;
        if (last_change) *last_change = change;
        if (change <= tol) break;
    }
    return done(START_OK);
}

start_status start_set_graph_replay(start_ctx *ctx, int enable)
{
    if (!ctx) return START_EINVAL;
    ctx->c.graphs = enable != 0;
    return START_OK;
}

start_status start_set_grid_pairs(start_ctx *ctx, int enable)
{
    if (!ctx) return START_EINVAL;
    ctx->c.grid_pairs = enable != 0;
    return START_OK;
}

start_status start_set_tile_targets(start_ctx *ctx, int tile_targets)
{
    if (!ctx) return START_EINVAL;
    if (tile_targets < 0 || tile_targets > 64) return fail(ctx, START_EINVAL, "tile_targets must be in [0, 64]");
    ctx->c.tile_fixed = tile_targets;
    return START_OK;
}

start_status start_autotune_rates(start_ctx *ctx, int n_items, const start_item *items, int reps, int *best_tile,
                                  double *best_ms)
{
    if (best_tile) *best_tile = 0;
    if (best_ms) *best_ms = 0.0;
    if (!ctx) return START_EINVAL;
    if (n_items < 0 || (n_items > 0 && !items)) return fail(ctx, START_EINVAL, "bad item array");
    if (reps < 1) return fail(ctx, START_EINVAL, "reps must be >= 1");
    std::vector<RateSpec> specs;
    for (int i = 0; i < n_items; ++i) {
        const start_item &it = items[i];
        start_status st = check_rate_args(ctx, it.tree, it.grid, it.n_t, it.tgt_xyz, it.theta_crit, it.sigma_cm2,
                                          it.prec, true);
        if (st) return st;
        if (it.n_t > 0 && !it.gamma_out) return fail(ctx, START_EINVAL, "gamma_out is NULL");
        if (it.n_t == 0) continue;
        RateSpec r = spec_of(it.tree, it.grid, it.n_t, it.tgt_xyz, it.self_src, it.theta_crit, it.sigma_cm2, it.prec);
        r.gamma = it.gamma_out;
        specs.push_back(r);
    }
    if (specs.empty()) return START_OK;
    int64_t total = 0, max_src = 0;
    batch_size(specs.data(), (int)specs.size(), &total, &max_src);
    hipSetDevice(ctx->c.device);
    start_status st = start_synchronize(ctx);
    if (st) return st;
    Ctx &c = ctx->c;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) hipEventDestroy(e0);
        return fail(ctx, START_EHIP, "hipEventCreate failed");
    }
    // candidates: the size-based choice first, then 64 (one target per lane)
    // down to one target per wave (the whole wave on one target's rays); a
    // candidate twice as slow as the best so far on its first run is not
    // repeated
    const int first = tile_from_size(total);
    const int cand[] = {first, 64, 32, 16, 8, 4, 1};
    int best = first;
    double best_t = 0.0;
    for (int ci = 0; ci < (int)(sizeof(cand) / sizeof(cand[0])) && st == START_OK; ++ci) {
        const int tile = cand[ci];
        if (ci > 0 && tile == first) continue;
        st = enqueue(ctx, specs.data(), (int)specs.size(), 0, tile);   // warm (and sizes scratch)
        if (st) break;
        double sum = 0.0;
        int runs = 0;
        for (int r = 0; r < reps; ++r) {
            hipEventRecord(e0, c.stream);
            st = enqueue(ctx, specs.data(), (int)specs.size(), 0, tile);
            if (st) break;
            hipEventRecord(e1, c.stream);
            if (hipEventSynchronize(e1) != hipSuccess) { st = fail(ctx, START_EHIP, "event wait failed"); break; }
            float ms = 0.0f;
            hipEventElapsedTime(&ms, e0, e1);
            sum += ms;
            ++runs;
            if (r == 0 && best_t > 0.0 && ms > 2.0 * best_t) break;
        }
        if (st || runs == 0) break;
        const double t = sum / runs;
        // the size-based choice is kept unless another size is clearly (3%)
        // faster: run-to-run noise must not pick a worse default
        if (best_t == 0.0 || t < (best == first ? 0.97 : 1.0) * best_t) {
            best_t = t;
            best = tile;
        } else if (tile < best && t > 1.25 * best_t) {
            break;   // still smaller tiles only add walk work
        }
    }
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    if (st) return st;
    st = start_synchronize(ctx);
    if (st) return st;
    c.tile_by_class[size_class(total, 39)][size_class(max_src, 31)] = best;
    if (best_tile) *best_tile = best;
    if (best_ms) *best_ms = best_t;
    return START_OK;
}

size_t start_estimate_bytes(int64_t n_t, int64_t n_s, int64_t n_gas, int grid_log2, start_precision prec)
{
    (void)prec;
    if (n_t < 0 || n_s < 0 || n_gas < 0 || grid_log2 < 0 || grid_log2 > 10) return 0;
    const size_t G3 = (size_t)1 << (3 * grid_log2);
    const int64_t G = (int64_t)1 << grid_log2, pad = (G >= 64 && G <= 512) ? 16 : 0;
    const size_t span = (size_t)((G - 1) * (G * (G + pad) + pad) + (G - 1) * (G + pad) + G);   // padded grid
    // tree: persistent (keys, perm, sources, 2 n_s nodes) + build temporaries
    const size_t tree = (size_t)n_s * (8 + 4 + 32 + 16) + (size_t)2 * n_s * (16 + 16 + 32 + 16 + 32) +
                        radix_temp_bytes(2 * n_s) + (size_t)n_s * 48 + (size_t)2 * n_s * 45 + 65536;
    // both grid copies with their guard bands (G <= 512)
    const int64_t sy = G + pad, sx = G * sy + pad;
    const size_t guard = G <= 512 ? (size_t)(6 * (sx + sy + 1)) : 0;
    const size_t grid = (span + 2 * guard) * 12 + (size_t)n_gas * 56 + radix_temp_bytes(n_gas) +
                        G3 * 4 * kMaxReachClasses + 65536;
    const size_t rates = (batch_scratch_bytes(n_t, 1, n_t) * 5) / 4 + 65536;   // up to one tile per target
    return tree + grid + rates;
}

start_status start_tree_export(start_ctx *ctx, const start_tree *tree, int64_t *n_nodes, uint64_t *keys_sorted,
                               uint32_t *perm, int32_t *node_geo, int32_t *node_link, double *node_mom)
{
    if (!ctx || !tree) return START_EINVAL;
    hipSetDevice(ctx->c.device);
    hipStreamSynchronize(ctx->c.stream);
    const Tree &t = tree->t;
    if (n_nodes) *n_nodes = t.n_nodes;
    const size_t m = (size_t)t.n_nodes, n = (size_t)t.n_src;
    hipError_t e = hipSuccess;
    if (keys_sorted && n) e = hipMemcpy(keys_sorted, t.keys, n * sizeof(uint64_t), hipMemcpyDefault);
    if (e == hipSuccess && perm && n) e = hipMemcpy(perm, t.perm, n * sizeof(unsigned), hipMemcpyDefault);
    if (e == hipSuccess && node_geo && m) e = hipMemcpy(node_geo, t.geo, m * sizeof(int4), hipMemcpyDefault);
    if (e == hipSuccess && node_mom && m) e = hipMemcpy(node_mom, t.mom, m * sizeof(double4), hipMemcpyDefault);
    if (e == hipSuccess && node_link && m) {
        std::vector<int> a(m), b(m), c(m), d(m);
        std::vector<int32_t> link(4 * m);
        e = hipMemcpy(a.data(), t.skip, m * sizeof(int), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(b.data(), t.first, m * sizeof(int), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(c.data(), t.count, m * sizeof(int), hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(d.data(), t.ref, m * sizeof(int), hipMemcpyDeviceToHost);
        for (size_t i = 0; i < m; ++i) {
            link[4 * i] = a[i];
            link[4 * i + 1] = b[i];
            link[4 * i + 2] = c[i];
            link[4 * i + 3] = d[i];
        }
        if (e == hipSuccess) e = hipMemcpy(node_link, link.data(), 4 * m * sizeof(int32_t), hipMemcpyDefault);
    }
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    return START_OK;
}

start_status start_interaction_lists(start_ctx *ctx, const start_tree *tree, int64_t n_t, const double *tgt_xyz,
                                     const int64_t *self_src, double theta_crit, int64_t *offsets,
                                     int64_t *entries, int64_t capacity)
{
    start_status st = check_rate_args(ctx, tree, nullptr, n_t, tgt_xyz, theta_crit, 0.0, START_FP64, false);
    if (st) return st;
    if (!offsets) return fail(ctx, START_EINVAL, "offsets is NULL");
    hipSetDevice(ctx->c.device);
    std::vector<int64_t> off((size_t)n_t + 1, 0);
    if (n_t == 0) {
        hipError_t e = hipMemcpy(offsets, off.data(), sizeof(int64_t), hipMemcpyDefault);
        return e == hipSuccess ? START_OK : fail(ctx, START_EHIP, hipGetErrorString(e));
    }
    hipStream_t s = ctx->c.stream;
    int64_t *d_counts = nullptr;
    if (dmalloc(&ctx->c, (void **)&d_counts, (size_t)(n_t + 1) * sizeof(int64_t)) != hipSuccess)
        return fail(ctx, START_ENOMEM, "device allocation failed");
    RateSpec r = spec_of(tree, nullptr, n_t, tgt_xyz, self_src, theta_crit, 0.0, START_FP64);
    r.counts = d_counts;
    st = enqueue(ctx, &r, 1, 2);
    if (!st) st = start_synchronize(ctx);
    if (st) {
        dfree(&ctx->c, d_counts, (size_t)(n_t + 1) * sizeof(int64_t));
        return st;
    }
    hipMemcpy(off.data() + 1, d_counts, (size_t)n_t * sizeof(int64_t), hipMemcpyDeviceToHost);
    for (int64_t i = 0; i < n_t; ++i) off[i + 1] += off[i];
    hipError_t e = hipMemcpy(offsets, off.data(), (size_t)(n_t + 1) * sizeof(int64_t), hipMemcpyDefault);
    if (e != hipSuccess || off[n_t] > capacity || !entries) {
        dfree(&ctx->c, d_counts, (size_t)(n_t + 1) * sizeof(int64_t));
        if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
        return fail(ctx, START_ECAPACITY, "entries capacity too small");
    }
    // offsets to the device, then the lists straight into a device staging buffer
    hipMemcpy(d_counts, off.data(), (size_t)(n_t + 1) * sizeof(int64_t), hipMemcpyHostToDevice);
    int64_t *d_ent = nullptr;
    const size_t ent_bytes = (size_t)(off[n_t] > 0 ? off[n_t] : 1) * sizeof(int64_t);
    if (dmalloc(&ctx->c, (void **)&d_ent, ent_bytes) != hipSuccess) {
        dfree(&ctx->c, d_counts, (size_t)(n_t + 1) * sizeof(int64_t));
        return fail(ctx, START_ENOMEM, "device allocation failed");
    }
    r.counts = nullptr;
    r.offsets = d_counts;
    r.entries = d_ent;
    st = enqueue(ctx, &r, 1, 3);
    e = hipStreamSynchronize(s);
    if (!st && e == hipSuccess && off[n_t] > 0)
        e = hipMemcpy(entries, d_ent, (size_t)off[n_t] * sizeof(int64_t), hipMemcpyDefault);
    dfree(&ctx->c, d_ent, ent_bytes);
    dfree(&ctx->c, d_counts, (size_t)(n_t + 1) * sizeof(int64_t));
    if (st) return st;
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    return START_OK;
}

start_status start_grid_export(start_ctx *ctx, const start_grid *grid, double *values)
{
    if (!ctx || !grid || !values) return START_EINVAL;
    hipSetDevice(ctx->c.device);
    hipStreamSynchronize(ctx->c.stream);
    const size_t n = (size_t)grid->g.G * grid->g.G * grid->g.G;
    double *lin = nullptr;
    if (dmalloc(&ctx->c, (void **)&lin, n * sizeof(double)) != hipSuccess)
        return fail(ctx, START_ENOMEM, "device allocation failed");
    launch_grid_unpad(&ctx->c, grid->g, lin);
    hipError_t e = hipStreamSynchronize(ctx->c.stream);
    if (e == hipSuccess) e = hipMemcpy(values, lin, n * sizeof(double), hipMemcpyDefault);
    dfree(&ctx->c, lin, n * sizeof(double));
    return e == hipSuccess ? START_OK : fail(ctx, START_EHIP, hipGetErrorString(e));
}

start_status start_rate_counters(start_ctx *ctx, const start_tree *tree, const start_grid *grid, int64_t n_t,
                                 const double *tgt_xyz, const int64_t *self_src, double theta_crit,
                                 start_precision prec, int64_t *counters)
{
    start_status st = check_rate_args(ctx, tree, grid, n_t, tgt_xyz, theta_crit, 0.0, prec, true);
    if (st) return st;
    if (n_t == 0) return START_OK;
    if (!counters) return fail(ctx, START_EINVAL, "counters is NULL");
    hipSetDevice(ctx->c.device);
    int64_t *d_stats = nullptr;
    const size_t bytes = (size_t)n_t * 4 * sizeof(int64_t);
    if (dmalloc(&ctx->c, (void **)&d_stats, bytes) != hipSuccess) return fail(ctx, START_ENOMEM, "allocation failed");
    RateSpec r = spec_of(tree, grid, n_t, tgt_xyz, self_src, theta_crit, 1.0, prec);
    r.stats = d_stats;
    st = enqueue(ctx, &r, 1, 1);
    if (!st) st = start_synchronize(ctx);
    hipError_t e = hipSuccess;
    if (!st) e = hipMemcpy(counters, d_stats, bytes, hipMemcpyDefault);
    dfree(&ctx->c, d_stats, bytes);
    if (st) return st;
    return e == hipSuccess ? START_OK : fail(ctx, START_EHIP, hipGetErrorString(e));
}

start_status start_profile_enable(start_ctx *ctx, int enable)
{
    if (!ctx) return START_EINVAL;
    ctx->c.profile = enable != 0;
    return START_OK;
}

start_status start_profile_read(start_ctx *ctx, int64_t *launches, double *total_ms, double *max_ms)
{
    if (!ctx) return START_EINVAL;
    Ctx &c = ctx->c;
    hipSetDevice(c.device);
    hipError_t e = hipStreamSynchronize(c.stream);
    if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
    double tot = 0.0, mx = 0.0;
    for (size_t i = 0; i + 1 < c.ev_used; i += 2) {
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, c.ev_pool[i], c.ev_pool[i + 1]);
        if (e != hipSuccess) return fail(ctx, START_EHIP, hipGetErrorString(e));
        tot += ms;
        mx = ms > mx ? ms : mx;
    }
    if (launches) *launches = (int64_t)(c.ev_used / 2);
    if (total_ms) *total_ms = tot;
    if (max_ms) *max_ms = mx;
    c.ev_used = 0;
    return START_OK;
}

}  // extern "C"
