// start_compute_rates_noalloc: the rate call of start_compute_rates with its
// temporaries (target keys and order, sorted positions, sort buffers, item
// and tile tables) in a fixed array that the library holds on every device
// it runs on, for callers that cannot allocate device memory.
//
// The array lives in the code object (file-scope __device__), so each GPU
// has its own copy at its own address.  Host code never uses the array's
// name as an address: its device address is looked up once per device with
// hipGetSymbolAddress when the first context on that device is created, and
// that address is what the kernels receive.  Every call on a GPU shares the
// array, so calls that overlap on one GPU (two streams, two contexts, two
// host threads) race; nothing in it needs to start at zero (each pass of
// the path writes what it later reads).
#include <mutex>

#include "internal.h"

namespace start {

namespace {

// Enough for any call of up to kNoAllocMaxTargets targets at any tile size.
constexpr int64_t kNoAllocMaxTargets = (int64_t)1 << 18;
constexpr size_t kScratchBytes = (size_t)24 << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_mu;
void *g_ptr[kMaxDevices] = {};

// This device's address of the array (null if not looked up).
void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(g_mu);
    return g_ptr[device];
}

}  // namespace

bool noalloc_init(int device)
{
    if (device < 0 || device >= kMaxDevices) return false;
    std::lock_guard<std::mutex> lock(g_mu);
    if (g_ptr[device]) return true;
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return false;
    }
    g_ptr[device] = p;
    return true;
}

// Enqueues one rate call on the fixed scratch; sizes beyond it are refused.
start_status noalloc_rates(Ctx *c, const RateSpec &r, int tile, const char **err)
{
    *err = nullptr;
    if (r.n_t > kNoAllocMaxTargets) {
        *err = "more targets than the fixed scratch of start_compute_rates_noalloc holds (2^18)";
        return START_ECAPACITY;
    }
    const size_t need = batch_scratch_bytes(r.n_t, 1, batch_tiles(&r, 1, tile));
    if (need > kScratchBytes) {
        *err = "the call needs more than the fixed scratch of start_compute_rates_noalloc (24 MiB)";
        return START_ECAPACITY;
    }
    void *p = scratch_ptr(c->device);
    if (!p) {
        *err = "the fixed scratch of start_compute_rates_noalloc is not available on this device";
        return START_EHIP;
    }
    run_single_fixed(c, r, tile, p);
    return START_OK;
}

}  // namespace start
