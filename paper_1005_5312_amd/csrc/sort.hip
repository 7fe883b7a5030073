// Device-wide exclusive scan and stable LSD radix sort for gfx950 (wave64).
//
// The radix sort orders the Morton keys of sources and targets and the
// depth-first order of the octree.  Each pass sorts on one 8-bit digit:
//   1. per-tile digit histogram (LDS atomics),
//   2. exclusive scan of the digit-major [256][tiles] count table,
//   3. stable scatter: ranks inside a wave come from 8 ballots that match
//      equal digits; waves and rounds are ordered through LDS counters; the
//      tile is staged in LDS in digit order and written out run by run.
#include "internal.h"

namespace start {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;
constexpr int kWaves = kSortThreads / 64;

__device__ inline unsigned block_exclusive_scan(unsigned v, unsigned *lds, unsigned *total)
{
    // Hillis-Steele over 256 threads in LDS (build-time primitive, not hot).
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        unsigned add = t >= off ? lds[t - off] : 0u;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    unsigned incl = lds[t];
    *total = lds[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kScanThreads) scan_tiles(unsigned *data, int64_t n, unsigned *sums)
{
    __shared__ unsigned lds[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    unsigned v[kScanItems];
    unsigned s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? data[i] : 0u;
        s += v[k];
    }
    unsigned total;
    unsigned run = block_exclusive_scan(s, lds, &total);
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) data[i] = run;
        run += v[k];
    }
    if (threadIdx.x == 0 && sums) sums[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) scan_add(unsigned *data, int64_t n, const unsigned *sums)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    const unsigned add = sums[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) data[i] += add;
    }
}

__global__ void __launch_bounds__(kSortThreads) radix_hist(const uint64_t *keys, int64_t n, int shift,
                                                           unsigned *counts, int64_t ntiles)
{
    __shared__ unsigned hist[256];
    hist[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortItems; ++r) {
        int64_t i = base + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&hist[(unsigned)(keys[i] >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = hist[threadIdx.x];
}

__global__ void __launch_bounds__(kSortThreads) radix_scatter(const uint64_t *keys_in, const unsigned *vals_in,
                                                              uint64_t *keys_out, unsigned *vals_out, int64_t n,
                                                              int shift, const unsigned *offsets, int64_t ntiles)
{
    __shared__ unsigned base[256];      // global start of each digit's run of this tile
    __shared__ unsigned loc[256];       // start of each digit inside the tile
    __shared__ unsigned running[256];
    __shared__ unsigned wave_cnt[kWaves][256];
    __shared__ unsigned scan_lds[kSortThreads];
    __shared__ uint64_t skey[kSortTile];
    __shared__ unsigned sval[kSortTile];
    const int t = threadIdx.x;
    const int lane = t & 63;
    const int w = t >> 6;
    const int64_t tile = blockIdx.x;
    // the tile's count of digit t, from the scanned digit-major count table
    const unsigned b0 = offsets[(int64_t)t * ntiles + tile];
    unsigned b1;
    if (tile + 1 < ntiles) b1 = offsets[(int64_t)t * ntiles + tile + 1];
    else b1 = t + 1 < 256 ? offsets[(int64_t)(t + 1) * ntiles] : (unsigned)n;
    base[t] = b0;
    unsigned tile_total;
    loc[t] = block_exclusive_scan(b1 - b0, scan_lds, &tile_total);
    running[t] = 0;
    for (int k = 0; k < kWaves; ++k) wave_cnt[k][t] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile0 = tile * kSortTile;
    // 1. stable rank of every item inside the tile, digit-major: staged in LDS
    for (int r = 0; r < kSortItems; ++r) {
        const int64_t i = tile0 + (int64_t)r * kSortThreads + t;
        const bool valid = i < n;
        uint64_t key = 0;
        unsigned val = 0, d = 0;
        if (valid) {
            key = keys_in[i];
            val = vals_in[i];
            d = (unsigned)(key >> shift) & 0xFFu;
        }
        uint64_t match = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            match &= bit ? bb : ~bb;
        }
        const unsigned rank = __popcll(match & lt_mask);
        if (valid && rank == 0) wave_cnt[w][d] = __popcll(match);
        __syncthreads();
        if (valid) {
            unsigned pre = running[d];
            for (int k = 0; k < w; ++k) pre += wave_cnt[k][d];
            const unsigned at = loc[d] + pre + rank;
            skey[at] = key;
            sval[at] = val;
        }
        __syncthreads();
        unsigned add = 0;
        for (int k = 0; k < kWaves; ++k) {
            add += wave_cnt[k][t];
            wave_cnt[k][t] = 0;
        }
        running[t] += add;
        __syncthreads();
    }
    // 2. out in tile order: neighbouring threads write neighbouring places of
    // one digit's run (coalesced), instead of up to 256 runs per wave
    for (unsigned i = t; i < tile_total; i += kSortThreads) {
        const uint64_t key = skey[i];
        const unsigned d = (unsigned)(key >> shift) & 0xFFu;
        const unsigned dst = base[d] + (i - loc[d]);
        keys_out[dst] = key;
        vals_out[dst] = sval[i];
    }
}

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace

size_t scan_temp_bytes(int64_t n)
{
    size_t total = 0;
    int64_t m = ceil_div(n, kScanTile);
    while (m > 1) {
        total += (size_t)m * sizeof(unsigned) + 256;
        m = ceil_div(m, kScanTile);
    }
    return total + 256;
}

void exclusive_scan_u32(unsigned *d_data, int64_t n, void *temp, hipStream_t s)
{
    if (n <= 0) return;
    int64_t blocks = ceil_div(n, kScanTile);
    if (blocks == 1) {
        scan_tiles<<<1, kScanThreads, 0, s>>>(d_data, n, nullptr);
        return;
    }
    unsigned *sums = reinterpret_cast<unsigned *>(temp);
    char *rest = reinterpret_cast<char *>(temp) + (((size_t)blocks * sizeof(unsigned) + 255) & ~(size_t)255);
    scan_tiles<<<(unsigned)blocks, kScanThreads, 0, s>>>(d_data, n, sums);
    exclusive_scan_u32(sums, blocks, rest, s);
    scan_add<<<(unsigned)blocks, kScanThreads, 0, s>>>(d_data, n, sums);
}

size_t radix_temp_bytes(int64_t n)
{
    int64_t ntiles = ceil_div(n > 0 ? n : 1, kSortTile);
    size_t cnt = (size_t)ntiles * 256;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    return al((size_t)n * sizeof(uint64_t)) + al((size_t)n * sizeof(unsigned)) +
           al(cnt * sizeof(unsigned)) + al(scan_temp_bytes((int64_t)cnt));
}

void radix_sort_pairs(uint64_t *keys, unsigned *vals, int64_t n, int bits, void *temp, hipStream_t s)
{
    if (n <= 1 || bits <= 0) return;
    auto al = [](size_t b) { return (b + 255) & ~(size_t)255; };
    const int64_t ntiles = ceil_div(n, kSortTile);
    char *p = reinterpret_cast<char *>(temp);
    uint64_t *k_alt = reinterpret_cast<uint64_t *>(p);
    p += al((size_t)n * sizeof(uint64_t));
    unsigned *v_alt = reinterpret_cast<unsigned *>(p);
    p += al((size_t)n * sizeof(unsigned));
    unsigned *counts = reinterpret_cast<unsigned *>(p);
    p += al((size_t)ntiles * 256 * sizeof(unsigned));
    void *scan_tmp = p;

    uint64_t *k_in = keys, *k_out = k_alt;
    unsigned *v_in = vals, *v_out = v_alt;
    const int passes = (bits + 7) / 8;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = pass * 8;
        radix_hist<<<(unsigned)ntiles, kSortThreads, 0, s>>>(k_in, n, shift, counts, ntiles);
        exclusive_scan_u32(counts, ntiles * 256, scan_tmp, s);
        radix_scatter<<<(unsigned)ntiles, kSortThreads, 0, s>>>(k_in, v_in, k_out, v_out, n, shift, counts,
                                                                 ntiles);
        uint64_t *tk = k_in;
        k_in = k_out;
        k_out = tk;
        unsigned *tv = v_in;
        v_in = v_out;
        v_out = tv;
    }
    if (k_in != keys) {
        hipMemcpyAsync(keys, k_in, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(vals, v_in, (size_t)n * sizeof(unsigned), hipMemcpyDeviceToDevice, s);
    }
}

}  // namespace start
