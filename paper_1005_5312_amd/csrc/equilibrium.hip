// Per-particle ionisation balance, one particle per thread: the
// photoionisation-equilibrium update, and the terms of the transfer of
// recombination photons of section 4.1 (emission, k_self, total k_ion).
//
// With neutral fraction x, total hydrogen density n_H and photoionisation
// rate per H I atom Gamma (Appendix A, eq. A2 for one frequency), the
// ionisations per unit volume x n_H Gamma balance the recombinations
// alpha n_e n_p = alpha (1 - x)^2 n_H^2 (n_e = n_p = (1 - x) n_H, no helium).
// Under the on-the-spot approximation of section 2.1 alpha is the case-B
// coefficient.  With a = alpha n_H the balance is a x^2 - (2a + Gamma) x + a = 0,
// whose roots multiply to one; the root in [0, 1] is taken as the reciprocal
// of the larger one, x = 2a / (2a + Gamma + sqrt(Gamma (Gamma + 4a))), which
// has no cancellation at any Gamma / a.  a = Gamma = 0 leaves x = 1.
//
// The update also writes n_HI = x n_H for the next grid fill and reduces
// max |x_new - x_old| into one word (non-negative doubles order like their
// bit patterns, so an unsigned atomic max works).
#include "internal.h"

namespace start {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

__device__ inline double block_max(double v)
{
    __shared__ double part[kWaves];
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) part[wv] = v;
    __syncthreads();
    double m = part[0];
    for (int w = 1; w < kWaves; ++w) m = fmax(m, part[w]);
    return m;
}

template <typename TG>
__global__ void __launch_bounds__(kThreads) eq_update(int64_t n, const double *__restrict__ n_h,
                                                      const TG *__restrict__ gamma, double alpha,
                                                      double *__restrict__ x, double *__restrict__ nhi,
                                                      unsigned long long *max_change, unsigned *flags)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double ch = 0.0;
    if (k < n) {
        const double nh = n_h[k], g = (double)gamma[k], xo = x[k];
        if (!isfinite(nh) || !isfinite(g) || !isfinite(xo) || nh < 0.0 || g < 0.0) {
            atomicOr(flags, kFlagEqInput);
        } else {
            const double a = alpha * nh;
            const double den = 2.0 * a + g + sqrt(g * (g + 4.0 * a));
            const double xn = den > 0.0 ? 2.0 * a / den : 1.0;
            ch = fabs(xn - xo);
            x[k] = xn;
            if (nhi) nhi[k] = xn * nh;
        }
    }
    if (!max_change) return;
    const double m = block_max(ch);
    if (threadIdx.x == 0 && m > 0.0) atomicMax(max_change, (unsigned long long)__double_as_longlong(m));
}

// With the transfer of recombination photons (section 4.1) every
// recombination counts (alpha_A) and a particle's own ground-state photons
// reionise it at k_self (eq. 30); with k_self's optical depth (eq. 28) taken
// from the previous x, k_ion = alpha_A n_e n_p is the balance above with
// alpha_eff = alpha_A - alpha_1 (1 - exp(-tau_self)), which is alpha_B where
// the gas is opaque.
template <typename TG>
__global__ void __launch_bounds__(kThreads) eq_update_diffuse(int64_t n, const double *__restrict__ n_h,
                                                              const TG *__restrict__ gamma,
                                                              const double *__restrict__ vol, double sigma,
                                                              double alpha_a, double alpha_1, double *__restrict__ x,
                                                              double *__restrict__ nhi,
                                                              unsigned long long *max_change, unsigned *flags)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    double ch = 0.0;
    if (k < n) {
        const double nh = n_h[k], g = (double)gamma[k], xo = x[k], v = vol[k];
        if (!isfinite(nh) || !isfinite(g) || !isfinite(xo) || !isfinite(v) || nh < 0.0 || g < 0.0 || v < 0.0) {
            atomicOr(flags, kFlagEqInput);
        } else {
            const double tau = sigma * (xo * nh) * cbrt(3.0 * v / (4.0 * M_PI));
            const double alpha = alpha_a - alpha_1 * -expm1(-tau);
            const double a = alpha * nh;
            const double den = 2.0 * a + g + sqrt(g * (g + 4.0 * a));
            const double xn = den > 0.0 ? 2.0 * a / den : 1.0;
            ch = fabs(xn - xo);
            x[k] = xn;
            nhi[k] = xn * nh;
        }
    }
    const double m = block_max(ch);
    if (threadIdx.x == 0 && m > 0.0) atomicMax(max_change, (unsigned long long)__double_as_longlong(m));
}

__global__ void __launch_bounds__(kThreads) iota64(int64_t n, int64_t *__restrict__ out)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k < n) out[k] = k;
}

// Checks n_H >= 0 and x in [0, 1], both finite, and writes n_HI = x n_H.
__global__ void __launch_bounds__(kThreads) eq_prepare(int64_t n, const double *__restrict__ n_h,
                                                       const double *__restrict__ x, double *__restrict__ nhi,
                                                       unsigned *flags)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const double nh = n_h[k], xv = x[k];
    if (!isfinite(nh) || !isfinite(xv) || nh < 0.0 || xv < 0.0 || xv > 1.0) {
        atomicOr(flags, kFlagEqInput);
        nhi[k] = 0.0;
        return;
    }
    nhi[k] = xv * nh;
}

// Recombination photons of each particle (section 4.1): the emission rate
// alpha_1 n_e n_p V of eq. (19) and the part a particle absorbs itself,
// k_self = alpha_1 n_e n_p (1 - exp(-tau)) of eq. (30) with the optical depth
// from its edge to its centre tau = sigma n_HI (3 V / (4 pi))^(1/3) of
// eq. (28); n_e = n_p = (1 - x) n_H.
__global__ void __launch_bounds__(kThreads) recomb_terms(int64_t n, const double *__restrict__ n_h,
                                                         const double *__restrict__ x,
                                                         const double *__restrict__ vol, double sigma,
                                                         double alpha_1, double *__restrict__ lum,
                                                         double *__restrict__ kself, unsigned *flags)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const double nh = n_h[k], xv = x[k], v = vol[k];
    if (!isfinite(nh) || !isfinite(xv) || !isfinite(v) || nh < 0.0 || xv < 0.0 || xv > 1.0 || v < 0.0) {
        atomicOr(flags, kFlagEqInput);
        if (lum) lum[k] = 0.0;
        if (kself) kself[k] = 0.0;
        return;
    }
    const double ne = (1.0 - xv) * nh;
    const double rec = alpha_1 * ne * ne;
    if (lum) lum[k] = rec * v;
    if (kself) {
        const double tau = sigma * (xv * nh) * cbrt(3.0 * v / (4.0 * M_PI));
        kself[k] = rec * -expm1(-tau);
    }
}

// k_ion = n_HI Gamma + k_self (eq. 25), Gamma the rate per H I atom from all
// other emitters (eq. 26 with eq. A2).
template <typename TG>
__global__ void __launch_bounds__(kThreads) total_rate(int64_t n, const double *__restrict__ n_h,
                                                       const double *__restrict__ x, const TG *__restrict__ gamma,
                                                       const double *__restrict__ kself, double *__restrict__ kion,
                                                       unsigned *flags)
{
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= n) return;
    const double nh = n_h[k], xv = x[k], g = (double)gamma[k], ks = kself ? kself[k] : 0.0;
    if (!isfinite(nh) || !isfinite(xv) || !isfinite(g) || !isfinite(ks) || nh < 0.0 || g < 0.0 || ks < 0.0) {
        atomicOr(flags, kFlagEqInput);
        kion[k] = 0.0;
        return;
    }
    kion[k] = xv * nh * g + ks;
}

__global__ void clear_u64(unsigned long long *w) { *w = 0ull; }

}  // namespace

void launch_clear_word(Ctx *c, unsigned long long *w) { clear_u64<<<1, 1, 0, c->stream>>>(w); }

void launch_iota(Ctx *c, int64_t n, int64_t *out)
{
    if (n > 0) iota64<<<blocks_for(n), kThreads, 0, c->stream>>>(n, out);
}

void launch_eq_update_diffuse(Ctx *c, int64_t n, const double *n_h, const void *gamma, int gamma_prec,
                              const double *vol, double sigma, double alpha_a, double alpha_1, double *x, double *nhi,
                              unsigned long long *max_change)
{
    if (n <= 0) return;
    if (gamma_prec == START_FP64)
        eq_update_diffuse<double><<<blocks_for(n), kThreads, 0, c->stream>>>(
            n, n_h, (const double *)gamma, vol, sigma, alpha_a, alpha_1, x, nhi, max_change, c->d_flags);
    else
        eq_update_diffuse<float><<<blocks_for(n), kThreads, 0, c->stream>>>(
            n, n_h, (const float *)gamma, vol, sigma, alpha_a, alpha_1, x, nhi, max_change, c->d_flags);
}

void launch_recomb_terms(Ctx *c, int64_t n, const double *n_h, const double *x, const double *vol, double sigma,
                         double alpha_1, double *lum, double *kself)
{
    if (n <= 0) return;
    recomb_terms<<<blocks_for(n), kThreads, 0, c->stream>>>(n, n_h, x, vol, sigma, alpha_1, lum, kself, c->d_flags);
}

void launch_total_rate(Ctx *c, int64_t n, const double *n_h, const double *x, const void *gamma, int gamma_prec,
                       const double *kself, double *kion)
{
    if (n <= 0) return;
    if (gamma_prec == START_FP64)
        total_rate<double><<<blocks_for(n), kThreads, 0, c->stream>>>(n, n_h, x, (const double *)gamma, kself, kion,
                                                                       c->d_flags);
    else
        total_rate<float><<<blocks_for(n), kThreads, 0, c->stream>>>(n, n_h, x, (const float *)gamma, kself, kion,
                                                                      c->d_flags);
}

void launch_eq_update(Ctx *c, int64_t n, const double *n_h, const void *gamma, int gamma_prec, double alpha,
                      double *x, double *nhi, unsigned long long *max_change)
{
    if (n <= 0) return;
    if (gamma_prec == START_FP64)
        eq_update<double><<<blocks_for(n), kThreads, 0, c->stream>>>(n, n_h, (const double *)gamma, alpha, x, nhi,
                                                                     max_change, c->d_flags);
    else
        eq_update<float><<<blocks_for(n), kThreads, 0, c->stream>>>(n, n_h, (const float *)gamma, alpha, x, nhi,
                                                                    max_change, c->d_flags);
}

void launch_eq_prepare(Ctx *c, int64_t n, const double *n_h, const double *x, double *nhi)
{
    if (n <= 0) return;
    eq_prepare<<<blocks_for(n), kThreads, 0, c->stream>>>(n, n_h, x, nhi, c->d_flags);
}

}  // namespace start
