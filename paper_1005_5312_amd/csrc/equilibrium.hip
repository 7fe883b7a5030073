// Photoionisation equilibrium of pure hydrogen, one particle per thread.
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

}  // namespace

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
