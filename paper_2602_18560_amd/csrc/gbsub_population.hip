// gbsub_population.hip -- synthetic galactic-binary catalogs drawn on the
// GPU from the population model of Sec. "Population model" (Table "priors",
// appendix "Copulas").
//
// Per source i (one thread each, no communication):
//   * four 53-bit uniforms from two Philox4x32-10 blocks (Salmon et al.,
//     SC 2011) with key = the 64-bit seed and counter = (i, block);
//   * three standard normals by Box-Muller; (z1, z2) = (n1, rho n1 +
//     sqrt(1 - rho^2) n2) is the Gaussian copula pair;
//   * f = inverse CDF of the power law f^alpha_PL on [f_lo, f_hi] at Phi(z1);
//   * log10(fdot) - mu_Gamma = inverse CDF of Gamma(alpha_Gamma, rate
//     beta_Gamma) at Phi(z2): Newton on the regularized incomplete gamma
//     from the Wilson-Hilferty start (z2 is already the normal quantile),
//     kept inside a bisection bracket;
//   * log10(f^(-2/3) A) - mu = exp(sigma n3) (log-normal, shape sigma).
// Outputs are the fp32 catalog columns the subtraction reads.
#include "gbsub_internal.h"

#include <math.h>

namespace gbs {

namespace {

struct Philox4 {
    uint32_t v[4];
};

__device__ __forceinline__ Philox4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                            uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;   // round multipliers
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;   // key increments
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t h0 = __umulhi(M0, c0), l0 = M0 * c0;
        const uint32_t h1 = __umulhi(M1, c2), l1 = M1 * c2;
        const uint32_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += W0;
        k1 += W1;
    }
    return {{c0, c1, c2, c3}};
}

__device__ __forceinline__ double unit53(uint32_t hi, uint32_t lo)
{
    const uint64_t b = ((static_cast<uint64_t>(hi) << 32) | lo) >> 11;
    return (static_cast<double>(b) + 0.5) * 0x1.0p-53;
}

// P(a, x): lower regularized incomplete gamma (series below a + 1, the
// complement of the continued fraction of Q above).
__device__ double reg_gamma_lower(double a, double x, double lga)
{
    if (!(x > 0.0)) return 0.0;
    const double pre = exp(a * log(x) - x - lga);
    if (x < a + 1.0) {
        double t = 1.0 / a, s = t;
        for (int k = 1; k < 1000; ++k) {
            t *= x / (a + k);
            s += t;
            if (fabs(t) < fabs(s) * 1e-17) break;
        }
        return s * pre;
    }
    constexpr double TINY = 1e-300;
    double b = x + 1.0 - a, c = 1.0 / TINY, d = 1.0 / b, h = d;
    for (int k = 1; k < 1000; ++k) {
        const double an = -k * (k - a);
        b += 2.0;
        d = an * d + b;
        d = fabs(d) < TINY ? TINY : d;
        c = b + an / c;
        c = fabs(c) < TINY ? TINY : c;
        d = 1.0 / d;
        const double r = d * c;
        h *= r;
        if (fabs(r - 1.0) <= 4e-16) break;
    }
    return 1.0 - pre * h;
}

// y with P(a, y) = p (unit rate); z = Phi^{-1}(p) seeds Wilson-Hilferty;
// lga = ln Gamma(a).
__device__ double gamma_quantile_unit(double a, double lga, double p, double z)
{
    double y;
    {
        const double c = 1.0 - 1.0 / (9.0 * a) + z / (3.0 * sqrt(a));
        y = c > 0.0 ? a * c * c * c : exp((log(p) + lga + log(a)) / a);   // small-y series start
    }
    double lo = 0.0, hi = INFINITY;
    for (int it = 0; it < 100; ++it) {
        const double P = reg_gamma_lower(a, y, lga);
        if (P < p) lo = y; else hi = y;
        const double dens = exp((a - 1.0) * log(y) - y - lga);
        double yn = y - (P - p) / dens;
        if (!(yn > lo && yn < hi)) yn = isinf(hi) ? 2.0 * y + 1.0 : 0.5 * (lo + hi);
        if (fabs(yn - y) <= 1e-15 * y) {
            y = yn;
            break;
        }
        y = yn;
    }
    return y;
}

__global__ __launch_bounds__(WG) void k_generate(PopParams pp, uint64_t seed, uint64_t first, uint64_t n,
                                                 float *A, float *F, float *FD, uint32_t *id)
{
    const uint32_t k0 = static_cast<uint32_t>(seed), k1 = static_cast<uint32_t>(seed >> 32);
    const double e = pp.alpha_pl + 1.0;
    const double flo_e = pow(pp.f_lo_hz, e), fhi_e = pow(pp.f_hi_hz, e);
    const double rc = sqrt(1.0 - pp.rho * pp.rho);
    const double lga = lgamma(pp.alpha_g);
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * WG + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * WG) {
        const uint64_t s = first + i;
        const uint32_t s0 = static_cast<uint32_t>(s), s1 = static_cast<uint32_t>(s >> 32);
        const Philox4 r = philox10(s0, s1, 0u, 0u, k0, k1);
        const Philox4 q = philox10(s0, s1, 1u, 0u, k0, k1);
        const double u1 = unit53(r.v[0], r.v[1]), u2 = unit53(r.v[2], r.v[3]);
        const double u3 = unit53(q.v[0], q.v[1]), u4 = unit53(q.v[2], q.v[3]);
        constexpr double TWO_PI = 6.283185307179586;
        const double rad = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos(TWO_PI * u2, &sn, &cs);
        const double n1 = rad * cs, n2 = rad * sn;
        const double n3 = sqrt(-2.0 * log(u3)) * cos(TWO_PI * u4);
        const double z1 = n1, z2 = pp.rho * n1 + rc * n2;
        const double pu = 0.5 * erfc(-z1 * 0.7071067811865476);
        const double pv = 0.5 * erfc(-z2 * 0.7071067811865476);
        const double f = pow(flo_e + pu * (fhi_e - flo_e), 1.0 / e);
        const double xt = gamma_quantile_unit(pp.alpha_g, lga, pv, z2) / pp.beta_g;
        const double at = exp(pp.sigma * n3);
        A[i] = static_cast<float>(pow(10.0, at + pp.mu) * pow(f, 2.0 / 3.0));
        F[i] = static_cast<float>(f);
        FD[i] = static_cast<float>(pow(10.0, xt + pp.mu_g));
        if (id) id[i] = static_cast<uint32_t>(s);
    }
}

}  // namespace

hipError_t launch_generate(const PopParams &pp, uint64_t seed, uint64_t first, uint64_t n, float *A, float *F,
                           float *FD, uint32_t *id, hipStream_t st)
{
    if (n == 0) return hipSuccess;
    const uint64_t blocks = (n + WG - 1) / WG;
    const unsigned grid = static_cast<unsigned>(blocks < 16384 ? blocks : 16384);
    k_generate<<<grid, WG, 0, st>>>(pp, seed, first, n, A, F, FD, id);
    return hipGetLastError();
}

}  // namespace gbs
