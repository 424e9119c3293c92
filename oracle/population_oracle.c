/*
 * population_oracle.c -- plain FP64 CPU oracle of the galactic-binary
 * population model (TEST INFRASTRUCTURE ONLY; part of the oracle library,
 * never loaded by the product path).
 *
 * What it computes follows Sec. "Population model", Table "priors" and
 * appendix "Copulas":
 *   f        power law p(f) ~ f^alpha_PL on [f_lo, f_hi];
 *   fdot~    = log10(fdot) - mu_Gamma ~ Gamma(shape alpha_Gamma, rate beta_Gamma);
 *   A~       = log10(f^(-2/3) A) - mu ~ log-normal with log-scale 0 and shape sigma;
 *   (f, fdot) coupled by a Gaussian copula with correlation rho: a standard
 *   bivariate normal pair (z1, z2) with correlation rho is mapped to
 *   (Phi(z1), Phi(z2)) and then through the inverse marginal CDFs.
 * Random numbers: the counter-based generator Philox4x32-10 (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011), key =
 * the 64-bit seed, counter = (source index, block); uniforms on (0, 1) with
 * 53 bits; normals by the Box-Muller transform.  Every step below is the
 * plain statement of its definition; the inverse Gamma CDF is found by
 * bisection to the last bit, on P summed in binary128.
 */
#include "gbsub_oracle.h"

#include <math.h>
#include <quadmath.h>
#include <stdint.h>

static const double PI = 3.14159265358979323846;

/* ---------------------------------------------------------------- Philox4x32-10 */

static void philox_round(uint32_t c[4], const uint32_t k[2])
{
    const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t n0 = hi1 ^ c[1] ^ k[0];
    const uint32_t n1 = lo1;
    const uint32_t n2 = hi0 ^ c[3] ^ k[1];
    const uint32_t n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr[0], ctr[1], ctr[2], ctr[3]};
    uint32_t k[2] = {key[0], key[1]};
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {                       /* key schedule: Weyl sequence */
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        philox_round(c, k);
    }
    for (int i = 0; i < 4; ++i) out[i] = c[i];
}

/* uniform on (0, 1) from two 32-bit words: the top 53 bits, centred */
static double u53(uint32_t hi, uint32_t lo)
{
    const uint64_t v = (((uint64_t)hi << 32) | lo) >> 11;
    return ((double)v + 0.5) * 0x1.0p-53;
}

/* ---------------------------------------------------------------- special functions */

/* Phi(z), the standard normal CDF */
static double norm_cdf(double z) { return 0.5 * erfc(-z / sqrt(2.0)); }

/* Regularized lower incomplete gamma P(a, x) = gamma(a, x) / Gamma(a), in
 * binary128: x^a e^-x times the series sum_k x^k / Gamma(a + k + 1), which
 * converges for every x and has only positive terms (DLMF 8.7.1), so nothing
 * cancels, not even where P is within an ulp of 1.  Summed until the terms,
 * past their peak at k ~ x - a, fall below 2^-120 of the sum. */
static __float128 gamma_p_q(double a, double x)
{
    if (!(x > 0.0)) return 0;
    const __float128 aq = a, xq = x;
    __float128 term = expq(aq * logq(xq) - xq - lgammaq(aq + 1)), sum = term;
    for (int k = 1; k < 1000000; ++k) {
        term *= xq / (aq + k);
        sum += term;
        if (k > x && term < sum * 0x1p-120Q) break;
    }
    return sum;
}

double orc_gamma_p(double a, double x) { return (double)gamma_p_q(a, x); }

/* x with P(shape, rate * x) = p, by bisection until the bracket stops
 * shrinking (the last representable bit); P is compared in binary128. */
double orc_gamma_quantile(double shape, double rate, double p)
{
    const __float128 pq = p;
    double lo = 0.0, hi = 1.0;
    while (gamma_p_q(shape, hi) < pq) hi *= 2.0;
    for (int it = 0; it < 2000; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (gamma_p_q(shape, mid) < pq) lo = mid; else hi = mid;
    }
    return 0.5 * (lo + hi) / rate;
}

/* ---------------------------------------------------------------- the model */

/* The deterministic part: from the copula uniforms (u, v) and the amplitude
 * normal w to (f, fdot, A). */
void orc_pop_transform(const orc_population *p, double u, double v, double w, double *f, double *fdot,
                       double *A)
{
    const double e = p->alpha_pl + 1.0;               /* alpha_PL != -1 (prior: [-4, -2]) */
    const double a0 = pow(p->f_lo_hz, e), a1 = pow(p->f_hi_hz, e);
    const double ff = pow(a0 + u * (a1 - a0), 1.0 / e);
    const double fdt = orc_gamma_quantile(p->alpha_g, p->beta_g, v);
    const double At = exp(p->sigma * w);              /* log-normal, log-scale 0, shape sigma */
    *f = ff;
    *fdot = pow(10.0, fdt + p->mu_g);
    *A = pow(10.0, At + p->mu) * pow(ff, 2.0 / 3.0);
}

/* Sources first .. first+n-1 of the catalog drawn with `seed`. */
int orc_pop_draw(const orc_population *p, uint64_t seed, uint64_t first, int64_t n, float *A, float *f,
                 float *fdot, uint32_t *id)
{
    if (!p || n < 0 || !(p->f_lo_hz > 0.0) || !(p->f_hi_hz > p->f_lo_hz) || p->alpha_pl == -1.0 ||
        !(p->alpha_g > 0.0) || !(p->beta_g > 0.0) || !(p->sigma >= 0.0) || !(p->rho > -1.0) ||
        !(p->rho < 1.0))
        return ORC_E_INVALID;
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t s = first + (uint64_t)i;
        uint32_t r[4], q[4];
        const uint32_t c0[4] = {(uint32_t)s, (uint32_t)(s >> 32), 0u, 0u};
        const uint32_t c1[4] = {(uint32_t)s, (uint32_t)(s >> 32), 1u, 0u};
        orc_philox4x32_10(c0, key, r);
        orc_philox4x32_10(c1, key, q);
        const double u1 = u53(r[0], r[1]), u2 = u53(r[2], r[3]);
        const double u3 = u53(q[0], q[1]), u4 = u53(q[2], q[3]);
        /* Box-Muller: two independent standard normals from (u1, u2), a third from (u3, u4) */
        const double rad = sqrt(-2.0 * log(u1)), ang = 2.0 * PI * u2;
        const double n1 = rad * cos(ang), n2 = rad * sin(ang);
        const double n3 = sqrt(-2.0 * log(u3)) * cos(2.0 * PI * u4);
        /* Gaussian copula: (z1, z2) standard bivariate normal with correlation rho */
        const double z1 = n1, z2 = p->rho * n1 + sqrt(1.0 - p->rho * p->rho) * n2;
        double ff, fd, aa;
        orc_pop_transform(p, norm_cdf(z1), norm_cdf(z2), n3, &ff, &fd, &aa);
        A[i] = (float)aa;
        f[i] = (float)ff;
        fdot[i] = (float)fd;
        if (id) id[i] = (uint32_t)s;
    }
    return ORC_OK;
}
