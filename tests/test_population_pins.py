"""Pins of the population-model oracle (oracle/population_oracle.c) against
what the paper and the mathematics fix (Sec. "Population model", Table
"priors", appendix "Copulas"), independent of the oracle's own code:

* Philox4x32-10 known-answer vectors of its published reference;
* the Gamma quantile against scipy's inverse regularized incomplete gamma;
* the transform on chosen uniforms against the closed-form inverse CDFs;
* the three marginals of a drawn catalog against scipy's distributions
  (Kolmogorov-Smirnov), whatever the copula correlation;
* the copula: Kendall's tau of (f, fdot) equals (2/pi) arcsin(rho) for a
  Gaussian copula, and the amplitude is independent of f after rescaling.
"""
import math

import numpy as np
import pytest
import scipy.special as sp
import scipy.stats as st

from oracle import oracle as O


@pytest.mark.parametrize("ctr,key,expect", [
    ((0, 0, 0, 0), (0, 0), (0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8)),
    ((0xffffffff,) * 4, (0xffffffff,) * 2, (0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd)),
    ((0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344), (0xa4093822, 0x299f31d0),
     (0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1)),
])
def test_philox_known_answers(ctr, key, expect):
    assert O.philox4x32_10(ctr, key) == expect


def test_gamma_p_and_quantile_against_scipy():
    rng = np.random.default_rng(1)
    for _ in range(200):
        a = rng.uniform(0.5, 5.0)
        x = rng.uniform(1e-3, 20.0)
        assert abs(O.gamma_p(a, x) - sp.gammainc(a, x)) <= 1e-13
        p = rng.uniform(1e-9, 1.0 - 1e-9)
        rate = rng.uniform(1.0, 3.0)
        q = O.gamma_quantile(a, rate, p)
        ref = sp.gammaincinv(a, p) / rate
        assert abs(q - ref) <= 1e-12 * ref


def test_transform_closed_forms():
    pop = O.population(alpha_pl=-3.0, alpha_g=1.0, beta_g=2.0, mu_g=-21.0, mu=-22.0, sigma=0.2)
    for u, v, w in [(0.1, 0.3, -1.0), (0.5, 0.5, 0.0), (0.9, 0.99, 2.0)]:
        f, fd, A = O.pop_transform(pop, u, v, w)
        lo, hi = 1e-4, 1e-2
        f_ref = (lo ** -2 + u * (hi ** -2 - lo ** -2)) ** -0.5      # inverse CDF of f^-3 on [lo, hi]
        x_ref = -math.log1p(-v) / 2.0                              # Gamma(1, rate 2) is exponential
        A_ref = 10.0 ** (math.exp(0.2 * w) - 22.0) * f_ref ** (2.0 / 3.0)
        assert abs(f - f_ref) <= 1e-14 * f_ref
        assert abs(math.log10(fd) - (x_ref - 21.0)) <= 1e-13
        assert abs(A - A_ref) <= 1e-13 * A_ref


@pytest.mark.parametrize("rho", [0.0, 0.6, 0.99])
def test_marginals_and_copula(rho):
    pop = O.population(alpha_pl=-2.9, alpha_g=1.96, beta_g=1.8, mu_g=-21.0, mu=-22.0, sigma=0.18,
                       rho=rho)
    n = 200_000
    A, f, fd, ids = O.pop_draw(pop, seed=11, n=n)
    assert np.array_equal(ids, np.arange(n, dtype=np.uint32))
    f64 = f.astype(np.float64)
    lo, hi, e = 1e-4, 1e-2, pop.alpha_pl + 1.0
    assert f64.min() >= lo * (1 - 1e-6) and f64.max() <= hi * (1 + 1e-6)
    cdf_f = lambda x: (np.power(x, e) - lo ** e) / (hi ** e - lo ** e)
    assert st.kstest(f64, cdf_f).pvalue > 1e-3
    xt = np.log10(fd.astype(np.float64)) - pop.mu_g
    assert st.kstest(xt, st.gamma(a=pop.alpha_g, scale=1.0 / pop.beta_g).cdf).pvalue > 1e-3
    at = np.log10(np.power(f64, -2.0 / 3.0) * A.astype(np.float64)) - pop.mu
    assert st.kstest(at, st.lognorm(s=pop.sigma).cdf).pvalue > 1e-3
    m = 20_000
    tau = st.kendalltau(f64[:m], xt[:m]).statistic
    assert abs(tau - 2.0 / math.pi * math.asin(rho)) < 0.02
    assert abs(st.kendalltau(f64[:m], at[:m]).statistic) < 0.02


def test_draw_is_a_function_of_seed_and_index():
    pop = O.population()
    a = O.pop_draw(pop, seed=5, n=1000)
    b = O.pop_draw(pop, seed=5, n=400, first=600)
    for x, y in zip(a, b):
        assert np.array_equal(x[600:], y)
    c = O.pop_draw(pop, seed=6, n=1000)
    assert not np.array_equal(a[1], c[1])
