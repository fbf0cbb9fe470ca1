"""Pins for the oracle's samplers of the vector-borne disease model.

The paper names the distributions of its SEIR listing (Beta priors, Binomial
transitions and observations, Poisson and Uniform initial conditions) but not
the algorithms; the oracle pins Marsaglia-Tsang for Gamma (Beta as a ratio of
Gammas), inversion for Binomials with mean below 10 and Hoermann's BTRS above,
and log k! by summation or the Stirling series. Each is checked here against
an exact reference outside the oracle: mpmath's log-gamma, and the exact
Binomial, Gamma and Beta distributions of scipy.
"""
import math

import mpmath
import numpy as np
import pytest
from scipy import stats


def test_log_factorial_against_mpmath(oracle):
    ks = list(range(0, 40)) + [50, 99, 100, 1000, 7370, 12345, 10 ** 5, 737000, 10 ** 7]
    for k in ks:
        exact = float(mpmath.loggamma(k + 1)) if k > 1 else 0.0
        got = oracle.log_factorial(k)
        assert abs(got - exact) <= 1e-14 * max(1.0, abs(exact)), (k, got, exact)


def test_log_binomial_pmf_against_scipy(oracle):
    rng = np.random.default_rng(5)
    for _ in range(400):
        z = int(rng.integers(0, 9000))
        y = int(rng.integers(0, z + 1)) if z > 0 else 0
        p = float(rng.uniform(0.001, 0.999))
        got = oracle.log_binomial_pmf(y, z, p)
        exact = stats.binom.logpmf(y, z, p)
        assert abs(got - exact) <= 1e-10 * max(1.0, abs(exact)), (y, z, p, got, exact)
    assert oracle.log_binomial_pmf(5, 4, 0.3) == -math.inf
    assert oracle.log_binomial_pmf(0, 7, 0.0) == 0.0 and oracle.log_binomial_pmf(3, 7, 0.0) == -math.inf
    assert oracle.log_binomial_pmf(7, 7, 1.0) == 0.0 and oracle.log_binomial_pmf(6, 7, 1.0) == -math.inf
    assert oracle.log_binomial_pmf(0, 0, 0.4) == 0.0


def chi_square_ok(samples, n, p, alpha=1e-4):
    """Pearson test against the exact pmf, bins merged to expected counts >= 20."""
    counts = np.bincount(samples.astype(np.int64), minlength=n + 1)
    expect = stats.binom.pmf(np.arange(n + 1), n, p) * len(samples)
    obs_b, exp_b, o, e = [], [], 0.0, 0.0
    for c, x in zip(counts, expect):
        o += c
        e += x
        if e >= 20:
            obs_b.append(o)
            exp_b.append(e)
            o = e = 0.0
    if obs_b:
        obs_b[-1] += o
        exp_b[-1] += e
    obs_b, exp_b = np.array(obs_b), np.array(exp_b)
    exp_b *= obs_b.sum() / exp_b.sum()
    chi = ((obs_b - exp_b) ** 2 / exp_b).sum()
    return stats.chi2.sf(chi, len(obs_b) - 1) > alpha, chi, len(obs_b)


@pytest.mark.parametrize("n,p", [
    (1, 0.3), (7, 0.5), (40, 0.1), (200, 0.02),          # inversion (n p < 10)
    (25, 0.4), (100, 0.3), (7370, 0.002), (7370, 0.5),   # BTRS
    (737000, 6.0 / 7.0), (100000, 1.0 / 7.0), (60, 0.95),  # p > 1/2 by symmetry; large n
])
def test_binomial_matches_exact_distribution(oracle, n, p):
    x = oracle.sample("binomial", n, p, 1000 + n, 200000)
    assert x.min() >= 0 and x.max() <= n
    ok, chi, bins = chi_square_ok(x, n, p)
    assert ok, (n, p, chi, bins)
    mean, var = n * p, n * p * (1 - p)
    assert abs(x.mean() - mean) <= 5 * math.sqrt(var / len(x)) + 1e-12


def test_binomial_degenerate_cases(oracle):
    assert np.all(oracle.sample("binomial", 0, 0.4, 1, 10) == 0)
    assert np.all(oracle.sample("binomial", 50, 0.0, 1, 10) == 0)
    assert np.all(oracle.sample("binomial", 50, 1.0, 1, 10) == 50)


@pytest.mark.parametrize("a", [1.0, 1.0 + 2.0 / 4.4, 3.0 - 2.0 / 6.5, 5.0, 30.0])
def test_gamma_matches_exact_distribution(oracle, a):
    x = oracle.sample("gamma", a, 0.0, 77, 100000)
    assert stats.kstest(x, stats.gamma(a).cdf).pvalue > 1e-4
    assert abs(x.mean() - a) <= 5 * math.sqrt(a / len(x))


@pytest.mark.parametrize("a,b", [
    (1.0, 1.0), (1.0 + 2.0 / 4.4, 3.0 - 2.0 / 4.4), (1.0 + 2.0 / 4.5, 3.0 - 2.0 / 4.5),
    (1.0 + 2.0 / 6.5, 3.0 - 2.0 / 6.5),
])
def test_beta_matches_exact_distribution(oracle, a, b):
    x = oracle.sample("beta", a, b, 91, 100000)
    assert np.all((x > 0) & (x < 1))
    assert stats.kstest(x, stats.beta(a, b).cdf).pvalue > 1e-4
