"""Pins for CRBD with static delayed sampling (the paper's CRBD experiment with
variance-reducing techniques, Sec. 5.3).

The paper states that delayed sampling was added to the CRBD models by hand
but not how; the oracle marginalises lambda and mu by Gamma conjugacy
(Negative Binomial predictive for hidden speciation counts, Lomax predictive
for hidden lifetimes, closed-form predictive factors for branch survival and
observed speciations). The estimate targets the same marginal likelihood as
CRBD with sampled rates, so it is pinned against the 2-D quadrature of the
closed-form likelihood over the Gamma priors (tests/analytic.py), and its
samplers against scipy's exact distributions.
"""
import math

import numpy as np
import pytest
from scipy import stats

import analytic as A
from paper_2112_00364_amd import inputs as I

SMALL_TREE = ((((0.0, 0.0, 0.21), 0.0, 0.55), ((0.0, 0.0, 0.33), 0.0, 0.62), 1.0))


def chi_square_ok(x, pmf, alpha=1e-4):
    x = x.astype(np.int64)
    kmax = int(x.max())
    counts = np.bincount(x, minlength=kmax + 1)
    expect = pmf(np.arange(kmax + 1)) * len(x)
    tail = (1.0 - pmf(np.arange(kmax + 1)).sum()) * len(x)
    obs_b, exp_b, o, e = [], [], 0.0, 0.0
    for c, v in zip(counts, expect):
        o += c
        e += v
        if e >= 20:
            obs_b.append(o)
            exp_b.append(e)
            o = e = 0.0
    obs_b[-1] += o
    exp_b[-1] += e + tail
    obs_b, exp_b = np.array(obs_b), np.array(exp_b)
    chi = ((obs_b - exp_b) ** 2 / exp_b).sum()
    return stats.chi2.sf(chi, len(obs_b) - 1) > alpha, chi


@pytest.mark.parametrize("a,th", [(1.0, 0.5), (3.0, 0.2), (7.0, 1.5), (2.0, 4.0), (40.0, 0.05)])
def test_negative_binomial_predictive(oracle, a, th):
    x = oracle.sample("negbin", a, th, 17, 200000)
    ok, chi = chi_square_ok(x, lambda k: stats.nbinom.pmf(k, a, 1.0 / (1.0 + th)))
    assert ok, (a, th, chi)


@pytest.mark.parametrize("a,th", [(1.0, 0.5), (4.0, 2.0), (25.0, 0.1)])
def test_lomax_predictive(oracle, a, th):
    x = oracle.sample("lomax", a, th, 19, 100000)
    assert np.all(x >= 0.0)
    assert stats.kstest(x, stats.lomax(a, scale=1.0 / th).cdf).pvalue > 1e-4


def mean_ratio_within(ratios, k=4.0):
    ratios = np.asarray(ratios)
    m = ratios.mean()
    se = ratios.std(ddof=1) / math.sqrt(len(ratios))
    return abs(m - 1.0) <= k * se, m, se


def test_unbiased_against_quadrature(oracle):
    tree = I.tree_from_newick_like(SMALL_TREE)
    Z = math.exp(A.crbd_log_marginal(tree, n_grid=200))
    spec = I.crbd_ds_spec(tree)
    ratios = []
    for s in range(20000):
        r = oracle.Run(spec, 4, s)
        st = r.run_to_end()
        ratios.append(math.exp(r.log_z) / Z if st == oracle.FINISHED else 0.0)
    ok, m, se = mean_ratio_within(ratios)
    assert ok, (m, se)


def test_converges_to_quadrature_with_less_variance(oracle):
    tree = I.yule_tree(6, 7)
    exact = A.crbd_log_marginal(tree, n_grid=200)
    ds = np.array([oracle.Run(I.crbd_ds_spec(tree), 1 << 13, 100 + s) for s in range(12)], dtype=object)
    vals = []
    for r in ds:
        assert r.run_to_end() == oracle.FINISHED
        vals.append(r.log_z)
    vals = np.array(vals)
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(vals.mean() - exact) < 4 * se + 2e-3, (vals.mean(), exact, se)
    plain = []
    for s in range(12):
        r = oracle.Run(I.crbd_spec(tree), 1 << 13, 100 + s)
        r.run_to_end()
        plain.append(r.log_z)
    assert vals.std(ddof=1) < np.std(plain, ddof=1), (vals.std(ddof=1), np.std(plain, ddof=1))


def test_posterior_bookkeeping(oracle):
    tree = I.yule_tree(12, 3)
    r = oracle.Run(I.crbd_ds_spec(tree), 256, 5)
    prev_th_l = prev_th_mu = None
    internal_seen = 0
    while True:
        r.step()
        a_l, th_l, a_mu, th_mu = (r.field(k, np.float64) for k in range(4))
        assert np.all(a_l == np.floor(a_l)) and np.all(a_mu == np.floor(a_mu))  # shapes stay integers
        assert np.all(a_l >= 1.0 + internal_seen)  # one per observed speciation, more for hidden ones
        if prev_th_l is not None:
            assert np.all(th_l <= prev_th_l) and np.all(th_mu < prev_th_mu)  # scales only shrink
        node = r.round  # the block of round r walked node r
        if node >= 1 and tree["left"][node] >= 0:
            internal_seen += 1
        st = r.resample()
        if st != oracle.OK:
            break
        prev_th_l, prev_th_mu = r.field(1, np.float64), r.field(3, np.float64)
    assert r.status == oracle.FINISHED
