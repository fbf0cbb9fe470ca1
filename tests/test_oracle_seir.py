"""Pins for the oracle's vector-borne disease (SEIR) model (Appendix listing).

With fixed rates and a handful of individuals the model's evidence is a finite
sum, computed exactly by the forward algorithm over the joint counts
(tests/analytic.py, exact Binomial probabilities). The SMC estimate Z_hat is
unbiased for every N, so the mean of Z_hat / Z over many seeds must be 1: a
wrong transition (a dropped term, a swapped rate, the births drawn from the
updated instead of the previous total, a wrong observation weight) shifts it.
"""
import math

import numpy as np
import pytest

import analytic as A
from paper_2112_00364_amd import inputs as I

TINY_Y = [1, 0, 1, -1, 1]
TINY_RATES = (0.5, 0.4, 0.3, 0.6, 0.5, 0.7)
TINY_INIT = (1, 1, 0, 2)


def mean_ratio_within(ratios, k=4.0):
    ratios = np.asarray(ratios)
    m = ratios.mean()
    se = ratios.std(ddof=1) / math.sqrt(len(ratios))
    return abs(m - 1.0) <= k * se, m, se


@pytest.fixture(scope="module")
def tiny_log_z():
    return A.seir_exact_log_evidence(TINY_Y, 3, TINY_RATES, TINY_INIT)


@pytest.mark.parametrize("n", [1, 3])
def test_seir_unbiased_against_forward_algorithm(oracle, tiny_log_z, n):
    spec = I.seir_spec(TINY_Y, 64, n=3, fixed_rates=TINY_RATES, initial=TINY_INIT)
    Z = math.exp(tiny_log_z)
    ratios = []
    for s in range(30000):
        r = oracle.Run(spec, n, s)
        st = r.run_to_end()
        assert st in (oracle.FINISHED, oracle.DEGENERATE)
        ratios.append(math.exp(r.log_z) / Z if st == oracle.FINISHED else 0.0)
    ok, m, se = mean_ratio_within(ratios)
    assert ok, (m, se)


def test_seir_converges_on_tiny_population(oracle, tiny_log_z):
    spec = I.seir_spec(TINY_Y, 64, n=3, fixed_rates=TINY_RATES, initial=TINY_INIT)
    vals = []
    for s in range(8):
        r = oracle.Run(spec, 1 << 16, s)
        assert r.run_to_end() == oracle.FINISHED
        vals.append(r.log_z)
    vals = np.array(vals)
    se = vals.std(ddof=1) / math.sqrt(len(vals))
    assert abs(vals.mean() - tiny_log_z) < 4 * se + 0.005, (vals, tiny_log_z)
    assert vals.std(ddof=1) < 0.1


def test_seir_counts_are_conserved(oracle):
    y = I.seir_data(30, 6001)
    spec = I.seir_spec(y, 32)
    r = oracle.Run(spec, 512, 3)
    while True:
        r.step()
        ints = [r.field(6 + k, np.int32).astype(np.int64) for k in range(10)]
        # humans neither die nor are born: hS + hE + hI + hR stays n
        assert np.all(ints[0] + ints[1] + ints[2] + ints[3] == I.SEIR_HUMANS)
        assert all(np.all(x >= 0) for x in ints[:9])
        assert np.all(ints[9] == r.round + 1)  # day cursor
        if r.resample() != oracle.OK:
            break
    assert r.status == oracle.FINISHED and r.round == len(y) - 1


def test_seir_missing_days_accumulate_new_cases(oracle):
    # every day missing: no weight, z counts all new infectious humans since day 0
    y = [-1.0] * 6
    y[0] = -1.0
    spec = I.seir_spec(y, 64, n=50, fixed_rates=(0.5, 0.4, 0.3, 0.6, 0.5, 0.7), initial=(3, 2, 0, 40))
    r = oracle.Run(spec, 64, 9)
    assert r.run_to_end() == oracle.FINISHED
    assert r.log_z == 0.0
    z = r.field(6 + 8, np.int32)
    hE, hI, hR = (r.field(6 + k, np.int32) for k in (1, 2, 3))
    # z = initial hI + all exposed-to-infectious moves = hI + hR (hR counts recoveries of infectious)
    assert np.array_equal(z, hI + hR)
