"""Pins for ESS-triggered resampling in the oracle.

Sec. 3.3 lists resampling triggered by the effective sample size among
RootPPL's features; the rule is this library's reading: the ESS is taken on
the quantised weights q of the resampling step, ESS = (sum q)^2 / sum q^2,
and a round resamples iff ESS < t N / 2^16 with t = rint(threshold 2^16)
(exact integer comparison). A round that does not resample keeps the
log-weights, takes identity ancestors and leaves log Z alone; the next
resampling (or the end of the run) folds the carried weights into log Z.

What pins it, from outside the oracle:
* the decision, against exact rational arithmetic on weight vectors whose
  quantised values are known integers;
* never resampling is importance sampling: the final log Z equals the log of
  the mean of w^heads computed from the particles' flip counts, and the
  estimate is unbiased;
* ESS-triggered runs stay unbiased (geometric program, Z = 1/(2 - w)) and
  converge to the Kalman evidence of the linear-Gaussian model.
"""
import math
from fractions import Fraction

import numpy as np
import pytest

import analytic as A
from paper_2112_00364_amd import inputs as I


def grid_bits(n):
    return min(32, 53 - math.ceil(math.log2(n))) if n > 1 else 32


def exact_rule(q, t):
    """Resample iff 2^16 (sum q)^2 < t N sum q^2, in exact integers."""
    s1 = sum(q)
    s2 = sum(x * x for x in q)
    return (1 << 16) * s1 * s1 < t * len(q) * s2


def lw_for_grid_units(q, G):
    """Log-weights whose quantised values are exactly the integers q (max 2^G)."""
    return np.array([math.log(x / 2.0 ** G) if x > 0 else -math.inf for x in q])


@pytest.mark.parametrize("n,m,tau,expect", [
    (10, 4, 0.5, 1), (10, 5, 0.5, 0), (10, 6, 0.5, 0),   # ESS = m against tau N = 5
    (10, 10, 1.0, 0), (10, 9, 1.0, 1),                   # tau = 1: only equal weights carry
    (10, 3, 0.3, 1),                                      # t = rint(0.3 2^16) = 19661 > 0.3 2^16
    (7, 7, 0.0, 1),                                       # tau = 0: always resample
])
def test_decision_counts_particles_at_the_maximum(oracle, n, m, tau, expect):
    lw = np.array([0.0] * m + [-math.inf] * (n - m))
    assert oracle.ess_resamples(lw, tau) == expect


def test_decision_rejects_thresholds_outside_unit_interval(oracle):
    assert oracle.ess_resamples(np.zeros(4), -0.1) == -1
    assert oracle.ess_resamples(np.zeros(4), 1.5) == -1


def test_decision_matches_exact_rationals(oracle):
    rng = np.random.default_rng(11)
    for trial in range(300):
        n = int(rng.integers(2, 60))
        G = grid_bits(n)
        q = [int(x) for x in rng.integers(0, 1 << G, size=n)]
        q[int(rng.integers(0, n))] = 1 << G
        if trial % 3 == 0:  # heavy skew: most mass on a few particles
            q = [x >> int(rng.integers(0, 20)) for x in q]
            q[0] = 1 << G
        lw = lw_for_grid_units(q, G)
        # the oracle's quantisation reproduces q exactly (exp error << half a unit)
        tau = float(rng.choice([0.1, 0.25, 0.5, 0.75, 0.9, 1.0, float(rng.random())]))
        t = int(round(tau * 65536))
        assert oracle.ess_resamples(lw, tau) == int(exact_rule(q, t)), (q, tau)
        # exact ESS on the rational weights agrees with the integer form
        ess = Fraction(sum(q)) ** 2 / sum(x * x for x in q)
        assert (ess < Fraction(t * n, 65536)) == exact_rule(q, t)


def test_threshold_zero_is_algorithm_1(oracle):
    spec = I.lgssm_spec(I.lgssm_data(30, 5), 64)
    a = oracle.Run(spec, 512, 3)
    b = oracle.Run(dict(spec, ess_threshold=0.0), 512, 3)
    assert a.run_to_end() == b.run_to_end() == oracle.FINISHED
    assert a.log_z == b.log_z
    assert b.resamples == b.round  # every round before the last resampled


def test_never_resampling_is_importance_sampling(oracle):
    # t = 1: ESS >= 1 > N / 2^16 for N < 2^16, so no round resamples
    w = 1.2
    spec = dict(I.geometric_spec(True, 0.5, w), ess_threshold=1.0 / 65536)
    n = 64
    r = oracle.Run(spec, n, 21)
    while True:
        r.step()
        st = r.resample()
        if st != oracle.OK:
            break
        assert np.array_equal(r.anc(), np.arange(n, dtype=np.uint32))
    assert st == oracle.FINISHED and r.resamples == 0
    flips = r.field(0, np.int32).astype(np.int64)
    heads = flips - 1  # every particle ends on its one tails flip
    expect = math.log(np.mean(np.power(w, heads.astype(np.float64))))
    assert abs(r.log_z - expect) < 1e-12, (r.log_z, expect)


def mean_ratio_within(ratios, k=4.0):
    ratios = np.asarray(ratios)
    m = ratios.mean()
    se = ratios.std(ddof=1) / math.sqrt(len(ratios))
    return abs(m - 1.0) <= k * se, m, se


@pytest.mark.parametrize("tau", [1.0 / 65536, 0.5])
@pytest.mark.parametrize("n", [2, 4])
def test_geometric_unbiased_with_ess_rule(oracle, n, tau):
    spec = dict(I.geometric_spec(True, 0.5, 1.2), ess_threshold=tau)
    Z = A.geometric_Z(0.5, 1.2)
    ratios = []
    for s in range(20000):
        r = oracle.Run(spec, n, s)
        assert r.run_to_end() == oracle.FINISHED
        ratios.append(math.exp(r.log_z) / Z)
    ok, m, se = mean_ratio_within(ratios)
    assert ok, (m, se)


def test_lgssm_ess_half_against_kalman(oracle):
    y = I.lgssm_data(100, 2000)
    spec = dict(I.lgssm_spec(y, 64), ess_threshold=0.5)
    a, b, q, rr, m0, s0 = spec["params"]
    exact = A.kalman_log_evidence(y, a, b, q, rr, m0, s0)
    vals = []
    for s in range(4):
        r = oracle.Run(spec, 1 << 12, s)
        assert r.run_to_end() == oracle.FINISHED
        assert 0 < r.resamples < r.round  # the rule both fires and holds off
        vals.append(r.log_z)
    assert abs(np.mean(vals) - exact) < 0.3, (vals, exact)


def test_carried_rounds_keep_log_z_and_identity_ancestors(oracle):
    spec = dict(I.lgssm_spec(I.lgssm_data(40, 9), 64), ess_threshold=0.5)
    r = oracle.Run(spec, 256, 4)
    carried = 0
    while True:
        r.step()
        before_z, before_res = r.log_z, r.resamples
        lw = r.lw()
        st = r.resample()
        if st != oracle.OK:
            break
        if r.resamples == before_res:
            carried += 1
            assert r.log_z == before_z
            assert np.array_equal(r.anc(), np.arange(256, dtype=np.uint32))
            assert np.array_equal(r.lw(), lw)  # weights carry into the next round
        else:
            assert np.all(r.lw() == 0.0)
    assert carried > 0
