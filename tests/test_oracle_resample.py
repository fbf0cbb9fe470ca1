"""Pins for the oracle's resampling step (Alg. 1 step 3; systematic resampling, Sec. 3.3).

Checked against: the defining properties of systematic resampling (offspring
counts are floor or ceil of N w_i and sum to N, ancestors sorted), an
independent rational-arithmetic formulation of the ancestor rule, the exact
expectation of the offspring counts over the uniform offset (a sweep over every
breakpoint of U), and the log-mean-exp increment computed in multiprecision.
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest


def grid_bits(n):
    return min(32, 53 - math.ceil(math.log2(n))) if n > 1 else 32


def ancestors_by_fractions(Q, U):
    """Output j sits at mass position (j + U/2^32) * Q_tot / N; it takes the
    first particle whose inclusive cumulative mass exceeds that position."""
    n = len(Q)
    tot = int(Q[-1])
    out = []
    i = 0
    for j in range(n):
        pos = (Fraction(j) + Fraction(U, 2**32)) * Fraction(tot, n)
        while not (int(Q[i]) > pos):
            i += 1
        out.append(i)
    return np.array(out, dtype=np.uint32)


def random_q(rng, n, zero_frac=0.3):
    q = rng.integers(0, 2**20, size=n).astype(np.uint64)
    q[rng.random(n) < zero_frac] = 0
    if q.sum() == 0:
        q[rng.integers(n)] = 1
    return q


@pytest.mark.parametrize("n", [1, 2, 3, 7, 64, 257])
def test_ancestor_rule_matches_fraction_definition(oracle, n):
    rng = np.random.default_rng(n)
    for _ in range(20):
        q = random_q(rng, n)
        Q = np.cumsum(q, dtype=np.uint64)
        U = int(rng.integers(0, 2**32))
        assert np.array_equal(oracle.ancestors(Q, U), ancestors_by_fractions(Q, U))
    # extreme offsets
    q = random_q(rng, n)
    Q = np.cumsum(q, dtype=np.uint64)
    for U in (0, 1, 2**31, 2**32 - 1):
        assert np.array_equal(oracle.ancestors(Q, U), ancestors_by_fractions(Q, U))


@pytest.mark.parametrize("n", [5, 64, 1000, 4099])
def test_offspring_counts_floor_ceil_and_sorted(oracle, n):
    rng = np.random.default_rng(100 + n)
    for _ in range(10):
        q = random_q(rng, n)
        Q = np.cumsum(q, dtype=np.uint64)
        U = int(rng.integers(0, 2**32))
        a = oracle.ancestors(Q, U).astype(np.int64)
        assert np.all(np.diff(a) >= 0)
        counts = np.bincount(a, minlength=n)
        assert counts.sum() == n
        tot = int(Q[-1])
        for i in range(n):
            lo = (n * int(q[i])) // tot
            hi = lo if (n * int(q[i])) % tot == 0 else lo + 1
            assert lo <= counts[i] <= hi
        assert np.all(counts[q == 0] == 0)


def test_exact_expectation_over_offset(oracle):
    """E_u[count_i] = N q_i / Q: sum the counts over every interval of the 2^32 offsets
    U on which the ancestor vector is constant (breakpoints found in exact
    arithmetic). Offsets are discrete, so each of the (at most two) jumps of
    count_i can move the average by 2^-32 from the continuous expectation."""
    rng = np.random.default_rng(9)
    for n in (3, 5, 8):
        q = random_q(rng, n, zero_frac=0.2)
        Q = np.cumsum(q, dtype=np.uint64)
        tot = int(Q[-1])
        # output j changes ancestor where (j 2^32 + U) tot = N Q_i 2^32 for some i
        breaks = {0, 2**32}
        for j in range(n):
            for i in range(n):
                num = n * int(Q[i]) * 2**32 - j * 2**32 * tot
                if num >= 0 and num % tot == 0:
                    b = num // tot
                    if 0 <= b < 2**32:
                        breaks.add(b)
                        breaks.add(b + 1)
                elif num > 0:
                    b = -(-num // tot)
                    if 0 <= b < 2**32:
                        breaks.add(b)
        pts = sorted(breaks)
        expect = [Fraction(0)] * n
        for lo, hi in zip(pts[:-1], pts[1:]):
            a = oracle.ancestors(Q, lo)
            assert np.array_equal(a, oracle.ancestors(Q, hi - 1))
            c = np.bincount(a.astype(np.int64), minlength=n)
            for i in range(n):
                expect[i] += Fraction(int(c[i]) * (hi - lo), 2**32)
        for i in range(n):
            assert abs(expect[i] - Fraction(n * int(q[i]), tot)) <= Fraction(2, 2**32)


def test_equal_weights_identity_and_single_mass(oracle):
    for n in (1, 2, 10, 1000):
        st, anc, inc, qtot = oracle.systematic(np.full(n, -3.25), seed=5, rnd=2)
        assert st == 0
        assert np.array_equal(anc, np.arange(n, dtype=np.uint32))
        assert abs(inc - (-3.25)) < 1e-15
        assert qtot == n * 2 ** grid_bits(n)
    lw = np.full(100, -np.inf)
    lw[37] = 4.0
    st, anc, inc, _ = oracle.systematic(lw, seed=1, rnd=0)
    assert st == 0 and np.all(anc == 37)
    assert abs(inc - (4.0 - math.log(100))) < 1e-14


def test_degenerate_and_nan(oracle):
    st, _, inc, _ = oracle.systematic(np.full(8, -np.inf), 1, 0)
    assert st == oracle.DEGENERATE and inc == -math.inf
    lw = np.zeros(8)
    lw[3] = np.nan
    assert oracle.systematic(lw, 1, 0)[0] == oracle.ERR_NAN


@pytest.mark.parametrize("n", [2, 17, 1000])
def test_log_z_increment_is_log_mean_exp(oracle, n):
    mp.mp.prec = 150
    rng = np.random.default_rng(n)
    lw = rng.normal(0, 5, n) - 700.0
    lw[rng.random(n) < 0.2] = -np.inf
    lw[0] = -690.0
    st, anc, inc, qtot = oracle.systematic(lw, 3, 1)
    exact = mp.log(mp.fsum(mp.exp(mp.mpf(float(x))) for x in lw if x > -np.inf) / n)
    assert abs(inc - float(exact)) < 1e-12 * abs(float(exact))


def test_quantised_weights_grid(oracle):
    """Weights below half a grid unit of the maximum get no offspring; the grid is 2^-G."""
    n = 1000
    G = grid_bits(n)
    assert G == 32
    lw = np.zeros(n)
    lw[1:] = -40.0  # exp(-40) < 2^-33: rounds to 0 on the grid
    st, anc, _, qtot = oracle.systematic(lw, 1, 0)
    assert qtot == 2 ** G
    assert np.all(anc == 0)
    assert grid_bits(1 << 24) == 29 and grid_bits(1 << 20) == 32


def test_resampling_uses_tag_one_and_round(oracle):
    """U is word 0 of Philox(counter {0, 0, round, 1}); different rounds give different U."""
    n = 4
    lw = np.log(np.array([0.1, 0.2, 0.3, 0.4]))
    for rnd in (0, 1, 7):
        U = oracle.word(77, 0, 0, rnd, 1)
        st, anc, _, qtot = oracle.systematic(lw, 77, rnd)
        e = np.array([oracle.exp(x - lw.max()) for x in lw])
        q = np.array([int(round(math.ldexp(v, 32))) for v in e], dtype=np.uint64)
        assert np.array_equal(anc, ancestors_by_fractions(np.cumsum(q, dtype=np.uint64), U))
