"""Pins for the oracle's primitives: Philox, uniforms, elementary functions, samplers.

Each check compares against something outside the oracle: published known-answer
vectors, rocRAND's Philox engine run on the host, multi-precision values from
mpmath, or exact Poisson quantiles.
"""
import json
import math
import os
import shutil
import subprocess
import tempfile

import mpmath as mp
import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def ulp_error(got, exact):
    exact_f = float(exact)
    if exact_f == 0.0:
        return abs(got) / 5e-324
    e = math.frexp(abs(exact_f))[1]
    ulp = math.ldexp(1.0, e - 53)
    return float(abs(mp.mpf(got) - exact) / ulp)


def test_philox_known_answers(oracle):
    kat = json.load(open(os.path.join(GOLDEN, "philox4x32_10_kat.json")))
    for v in kat["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        out = [int(x, 16) for x in v["out"]]
        assert list(oracle.philox(ctr, key)) == out


ROCRAND_PROBE = r"""
#include <cstdio>
#include <cstdlib>
#include <rocrand/rocrand_philox4x32_10.h>
int main(int argc, char** argv) {
    // args: key(64-bit) subsequence(64-bit: counter words 2,3) block(64-bit: counter words 0,1)
    unsigned long long key = strtoull(argv[1], 0, 10);
    unsigned long long sub = strtoull(argv[2], 0, 10);
    unsigned long long blk = strtoull(argv[3], 0, 10);
    rocrand_device::philox4x32_10_engine e(key, sub, blk * 4ull);
    for (int i = 0; i < 4; ++i) printf("%u\n", e.next());
    return 0;
}
"""


def test_philox_matches_rocrand_engine(oracle):
    """rocRAND's philox4x32_10 engine, run on the host, as an independent library check."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc) or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "probe.cpp")
        exe = os.path.join(d, "probe")
        open(src, "w").write(ROCRAND_PROBE)
        r = subprocess.run([hipcc, "-O1", "-x", "hip", "--offload-arch=gfx950",
                            "-o", exe, src], capture_output=True, text=True)
        if r.returncode != 0:
            pytest.skip("could not build the rocRAND host probe: " + r.stderr[-400:])
        rng = np.random.default_rng(11)
        for _ in range(6):
            key = int(rng.integers(0, 2**63))
            c = [int(x) for x in rng.integers(0, 2**32, size=4)]
            c[1] &= 0x3FFFFFFF  # the engine takes the block index as a word offset (4 x block)
            sub = c[2] | (c[3] << 32)
            blk = c[0] | (c[1] << 32)
            out = subprocess.run([exe, str(key), str(sub), str(blk)], capture_output=True,
                                 text=True, check=True).stdout.split()
            ref = [int(x) for x in out]
            mine = oracle.philox(c, [key & 0xFFFFFFFF, key >> 32])
            assert list(mine) == ref


def test_word_stream_layout(oracle):
    """Word k of (particle, round, tag) is lane k%4 of counter {k/4, particle, round, tag}."""
    seed = 0x1234_5678_9ABC_DEF0
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for k in (0, 1, 2, 3, 4, 7, 41):
        blk = oracle.philox([k // 4, 5, 9, 1], key)
        assert oracle.word(seed, k, 5, 9, 1) == blk[k % 4]


def test_uniform_open_interval_exact(oracle):
    assert oracle.uniform_from_word(0) == 2.0 ** -33
    assert oracle.uniform_from_word(2**32 - 1) == 1.0 - 2.0 ** -33
    ws = np.random.default_rng(0).integers(0, 2**32, size=2000)
    for w in ws:
        u = oracle.uniform_from_word(int(w))
        assert 0.0 < u < 1.0
        assert mp.mpf(u) == (2 * mp.mpf(int(w)) + 1) / mp.mpf(2) ** 33


def test_exp_accuracy_and_specials(oracle):
    mp.mp.prec = 120
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-708, 709, 6000), rng.uniform(-1, 1, 3000),
                         rng.uniform(-40, 0, 3000), [0.0, -0.0, 1e-300, -1e-300, 0.5, -0.5,
                                                     math.log(2), -745.0 + 37.5, 708.9]])
    worst = 0.0
    for x in xs:
        worst = max(worst, ulp_error(oracle.exp(x), mp.exp(mp.mpf(float(x)))))
    assert worst <= 1.0, worst
    assert oracle.exp(0.0) == 1.0
    assert oracle.exp(-math.inf) == 0.0
    assert oracle.exp(math.inf) == math.inf
    assert math.isnan(oracle.exp(math.nan))
    assert oracle.exp(-708.5) == 0.0      # pinned flush below -708
    assert oracle.exp(709.5) == math.inf  # pinned overflow above 709


def test_log_accuracy_and_specials(oracle):
    mp.mp.prec = 120
    rng = np.random.default_rng(2)
    xs = np.concatenate([np.exp(rng.uniform(-700, 700, 5000)), rng.uniform(0.5, 2.0, 5000),
                         1.0 + rng.uniform(-1e-6, 1e-6, 500), [5e-324, 1e-310, 2.0 ** -1022,
                                                             1.0 + 2**-52, 1.0 - 2**-53, 1.7976931348623157e308]])
    worst = 0.0
    for x in xs:
        worst = max(worst, ulp_error(oracle.log(x), mp.log(mp.mpf(float(x)))))
    assert worst <= 2.0, worst
    assert oracle.log(1.0) == 0.0
    assert oracle.log(2.0) == float(mp.log(2))
    assert oracle.log(0.0) == -math.inf
    assert oracle.log(math.inf) == math.inf
    assert math.isnan(oracle.log(-1.0))


def test_cos2pi_accuracy(oracle):
    mp.mp.prec = 120
    rng = np.random.default_rng(3)
    us = np.concatenate([rng.uniform(0, 1, 8000), [0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875,
                                                    2.0 ** -33, 1 - 2.0 ** -33]])
    worst = 0.0
    for u in us:
        exact = mp.cos(2 * mp.pi * mp.mpf(float(u)))
        worst = max(worst, float(abs(mp.mpf(oracle.cos2pi(u)) - exact)))
    assert worst <= 2.0 ** -52, worst
    assert oracle.cos2pi(0.25) == 0.0 or abs(oracle.cos2pi(0.25)) < 1e-300
    assert oracle.cos2pi(0.5) == -1.0


def _poisson_quantile(m, u):
    """Smallest k with CDF(k; m) >= u, in 80-digit arithmetic."""
    mp.mp.dps = 40
    p = mp.e ** (-mp.mpf(m))
    F = p
    k = 0
    while F < u and k < 20000:
        k += 1
        p = p * mp.mpf(m) / k
        F += p
    return k, F


@pytest.mark.parametrize("m", [0.01, 0.7, 3.5, 20.0, 31.9])
def test_poisson_single_chunk_is_inverse_cdf(oracle, m):
    rng = np.random.default_rng(int(m * 100))
    for w in rng.integers(0, 2**32, size=300):
        u = oracle.uniform_from_word(int(w))
        k, used = oracle.poisson_words(m, [int(w)])
        assert used == 1
        ref, _ = _poisson_quantile(m, mp.mpf(u))
        if k != ref:
            # only admissible when u sits within rounding of a CDF step
            _, F = _poisson_quantile(m, mp.mpf(u))
            mp.mp.dps = 40
            p = mp.e ** (-mp.mpf(m))
            Fk = p
            for j in range(1, min(k, ref) + 1):
                p = p * m / j
                Fk += p
            assert abs(Fk - mp.mpf(u)) < 1e-13, (m, u, k, ref)


@pytest.mark.parametrize("m", [32.5, 100.0, 777.7])
def test_poisson_chunks_sum_of_inverse_cdfs(oracle, m):
    chunks = math.ceil(m / 32.0)
    mc = m / chunks
    rng = np.random.default_rng(7)
    for _ in range(40):
        ws = [int(x) for x in rng.integers(0, 2**32, size=chunks)]
        k, used = oracle.poisson_words(m, ws)
        assert used == chunks
        ref = sum(_poisson_quantile(mc, mp.mpf(oracle.uniform_from_word(w)))[0] for w in ws)
        assert abs(k - ref) <= 1, (k, ref)


def test_poisson_caps_and_zero(oracle):
    assert oracle.poisson_words(0.0, [])[0] == 0
    assert oracle.poisson_words(1e4 + 1.0, [1, 2, 3])[0] == -1
    assert oracle.poisson_words(math.nan, [1])[0] == -1


def test_poisson_moments(oracle):
    rng = np.random.default_rng(5)
    for m in (0.3, 5.0, 70.0):
        chunks = math.ceil(m / 32)
        ks = np.array([oracle.poisson_words(m, rng.integers(0, 2**32, size=chunks))[0]
                       for _ in range(4000)])
        se = math.sqrt(m / len(ks))
        assert abs(ks.mean() - m) < 4 * se
        assert abs(ks.var() / m - 1.0) < 0.15
