"""Pins of the source-level program oracle (oracle/ppl_oracle.py).

The oracle runs Algorithm 1 over direct executions of a program's source.
What fixes it from outside itself:
* the weighted geometric program (Sec. 2, Fig. 2) and the state-space model
  of eq. (2) written as recursive programs give, bit for bit, the log Z,
  log-weights and ancestors of the C oracle's built-in models (themselves
  pinned to closed forms and the Kalman filter);
* a two-state hidden Markov model: the estimate is unbiased for the evidence
  computed by the forward algorithm, and converges to it;
* observation log-densities agree with scipy;
* faults (a data index out of range, an invalid sampler argument) give weight
  -inf and stop the particle.
"""
import math

import numpy as np
import pytest

from paper_2112_00364_amd import inputs as I


@pytest.fixture(scope="module")
def PO(oracle):
    from oracle import ppl_oracle
    return ppl_oracle


@pytest.mark.parametrize("n,seed", [(1, 0), (7, 1), (64, 2), (300, 3)])
def test_geometric_program_is_the_builtin_model(oracle, PO, n, seed):
    a = PO.ProgramRun(I.geometric_program(0.5, 1.2), n, seed)
    b = oracle.Run(I.geometric_spec(True, 0.5, 1.2), n, seed)
    while True:
        a.step()
        b.step()
        assert np.array_equal(a.lw, b.lw())
        sa, sb = a.resample(), b.resample()
        assert sa == sb
        if sa != oracle.OK:
            break
        assert np.array_equal(a.anc, b.anc())
    assert a.log_z == b.log_z and a.round == b.round


@pytest.mark.parametrize("seed", [0, 5])
def test_lgssm_program_is_the_builtin_model(oracle, PO, seed):
    y = I.lgssm_data(25, 2000)
    a = PO.ProgramRun(I.lgssm_program(y), 200, seed)
    b = oracle.Run(I.lgssm_spec(y, 64), 200, seed)
    while True:
        a.step()
        b.step()
        assert np.array_equal(a.lw, b.lw())
        sa, sb = a.resample(), b.resample()
        assert sa == sb
        if sa != oracle.OK:
            break
        assert np.array_equal(a.anc, b.anc())
    assert a.log_z == b.log_z


def hmm_log_evidence(ys, p0=0.5, flip=0.2, emit=(0.1, 0.9)):
    """Forward algorithm for the two-state model of hmm_program."""
    alpha = np.array([1.0 - p0, p0])
    T = np.array([[1.0 - flip, flip], [flip, 1.0 - flip]])
    logz = 0.0
    for y in ys:
        alpha = alpha @ T
        like = np.array([emit[0] if y == 1.0 else 1.0 - emit[0], emit[1] if y == 1.0 else 1.0 - emit[1]])
        alpha = alpha * like
        s = alpha.sum()
        logz += math.log(s)
        alpha /= s
    return logz


def test_forward_algorithm_against_enumeration():
    """The test's own reference, checked by brute force over all state paths."""
    ys = [1.0, 0.0, 1.0]
    total = 0.0
    for s0 in (0, 1):
        for path in range(8):
            states = [(path >> i) & 1 for i in range(3)]
            pr = 0.5
            prev = s0
            for t, s in enumerate(states):
                pr *= 0.2 if s != prev else 0.8
                e = 0.9 if s == 1 else 0.1
                pr *= e if ys[t] == 1.0 else 1.0 - e
                prev = s
            total += pr
    assert abs(math.log(total) - hmm_log_evidence(ys)) < 1e-12


@pytest.mark.slow
def test_hmm_program_unbiased(PO):
    ys = [1.0, 0.0, 1.0, 1.0, 0.0]
    Z = math.exp(hmm_log_evidence(ys))
    ratios = []
    txt = I.hmm_program(ys)
    for seed in range(3000):
        r = PO.ProgramRun(txt, 2, seed)
        r.run_to_end()
        ratios.append(math.exp(r.log_z) / Z)
    ratios = np.array(ratios)
    se = ratios.std(ddof=1) / math.sqrt(len(ratios))
    assert abs(ratios.mean() - 1.0) <= 4 * se, (ratios.mean(), se)


def test_hmm_program_converges(PO):
    ys = I.hmm_observations(12, 7)
    exact = hmm_log_evidence(ys)
    r = PO.ProgramRun(I.hmm_program(ys), 2000, 11)
    r.run_to_end()
    assert abs(r.log_z - exact) < 0.15, (r.log_z, exact)


def test_observation_densities_against_scipy(PO):
    from scipy import stats
    cases = [
        ("normal", [0.3, 1.7], [-2.0, 0.3, 4.1]),
        ("uniform", [-1.0, 2.5], [-1.0, 0.0, 2.5]),
        ("exponential", [1.7], [0.0, 0.4, 3.0]),
        ("bernoulli", [0.3], [0.0, 1.0]),
        ("poisson", [2.5], [0.0, 1.0, 7.0, 30.0]),
        ("binomial", [12.0, 0.35], [0.0, 5.0, 12.0]),
    ]
    ref = {
        "normal": lambda a, v: stats.norm.logpdf(v, a[0], a[1]),
        "uniform": lambda a, v: stats.uniform.logpdf(v, a[0], a[1] - a[0]),
        "exponential": lambda a, v: stats.expon.logpdf(v, scale=1.0 / a[0]),
        "bernoulli": lambda a, v: stats.bernoulli.logpmf(v, a[0]),
        "poisson": lambda a, v: stats.poisson.logpmf(v, a[0]),
        "binomial": lambda a, v: stats.binom.logpmf(v, int(a[0]), a[1]),
    }
    for dist, args, vals in cases:
        for v in vals:
            got = PO.observe_logpdf(dist, args, v)
            want = float(ref[dist](args, v))
            assert abs(got - want) <= 1e-12 * max(1.0, abs(want)), (dist, args, v, got, want)
    # outside the support
    assert PO.observe_logpdf("poisson", [2.0], 1.5) == -math.inf
    assert PO.observe_logpdf("binomial", [3.0, 0.5], 4.0) == -math.inf
    assert PO.observe_logpdf("exponential", [1.0], -0.1) == -math.inf
    with pytest.raises(PO.Fault):
        PO.observe_logpdf("normal", [0.0, 0.0], 1.0)


def test_faults_stop_the_particle(oracle, PO):
    txt = """(program (data d 1 2 3)
      (def main () (sample u uniform 0 4) (let v (at d (floor u))) (resample) (return v)))"""
    r = PO.ProgramRun(txt, 200, 3)
    r.step()
    lw = r.lw.copy()
    assert np.isneginf(lw).any() and np.isfinite(lw).any()  # floor(u) = 3 is out of range
    assert r.stopped()[np.isneginf(lw)].all()
    txt = "(program (def main () (sample g gamma 0.5 1) (return g)))"
    r = PO.ProgramRun(txt, 4, 0)
    r.step()
    assert np.isneginf(r.lw).all()
    assert r.resample() == oracle.DEGENERATE


SMALL_TREE = ((((0.0, 0.0, 0.21), 0.0, 0.55), ((0.0, 0.0, 0.33), 0.0, 0.62), 1.0))


def test_crbd_program_unbiased_for_closed_form(oracle, PO):
    """The Appendix CRBD model compiled from source (fixed rates): the
    estimate is unbiased for the closed-form tree likelihood, as for the
    built-in model."""
    import analytic as A
    tree = I.tree_from_newick_like(SMALL_TREE)
    lam, mu = 1.5, 0.8
    L = math.exp(A.crbd_log_lik(tree, lam, mu))
    txt = I.crbd_program(tree, fixed=(lam, mu))
    ratios = []
    for s in range(3000):
        r = PO.ProgramRun(txt, 4, s)
        st = r.run_to_end()
        ratios.append(math.exp(r.log_z) / L if st == oracle.FINISHED else 0.0)
    ratios = np.array(ratios)
    se = ratios.std(ddof=1) / math.sqrt(len(ratios))
    assert abs(ratios.mean() - 1.0) <= 4 * se, (ratios.mean(), se)


@pytest.mark.parametrize("seed", [1, 4])
def test_seir_program_is_the_builtin_model(oracle, PO, seed):
    """The Appendix vector-borne disease model written as a program equals the
    C oracle's built-in SEIR model (FP64 state) bit for bit."""
    y = I.seir_data(10, 6000)
    a = PO.ProgramRun(I.seir_program(y), 96, seed)
    b = oracle.Run(I.seir_spec(y, 64), 96, seed)
    while True:
        a.step()
        b.step()
        assert np.array_equal(a.lw.view(np.uint64), b.lw().view(np.uint64))
        sa, sb = a.resample(), b.resample()
        assert sa == sb
        if sa != oracle.OK:
            break
        assert np.array_equal(a.anc, b.anc())
    assert a.log_z == b.log_z
