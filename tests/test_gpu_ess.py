"""GPU parity for ESS-triggered resampling (a model's ess_threshold > 0).

Each round's resampling decision, the carried log-weights, the identity
ancestors of rounds that keep their weights, the gathered state and log Z are
compared with the oracle, on the single-run path (work-groups fold the
partials themselves), the large-run path (one-work-group fold kernels), the
graph replay of smc_run_to_end and the batch API.
"""
import math

import numpy as np
import pytest

from paper_2112_00364_amd import inputs as I
from test_gpu_parity import LOGZ_RTOL, run_lockstep, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def smc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2112_00364_amd import smc as S
    S.lib()
    return S


@pytest.fixture(scope="module")
def ctx(smc):
    c = smc.Context(0)
    yield c
    c.close()


def ess(spec, tau):
    return dict(spec, ess_threshold=tau)


def test_geometric_with_ess_rule_matches(smc, oracle, ctx):
    for tau, n in ((0.5, 1000), (1.0 / 65536, 777), (1.0, 513)):
        say("geometric ess", tau, n)
        run_lockstep(smc, oracle, ctx, ess(I.geometric_spec(True), tau), n, 3)


def test_lgssm_with_ess_rule_matches(smc, oracle, ctx):
    y = I.lgssm_data(100, 2000)
    say("lgssm ess T=100 N=65536")
    _, ref = run_lockstep(smc, oracle, ctx, ess(I.lgssm_spec(y, 32), 0.5), 1 << 16, 1, check_every=3)
    assert 0 < ref.resamples < ref.round


def test_crbd_and_clads_with_ess_rule_match(smc, oracle, ctx):
    say("crbd ess 20 tips")
    run_lockstep(smc, oracle, ctx, ess(I.crbd_spec(I.yule_tree(20, 1000), precision=64), 0.5), 1000, 1)
    say("crbd ess fp32 48 tips ragged")
    run_lockstep(smc, oracle, ctx, ess(I.crbd_spec(I.yule_tree(48, 9), precision=32), 0.75), 3001, 2,
                 check_every=5)
    say("clads ess")
    run_lockstep(smc, oracle, ctx, ess(I.clads_spec(I.yule_tree(24, 71), precision=32), 0.5), 2048, 5,
                 check_every=3)


def test_large_run_fold_path_with_ess_rule(smc, oracle, ctx):
    y = I.lgssm_data(6, 31)
    say("lgssm ess N=2^20+4097")
    run_lockstep(smc, oracle, ctx, ess(I.lgssm_spec(y, 32), 0.9), (1 << 20) + 4097, 12, check_every=2)


def test_run_to_end_and_batch_with_ess_rule(smc, oracle, ctx):
    specs = [ess(I.crbd_spec(I.yule_tree(30, 77), precision=32), 0.5),
             ess(I.clads_spec(I.yule_tree(20, 78), precision=32), 0.6),
             ess(I.lgssm_spec(I.lgssm_data(40, 79), 32), 0.5)]
    ns = [3000, 2048, 4097]
    refs = []
    for i, (s, n) in enumerate(zip(specs, ns)):
        r = oracle.Run(s, n, 200 + i)
        r.run_to_end()
        refs.append(r)
    # graph replay after a reset, twice, then an eager run
    for i, (s, n) in enumerate(zip(specs, ns)):
        model = smc.Model(ctx, s)
        run = smc.Run(model, n, 1)
        for _ in range(2):
            run.reset(200 + i)
            assert run.run_to_end() == smc.FINISHED
            st = run.stats()
            say("run_to_end ess", i, st["resamples"], refs[i].resamples)
            assert st["resamples"] == refs[i].resamples and st["block_steps"] == refs[i].block_steps
            assert abs(st["log_z"] - refs[i].log_z) <= LOGZ_RTOL * abs(refs[i].log_z)
        run.close()
        model.close()
    # the same runs advanced together
    models = [smc.Model(ctx, s) for s in specs]
    b = smc.Batch(ctx)
    slots = [b.add(m, n, 200 + i) for i, (m, n) in enumerate(zip(models, ns))]
    for _ in range(200):
        b.tick(3)
        done, lz, st, steps = b.poll()
        if done.all():
            break
    assert done.all()
    for i, ref in enumerate(refs):
        assert st[slots[i]] == ref.status and steps[slots[i]] == ref.block_steps
        assert abs(lz[slots[i]] - ref.log_z) <= LOGZ_RTOL * abs(ref.log_z), (i, lz[slots[i]], ref.log_z)
    for s in slots:
        b.retire(s)
    b.close()
    for m in models:
        m.close()


def test_invalid_threshold_rejected(smc, ctx):
    with pytest.raises(smc.SMCError):
        smc.Model(ctx, ess(I.geometric_spec(True), 1.5))
