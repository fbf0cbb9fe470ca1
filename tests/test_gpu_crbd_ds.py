"""GPU parity for CRBD with static delayed sampling (Sec. 5.3's CRBD with
variance-reducing techniques): the Negative Binomial and Lomax predictive
samplers bit for bit, and whole runs round by round (blocks, log-weights,
posterior shapes and scales, ancestors, log Z) in FP64 and FP32, with the ESS
rule, through the deep-stack recomputation, graph replay and a batch.
"""
import numpy as np
import pytest

from paper_2112_00364_amd import inputs as I
from test_gpu_parity import LOGZ_RTOL, bits, run_lockstep, say

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


@pytest.mark.parametrize("kind,op", [("negbin", 11), ("lomax", 12)])
def test_predictive_samplers_bit_identical(ctx, oracle, kind, op):
    rng = np.random.default_rng(op)
    rows = [[float(rng.integers(1, 60)), float(10 ** rng.uniform(-3, 1.5)), float(rng.integers(0, 2 ** 52))]
            for _ in range(4000)]
    got = ctx.selftest_math(op, np.array(rows).reshape(-1))
    ref = np.array([oracle.sample(kind, a, th, int(s), 1)[0] for a, th, s in rows])
    assert np.array_equal(bits(got), bits(ref))


def test_crbd_ds_runs_match(smc, oracle, ctx):
    say("crbd_ds 20 tips fp64")
    run_lockstep(smc, oracle, ctx, I.crbd_ds_spec(I.yule_tree(20, 1000), precision=64), 1000, 1)
    say("crbd_ds 48 tips fp32 ragged")
    run_lockstep(smc, oracle, ctx, I.crbd_ds_spec(I.yule_tree(48, 9), precision=32), 3001, 2, check_every=4)
    say("crbd_ds with ESS rule")
    run_lockstep(smc, oracle, ctx, dict(I.crbd_ds_spec(I.yule_tree(40, 12), precision=32), ess_threshold=0.5),
                 4096, 3, check_every=3)


def test_crbd_ds_deep_recursion_matches(smc, oracle, ctx):
    """Large prior scales make hidden lineages recurse deeply, so particles
    take the LDS-stack recomputation."""
    say("crbd_ds deep")
    spec = I.crbd_ds_spec(I.yule_tree(16, 5), precision=64, scale_lambda=10.0, scale_mu=10.0)
    run_lockstep(smc, oracle, ctx, spec, 2000, 7)


def test_crbd_ds_run_to_end_and_batch(smc, oracle, ctx):
    specs = [I.crbd_ds_spec(I.yule_tree(30, 91), precision=32), I.crbd_spec(I.yule_tree(25, 92), precision=32),
             dict(I.crbd_ds_spec(I.yule_tree(22, 93), precision=64), ess_threshold=0.7)]
    ns = [3000, 2048, 1025]
    refs = []
    for i, (s, n) in enumerate(zip(specs, ns)):
        r = oracle.Run(s, n, 400 + i)
        r.run_to_end()
        refs.append(r)
    model = smc.Model(ctx, specs[0])
    run = smc.Run(model, ns[0], 1)
    for _ in range(2):
        run.reset(400)
        assert run.run_to_end() == refs[0].status
        st = run.stats()
        assert st["block_steps"] == refs[0].block_steps
        assert abs(st["log_z"] - refs[0].log_z) <= LOGZ_RTOL * abs(refs[0].log_z)
    run.close()
    model.close()
    models = [smc.Model(ctx, s) for s in specs]
    b = smc.Batch(ctx)
    slots = [b.add(m, n, 400 + i) for i, (m, n) in enumerate(zip(models, ns))]
    for _ in range(100):
        b.tick(4)
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


def test_crbd_ds_invalid_scales_rejected(smc, ctx):
    with pytest.raises(smc.SMCError):
        smc.Model(ctx, I.crbd_ds_spec(I.yule_tree(8, 1), scale_lambda=0.0))
