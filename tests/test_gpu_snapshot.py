"""Checkpoint and resume (smc_snapshot / smc_restore) on the GPU: a run
restored from a snapshot finishes exactly as the uninterrupted run does."""
import sys

import numpy as np
import pytest

from paper_2112_00364_amd import inputs as I
from paper_2112_00364_amd import ppl

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


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


def finish(run, smc, limit=10000):
    for _ in range(limit):
        done, st = run.done()
        if done:
            return st
        run.step()
        run.resample()
    raise AssertionError("run did not finish")


def rounds(run, k):
    for _ in range(k):
        run.step()
        run.resample()


MODELS = {
    "crbd": lambda smc, ctx: smc.Model(ctx, I.crbd_spec(I.yule_tree(40, 1001), precision=32)),
    "clads": lambda smc, ctx: smc.Model(ctx, I.clads_spec(I.yule_tree(24, 1002), precision=32)),
    "program": lambda smc, ctx: smc.Model(ctx, {"kind": "program", "precision": 64, "program":
                                              ppl.compile_program(I.branching_program(I.branching_observations(9, 8)))}),
}


@pytest.mark.parametrize("name", list(MODELS))
def test_resume_from_snapshot_finishes_identically(smc, ctx, name):
    model = MODELS[name](smc, ctx)
    n = 5000
    a = smc.Run(model, n, 17)
    rounds(a, 5)
    say(name, "snapshot after 5 rounds")
    snap = a.snapshot()
    lw = a.lw()
    assert finish(a, smc) == smc.FINISHED
    want = a.log_z()
    b = smc.Run(model, n, 99)  # another seed: the snapshot carries the run's key
    b.restore(snap)
    assert np.array_equal(b.lw(), lw)
    assert finish(b, smc) == smc.FINISHED
    assert b.log_z() == want
    a.close()
    b.close()
    model.close()


def test_snapshot_between_step_and_resample(smc, ctx):
    model = MODELS["program"](smc, ctx)
    a = smc.Run(model, 3000, 5)
    rounds(a, 2)
    a.step()  # the resampling of this round is still due
    snap = a.snapshot()
    a.resample()
    finish(a, smc)
    b = smc.Run(model, 3000, 5)
    b.restore(snap)
    with pytest.raises(smc.SMCError):
        b.step()  # Algorithm 1's alternation is part of the state
    b.resample()
    finish(b, smc)
    assert b.log_z() == a.log_z()


def test_snapshot_of_a_finished_run_and_shape_checks(smc, ctx):
    model = MODELS["crbd"](smc, ctx)
    a = smc.Run(model, 2048, 3)
    assert finish(a, smc) == smc.FINISHED
    snap = a.snapshot()
    b = smc.Run(model, 2048, 4)
    b.restore(snap)
    assert b.done() == (True, smc.FINISHED)
    assert b.log_z() == a.log_z()
    c = smc.Run(model, 2047, 3)
    with pytest.raises(smc.SMCError) as e:
        c.restore(snap)
    assert e.value.code == smc.ERR_INVALID
    other = MODELS["clads"](smc, ctx)
    d = smc.Run(other, 2048, 3)
    with pytest.raises(smc.SMCError):
        d.restore(snap)
    with pytest.raises(smc.SMCError):
        d.restore(b"not a snapshot")
