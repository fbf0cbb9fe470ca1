"""Block bucketing on the GPU (smc_set_bucketing): the counting sort of
particle slots by resume block changes which lane runs which slot, never the
results. Checked round by round (log-weights, ancestors, blocks bit-exact)
against the same run without it, against the source-level oracle, inside a
captured graph, and under the autotuner."""
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


def bits(a):
    return np.asarray(a, dtype=np.float64).view(np.uint64)


def program(smc, ctx, txt, stack_words=256):
    return smc.Model(ctx, {"kind": "program", "precision": 64, "program": ppl.compile_program(txt, stack_words)})


MODELS = {
    "regime": lambda smc, ctx: program(smc, ctx, I.regime_program(I.branching_observations(8, 9), draws=4)),
    "branching": lambda smc, ctx: program(smc, ctx, I.branching_program(I.branching_observations(7, 8))),
    "geometric_program": lambda smc, ctx: program(smc, ctx, I.geometric_program(0.5, 1.2)),
    "crbd": lambda smc, ctx: smc.Model(ctx, I.crbd_spec(I.yule_tree(20, 1000), precision=64)),
    "geometric": lambda smc, ctx: smc.Model(ctx, I.geometric_spec(True, 0.5, 1.2)),
}


@pytest.mark.parametrize("name", list(MODELS))
@pytest.mark.parametrize("n", [1000, 5000])
def test_bucketing_changes_no_result(smc, ctx, name, n):
    model = MODELS[name](smc, ctx)
    a = smc.Run(model, n, 13)
    b = smc.Run(model, n, 13)
    b.set_bucketing(True)
    for r in range(400):
        say(name, n, "round", r)
        a.step()
        b.step()
        assert np.array_equal(bits(a.lw()), bits(b.lw())), (name, r)
        assert np.array_equal(a.blk(), b.blk()), (name, r)
        a.resample()
        b.resample()
        da, sa = a.done()
        db, sb = b.done()
        assert (da, sa) == (db, sb)
        if da:
            break
        assert np.array_equal(a.anc(), b.anc())
    assert da
    assert a.log_z() == b.log_z()
    a.close()
    b.close()
    model.close()


def test_bucketed_program_matches_oracle(smc, ctx, oracle):
    from oracle import ppl_oracle as PO
    txt = I.regime_program(I.branching_observations(6, 9), draws=3)
    model = program(smc, ctx, txt)
    n = 1500
    run = smc.Run(model, n, 4)
    run.set_bucketing(True)
    ref = PO.ProgramRun(txt, n, 4)
    while True:
        run.step()
        ref.step()
        assert np.array_equal(bits(run.lw()), bits(ref.lw))
        run.resample()
        ref.resample()
        done, st = run.done()
        assert st == ref.status
        if done:
            break
        assert np.array_equal(run.anc(), ref.anc)
    assert abs(run.log_z() - ref.log_z) <= 1e-9 * max(1.0, abs(ref.log_z))


def test_bucketing_inside_captured_graph(smc, ctx):
    """A lockstep run replays a captured graph after a reset; turning bucketing
    on drops the graph and the next capture includes the sort."""
    model = smc.Model(ctx, I.crbd_spec(I.yule_tree(20, 1000), precision=64))
    run = smc.Run(model, 4096, 3)
    run.run_to_end()
    plain = run.log_z()
    run.reset(3)
    run.run_to_end()  # graph captured and replayed
    assert run.log_z() == plain
    run.set_bucketing(True)
    for _ in range(3):
        run.reset(3)
        assert run.run_to_end() == smc.FINISHED
        assert run.log_z() == plain
    run.set_bucketing(False)
    run.reset(3)
    run.run_to_end()
    assert run.log_z() == plain


def test_autotuner_keeps_results(smc, ctx):
    from paper_2112_00364_amd import autotune
    model = program(smc, ctx, I.regime_program(I.branching_observations(8, 9), draws=6))
    n = 1 << 15
    ref = smc.Run(model, n, 21)
    ref.run_to_end()
    run = smc.Run(model, n, 21)
    choice = autotune.choose_bucketing(run, 21, rounds=3, repeats=1)
    say("autotuner", choice)
    assert set(choice) == {"bucketing", "ms_off", "ms_on", "rounds"}
    assert run.run_to_end() == smc.FINISHED
    assert run.log_z() == ref.log_z()


@pytest.mark.parametrize("name", ["crbd", "seir", "regime"])
def test_workgroup_size_changes_no_result(smc, ctx, name):
    """smc_set_workgroup changes the propagation's lanes per work-group (128 or
    256), never the results."""
    if name == "seir":
        model = smc.Model(ctx, I.seir_spec(I.seir_data(20, 6000), 32))
    elif name == "crbd":
        model = MODELS["crbd"](smc, ctx)
    else:
        model = MODELS["regime"](smc, ctx)
    n = 4099
    zs, lws = [], []
    for lanes in (128, 256):
        run = smc.Run(model, n, 23)
        run.set_workgroup(lanes)
        for _ in range(3):
            run.step()
            run.resample()
        lws.append(run.lw())
        run.run_to_end()
        zs.append(run.log_z())
        run.close()
    assert np.array_equal(bits(lws[0]), bits(lws[1]))
    assert zs[0] == zs[1]
    with pytest.raises(smc.SMCError):
        smc.Run(model, 64, 1).set_workgroup(96)


def test_launch_autotuner_keeps_results(smc, ctx):
    from paper_2112_00364_amd import autotune
    model = program(smc, ctx, I.regime_program(I.branching_observations(8, 9), draws=6))
    n = 1 << 15
    ref = smc.Run(model, n, 21)
    ref.run_to_end()
    run = smc.Run(model, n, 21)
    choice = autotune.choose_launch(run, 21, rounds=3, repeats=1)
    say("launch autotuner", choice)
    assert choice["lanes"] in (128, 256) and len(choice["ms"]) == 4
    assert run.run_to_end() == smc.FINISHED
    assert run.log_z() == ref.log_z()
