"""Batched runs under either propagation work-group size or owned by one
work-group (launch options):
results identical to the default size and to the runs alone; the batch
autotuner's choice is a size and its cache round-trips."""
import numpy as np
import pytest

from paper_2112_00364_amd import inputs as I

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


def _batch(smc, ctx, models, ns, lanes):
    b = smc.Batch(ctx)
    slots = [b.add(m, n, 700 + i) for i, (m, n) in enumerate(zip(models, ns))]
    for s, l in zip(slots, lanes):
        b.set_workgroup(s, l)
    for _ in range(500):
        b.tick(5)
        done, lz, st, steps = b.poll()
        if done.all():
            break
    assert done.all()
    b.close()
    return [(int(st[s]), float(lz[s]), int(steps[s])) for s in slots]


def test_batch_workgroup_sizes_give_identical_results(smc, oracle, ctx):
    specs = [I.crbd_spec(I.yule_tree(24 + 4 * i, 60 + i), precision=32) for i in range(3)]
    specs += [I.clads_spec(I.yule_tree(20 + 6 * i, 80 + i), precision=32) for i in range(2)]
    specs += [I.lgssm_spec(I.lgssm_data(30, 9), 32)]
    ns = [4096, 1000, 3000, 2048, 1500, 5000]
    models = [smc.Model(ctx, s) for s in specs]
    try:
        base = _batch(smc, ctx, models, ns, [128] * len(ns))
        wide = _batch(smc, ctx, models, ns, [256] * len(ns))
        mixed = _batch(smc, ctx, models, ns, [256, 128, 256, 128, 256, 128])
        assert base == wide == mixed
        for i, (s, n) in enumerate(zip(specs, ns)):
            ref = oracle.Run(s, n, 700 + i)
            ref.run_to_end()
            st, lz, steps = base[i]
            assert st == ref.status and steps == ref.block_steps
            assert abs(lz - ref.log_z) <= 1e-9 * abs(ref.log_z)
        b = smc.Batch(ctx)
        slot = b.add(models[0], 100, 1)
        with pytest.raises(smc.SMCError):
            b.set_workgroup(slot, 64)
        with pytest.raises(smc.SMCError):
            b.set_workgroup(slot + 5, 128)
        b.close()
    finally:
        for m in models:
            m.close()


def test_batch_autotuner_caches_its_choice(smc, ctx, tmp_path):
    from paper_2112_00364_amd import autotune as A
    spec = I.clads_spec(I.yule_tree(40, 4001), precision=32)
    model = smc.Model(ctx, spec)
    try:
        cache = A.LaunchCache(str(tmp_path / "launch.json"))
        lanes = A.batch_workgroup(cache, ctx, model, "clads", 32, 4096, 40, probe_runs=4)
        assert lanes in (128, 256)
        key = A.shape_key("clads", 32, 4096, 40)
        again = A.LaunchCache(str(tmp_path / "launch.json"))
        assert again.get(key)["lanes"] == lanes
        # 4096 particles: owning by a work-group is a candidate too
        assert set(again.get(key)["ms"]) == {"lanes128", "lanes256", "owned"}
        choice = A.batch_launch(again, ctx, model, "clads", 32, 4096, 40)
        assert choice["lanes"] == lanes and choice["owned"] == again.get(key)["owned"]
    finally:
        model.close()


# --- runs owned by one work-group --------------------------------------------------------------

def _owned_batch(smc, ctx, models, ns, owned, rounds=5, toggle_after=None):
    b = smc.Batch(ctx)
    slots = [b.add(m, n, 900 + i) for i, (m, n) in enumerate(zip(models, ns))]
    for s, o in zip(slots, owned):
        b.set_owned(s, o)
    for tick in range(2000):
        b.tick(rounds)
        if toggle_after is not None and tick + 1 == toggle_after:
            for s, o in zip(slots, owned):
                b.set_owned(s, not o)  # switch paths between two ticks
        done, lz, st, steps = b.poll()
        if done.all():
            break
    assert done.all()
    b.close()
    return [(int(st[s]), float(lz[s]), int(steps[s])) for s in slots]


def _owned_workload(smc, ctx):
    specs = [I.geometric_spec(), I.lgssm_spec(I.lgssm_data(40, 3), 32),
             I.crbd_spec(I.yule_tree(30, 61), precision=32), I.crbd_spec(I.yule_tree(50, 62), precision=64),
             I.clads_spec(I.yule_tree(24, 81), precision=32), I.seir_spec(I.seir_data(12, 6001), 32),
             dict(I.crbd_ds_spec(I.yule_tree(28, 63), precision=32), ess_threshold=0.5)]
    ns = [1, 777, 1024, 4096, 300, 500, 2000]
    return specs, ns, [smc.Model(ctx, s) for s in specs]


def test_owned_runs_match_runs_alone(smc, oracle, ctx):
    """Every built-in model, sizes from 1 to 4096 particles (ragged tiles), ESS
    resampling: owned, segmented and mixed batches, and a batch whose runs
    switch paths between ticks, all give each run's results alone, bit for bit."""
    specs, ns, models = _owned_workload(smc, ctx)
    try:
        alone = []
        for i, (m, n) in enumerate(zip(models, ns)):
            r = smc.Run(m, n, 900 + i)
            st = r.run_to_end()
            s = r.stats()
            alone.append((int(st), float(s["log_z"]), int(s["block_steps"])))
            r.close()
        k = len(ns)
        owned = _owned_batch(smc, ctx, models, ns, [True] * k)
        mixed = _owned_batch(smc, ctx, models, ns, [i % 2 == 0 for i in range(k)], rounds=3)
        switched = _owned_batch(smc, ctx, models, ns, [True] * k, rounds=4, toggle_after=2)
        assert owned == alone
        assert mixed == alone
        assert switched == alone
        for i in (2, 4):  # CRBD and ClaDS owned runs against the oracle too
            ref = oracle.Run(specs[i], ns[i], 900 + i)
            ref.run_to_end()
            st, lz, steps = owned[i]
            assert st == ref.status and steps == ref.block_steps
            assert abs(lz - ref.log_z) <= 1e-9 * abs(ref.log_z)
    finally:
        for m in models:
            m.close()


def test_owned_run_limits(smc, ctx):
    from paper_2112_00364_amd import ppl
    crbd = smc.Model(ctx, I.crbd_spec(I.yule_tree(20, 64), precision=32))
    img = ppl.compile_program(I.lgssm_program(I.lgssm_data(8, 2000)), 256)
    prog = smc.Model(ctx, {"kind": "program", "precision": 64, "program": img})
    try:
        b = smc.Batch(ctx)
        big = b.add(crbd, 4097, 1)
        small_prog = b.add(prog, 64, 2)
        with pytest.raises(smc.SMCError):
            b.set_owned(big)
        with pytest.raises(smc.SMCError):
            b.set_owned(small_prog)
        with pytest.raises(smc.SMCError):
            b.set_owned(small_prog + 7)
        b.set_owned(big, False)  # leaving a run segmented is always allowed
        b.close()
    finally:
        crbd.close()
        prog.close()
