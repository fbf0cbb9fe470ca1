"""Batched runs under either propagation work-group size (a launch option):
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
        assert set(again.get(key)["ms"]) == {"lanes128", "lanes256"}
    finally:
        model.close()
