"""GPU parity at the full configurations: the headline CRBD run (256-tip Yule
tree, 2^20 particles, 511 rounds) compared with the oracle on every particle in
every round, and the batched ClaDS workload (512 runs of 4096 particles) at its
full shape (Algorithm 1, Sec. 3.2; the engine's loop, Sec. 3.3).

Bar: block indices, ancestors and FP32 state bit-exact, FP64 log-weights
bit-exact, log Z within 1e-9 relative, block-step counts exact.
"""
import math
import multiprocessing as mp
import sys

import numpy as np
import pytest

from paper_2112_00364_amd import inputs as I

pytestmark = pytest.mark.gpu

LOGZ_RTOL = 1e-9


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


def u32(a):
    return np.ascontiguousarray(a).view(np.uint32)


def u64(a):
    return np.ascontiguousarray(a, dtype=np.float64).view(np.uint64)


def test_crbd_headline_every_round_every_particle(smc, oracle, ctx):
    """2^20 particles on the 256-tip tree (seed 3000), FP32 state: all 511
    rounds stepped in lockstep with the oracle, every particle compared after
    each propagation (blocks, log-weight bits, lambda/mu bits) and after each
    resampling (ancestors, gathered state); final log Z and block steps. Then
    the launch configuration the benchmark times (reset + run_to_end, replayed
    from a captured graph) on the same seed gives the same log Z bits and final
    state as the lockstep run."""
    n = 1 << 20
    tree = I.yule_tree(256, 3000)
    spec = I.crbd_spec(tree, precision=32)
    model = smc.Model(ctx, spec)
    gpu = smc.Run(model, n, 1)
    ref = oracle.Run(spec, n, 1)
    say("crbd headline lockstep", n)
    rnd = 0
    try:
        while True:
            gpu.step()
            ref.step()
            assert np.array_equal(gpu.blk(), ref.blk()), f"blocks round {rnd}"
            assert np.array_equal(u64(gpu.lw()), u64(ref.lw())), f"log-weights round {rnd}"
            for k in (0, 1):
                assert np.array_equal(u32(gpu.field(k, np.float32)), u32(ref.field(k, np.float32))), (rnd, k)
            st_ref = ref.resample()
            gpu.resample()
            done, st = gpu.done()
            assert st == st_ref, (rnd, st, st_ref)
            if st_ref != oracle.OK:
                break
            assert np.array_equal(gpu.anc(), ref.anc()), f"ancestors round {rnd}"
            for k in (0, 1):
                assert np.array_equal(u32(gpu.field(k, np.float32)), u32(ref.field(k, np.float32))), (rnd, k)
            if rnd % 64 == 0:
                say("  round", rnd)
            rnd += 1
            assert rnd < 600
        assert rnd == 510 and st_ref == oracle.FINISHED
        lz, lz_ref = gpu.log_z(), ref.log_z
        assert math.isfinite(lz_ref)
        assert abs(lz - lz_ref) <= LOGZ_RTOL * abs(lz_ref), (lz, lz_ref)
        s = gpu.stats()
        assert s["block_steps"] == ref.block_steps == n * 511
        lam_ref, mu_ref = ref.field(0, np.float32), ref.field(1, np.float32)
        blk_ref = ref.blk()
    finally:
        gpu.close()
        del ref

    say("crbd headline, graph-replayed run_to_end")
    timed = smc.Run(model, n, 77)
    try:
        timed.run_to_end()        # first use: launched directly
        timed.reset(1)
        assert timed.run_to_end() == smc.FINISHED  # replayed from the captured graph
        t = timed.stats()
        assert t["log_z"] == lz, (t["log_z"], lz)
        assert t["block_steps"] == n * 511
        assert np.array_equal(u32(timed.field(0, np.float32)), u32(lam_ref))
        assert np.array_equal(u32(timed.field(1, np.float32)), u32(mu_ref))
        assert np.array_equal(timed.blk(), blk_ref)
    finally:
        timed.close()
        model.close()


# --- the batched ClaDS workload at full shape ----------------------------------------------

RUNS, N_RUN = 512, 4096


def clads_batch_tips():
    return np.random.default_rng(4000).integers(32, 129, size=RUNS)


def _oracle_clads(job):
    """One run of the batch on the oracle (worker process: no GPU)."""
    r, tips = job
    from oracle import oracle as O
    run = O.Run(I.clads_spec(I.yule_tree(tips, 4000 + r), precision=32), N_RUN, 40000 + r)
    st = run.run_to_end()
    return r, st, run.log_z, run.block_steps


def _run_batch(smc, ctx, models, order, rounds_per_tick):
    b = smc.Batch(ctx)
    slot = {}
    for r in order:
        slot[r] = b.add(models[r], N_RUN, 40000 + r)
    for _ in range(10000):
        b.tick(rounds_per_tick)
        done, lz, st, steps = b.poll()
        if done.all():
            break
    assert done.all()
    out = {r: (int(st[s]), float(lz[s]), int(steps[s])) for r, s in slot.items()}
    b.close()
    return out


def test_clads_batch_full_shape(smc, oracle, ctx):
    """512 ClaDS runs (trees of 32-128 tips, seeds 4000 + r; run seeds
    40000 + r), 4096 particles each, in one batch advanced 16 rounds per tick
    as the benchmark does. Runs 0-47 against the oracle (status, log Z, block
    steps; 16 oracle processes); every run against the same batch built in the
    reverse order and advanced 7 rounds per tick (results depend on neither);
    a sample of 24 runs against the run executed alone."""
    tips = clads_batch_tips()
    n_ref = 48
    say("clads batch: oracle runs 0-47 in worker processes")
    with mp.get_context("spawn").Pool(16) as pool:
        async_ref = pool.map_async(_oracle_clads, [(r, int(tips[r])) for r in range(n_ref)], chunksize=1)
        models = [smc.Model(ctx, I.clads_spec(I.yule_tree(int(t), 4000 + r), precision=32))
                  for r, t in enumerate(tips)]
        try:
            say("clads batch 512 x 4096, 16 rounds per tick")
            first = _run_batch(smc, ctx, models, list(range(RUNS)), 16)
            say("clads batch again, reverse order, 7 rounds per tick")
            second = _run_batch(smc, ctx, models, list(reversed(range(RUNS))), 7)
            for r in range(RUNS):
                assert first[r] == second[r], (r, first[r], second[r])
            finished = sum(1 for r in range(RUNS) if first[r][0] == smc.FINISHED)
            assert finished >= RUNS * 9 // 10, finished
            rng = np.random.default_rng(11)
            for r in sorted(rng.choice(np.arange(n_ref, RUNS), size=24, replace=False)):
                alone = smc.Run(models[r], N_RUN, 40000 + int(r))
                st = alone.run_to_end()
                s = alone.stats()
                alone.close()
                assert (st, s["log_z"], s["block_steps"]) == first[r], (r, st, s, first[r])
            say("clads batch: waiting for the oracle")
            refs = async_ref.get(timeout=900)
        finally:
            for m in models:
                m.close()
    for r, st_ref, lz_ref, steps_ref in refs:
        st, lz, steps = first[r]
        assert st == st_ref, (r, st, st_ref)
        if math.isfinite(lz_ref):
            assert abs(lz - lz_ref) <= LOGZ_RTOL * abs(lz_ref), (r, lz, lz_ref)
        else:
            assert lz == lz_ref
        assert steps == steps_ref, (r, steps, steps_ref)
