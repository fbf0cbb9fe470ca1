"""GPU parity: the HIP path (through the C interface) against the CPU oracle.

Bar: ancestors, block indices and integer state bit-exact; log Z within 1e-9
relative; FP64 log-weights and FP32/FP64 state bit-exact as well (both sides
run the same pinned arithmetic), with the stated tolerances as the pass line.
"""
import math
import sys

import numpy as np
import pytest

from paper_2112_00364_amd import inputs as I

pytestmark = pytest.mark.gpu

LOGZ_RTOL = 1e-9
STATE_RTOL = 1e-5


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


# --- primitives -----------------------------------------------------------------------------

def test_philox_device_matches_oracle(ctx, oracle):
    rng = np.random.default_rng(1)
    n = 4096
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(n, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    key[0] = 0
    say("philox", n)
    out = ctx.selftest_philox(ctr, key)
    for i in range(0, n, 7):
        assert list(out[i]) == list(oracle.philox(ctr[i], key[i]))


def _edge_inputs():
    return [0.0, -0.0, 1.0, -1.0, 0.5, 2.0, 1e-300, 5e-324, 2.0 ** -1022, 708.9, -707.9, -708.5, 709.5,
            math.inf, -math.inf, 1.0 + 2 ** -52, 1.0 - 2 ** -53]


@pytest.mark.parametrize("op", ["exp", "log", "cos2pi", "sqrt", "uniform", "exp/vreg", "log/vreg", "cos2pi/vreg"])
def test_elementary_functions_bit_identical(ctx, oracle, op):
    # "/vreg": the same function with compiler-placed coefficients (ClaDS)
    code = {"exp": 0, "log": 1, "cos2pi": 2, "sqrt": 3, "uniform": 4, "exp/vreg": 13, "log/vreg": 14,
            "cos2pi/vreg": 15}[op]
    op = op.split("/")[0]
    rng = np.random.default_rng(sum(map(ord, op)))
    n = 1 << 16
    if op == "exp":
        x = np.concatenate([rng.uniform(-708, 709, n), rng.uniform(-40, 0, n), _edge_inputs()])
        ref = [oracle.exp(v) for v in x]
    elif op == "log":
        x = np.concatenate([np.exp(rng.uniform(-700, 700, n)), rng.uniform(0, 2, n), _edge_inputs()])
        ref = [oracle.log(v) for v in x]
    elif op == "cos2pi":
        w = rng.integers(0, 2**32, size=2 * n)
        x = np.array([oracle.uniform_from_word(int(v)) for v in w] + [0.125, 0.25, 0.5, 0.75, 0.0, 1.0])
        ref = [oracle.cos2pi(v) for v in x]
    elif op == "sqrt":
        x = np.concatenate([np.exp(rng.uniform(-700, 700, n)), rng.uniform(0, 4, n), [0.0, 1.0, 2.0, 5e-324]])
        ref = [math.sqrt(v) for v in x]
    else:
        x = np.concatenate([rng.integers(0, 2**32, size=n).astype(np.float64), [0.0, 2.0**32 - 1]])
        ref = [oracle.uniform_from_word(int(v)) for v in x]
    say("selftest", op, code, len(x))
    got = ctx.selftest_math(code, x)
    ref = np.array(ref)
    same = (bits(got) == bits(ref)) | (np.isnan(got) & np.isnan(ref))
    assert same.all(), (op, x[~same][:5], got[~same][:5], ref[~same][:5])


def test_normal_and_poisson_bit_identical(ctx, oracle):
    rng = np.random.default_rng(3)
    n = 1 << 14
    w = rng.integers(0, 2**32, size=(n, 2)).astype(np.float64)
    say("selftest normal", n)
    got = ctx.selftest_math(5, w.reshape(-1))
    ref = np.array([math.sqrt(-2.0 * oracle.log(oracle.uniform_from_word(int(a)))) *
                    oracle.cos2pi(oracle.uniform_from_word(int(b))) for a, b in w])
    assert np.array_equal(bits(got), bits(ref))
    means = np.concatenate([rng.uniform(0, 5, 2000), rng.uniform(5, 200, 200), [0.0, 31.99, 32.0, 32.01, 1e4 + 1]])
    seeds = rng.integers(0, 2**52, size=len(means)).astype(np.float64)
    pairs = np.stack([means, seeds], axis=1).reshape(-1)
    say("selftest poisson", len(means))
    got = ctx.selftest_math(6, pairs)
    for i, (m, sd) in enumerate(zip(means, seeds)):
        chunks = max(1, math.ceil(m / 32.0))
        words = [oracle.word(int(sd), k, i, 0, 0) for k in range(chunks)]
        k, _ = oracle.poisson_words(m, words)
        assert got[i] == k, (m, got[i], k)


# --- resampling alone -------------------------------------------------------------------------

def _weights(kind, n, rng):
    if kind == "normal":
        return rng.normal(0, 3, n) - 50.0
    if kind == "wide":
        lw = rng.normal(0, 30, n)
        lw[rng.random(n) < 0.3] = -np.inf
        lw[rng.integers(n)] = 5.0
        return lw
    if kind == "equal":
        return np.full(n, 1.25)
    if kind == "single":
        lw = np.full(n, -np.inf)
        lw[rng.integers(n)] = -3.0
        return lw
    if kind == "tiny":  # most weights below half a grid unit
        lw = rng.uniform(-60, 0, n)
        return lw
    raise ValueError(kind)


# above 2^20 the tile sums go through the fold kernel: 1025 tiles (one tile past the
# fused path) and 3085 tiles (six full rows of 512 and a ragged seventh)
@pytest.mark.parametrize("n", [1, 2, 3, 1000, 1023, 1024, 1025, 4096 + 17, 65536, 1 << 20, (1 << 20) + 1,
                               3 * (1 << 20) + 12345])
@pytest.mark.parametrize("kind", ["normal", "wide", "equal", "single", "tiny"])
def test_resample_weights_matches_oracle(ctx, oracle, n, kind):
    rng = np.random.default_rng(n * 31 + len(kind))
    lw = _weights(kind, n, rng)
    seed, rnd = int(rng.integers(1 << 62)), int(rng.integers(1 << 20))
    say("resample", kind, n)
    st, anc, inc = ctx.resample_weights(lw, seed, rnd)
    st_ref, anc_ref, inc_ref, _ = oracle.systematic(lw, seed, rnd)
    assert st == st_ref
    assert np.array_equal(anc, anc_ref)
    assert abs(inc - inc_ref) <= LOGZ_RTOL * max(1.0, abs(inc_ref))


def test_resample_weights_degenerate_and_nan(ctx, smc):
    st, _, inc = ctx.resample_weights(np.full(5000, -np.inf), 1, 0)
    assert st == smc.DEGENERATE and inc == -math.inf
    lw = np.zeros(3000)
    lw[1234] = np.nan
    st, _, _ = ctx.resample_weights(lw, 1, 0)
    assert st == smc.ERR_NAN


def test_resample_weights_max_size(ctx, oracle):
    n = 1 << 24
    rng = np.random.default_rng(24)
    lw = rng.normal(0, 2, n)
    say("resample max size", n)
    st, anc, inc = ctx.resample_weights(lw, 99, 3)
    st_ref, anc_ref, inc_ref, _ = oracle.systematic(lw, 99, 3)
    assert st == st_ref == 0
    assert np.array_equal(anc, anc_ref)
    assert abs(inc - inc_ref) <= LOGZ_RTOL * max(1.0, abs(inc_ref))


# --- whole runs, round by round -------------------------------------------------------------

def _compare_fields(smc, gpu, ref, spec):
    kind = spec["kind"]
    n_real, names = smc.FIELDS[kind]
    prec = spec.get("precision", 64)
    rdt = np.float32 if prec == 32 else np.float64
    for k in range(n_real):
        g = gpu.field(k, rdt)
        r = ref.field(k, rdt)
        assert np.array_equal(g.view(np.uint32 if prec == 32 else np.uint64),
                              r.view(np.uint32 if prec == 32 else np.uint64)), names[k]
    for k in range(len(names) - n_real):
        assert np.array_equal(gpu.field(n_real + k, np.int32), ref.field(n_real + k, np.int32)), names[n_real + k]
    if kind == "clads":
        depth = gpu.stats()["stack_depth"]
        assert depth == ref.max_stack
        sp = ref.field(5, np.int32)[0]
        g = gpu.field(len(names), rdt, depth)[:, :sp]
        r = ref.field(len(names), rdt, depth)[:, :sp]
        assert np.array_equal(g, r), "stack"


def run_lockstep(smc, oracle, ctx, spec, n, seed, check_every=1, max_rounds=10**6):
    model = smc.Model(ctx, spec)
    gpu = smc.Run(model, n, seed)
    ref = oracle.Run(spec, n, seed)
    rnd = 0
    try:
        while rnd < max_rounds:
            gpu.step()
            ref.step()
            if rnd % check_every == 0:
                assert np.array_equal(gpu.blk(), ref.blk()), f"blocks round {rnd}"
                assert np.array_equal(bits(gpu.lw()), bits(ref.lw())), f"log-weights round {rnd}"
                _compare_fields(smc, gpu, ref, spec)
            st_ref = ref.resample()
            gpu.resample()
            done, st = gpu.done()
            assert st == st_ref, (rnd, st, st_ref)
            if st_ref != oracle.OK:
                break
            if rnd % check_every == 0:
                assert np.array_equal(gpu.anc(), ref.anc()), f"ancestors round {rnd}"
                _compare_fields(smc, gpu, ref, spec)  # gathered state
                assert gpu.stats()["resamples"] == ref.resamples, f"resampling decisions round {rnd}"
            rnd += 1
        lz, lz_ref = gpu.log_z(), ref.log_z
        if math.isfinite(lz_ref):
            assert abs(lz - lz_ref) <= LOGZ_RTOL * abs(lz_ref), (lz, lz_ref)
        else:
            assert lz == lz_ref
        s = gpu.stats()
        assert s["block_steps"] == ref.block_steps
        return lz, ref
    finally:
        gpu.close()
        model.close()


def test_geometric_runs_match(smc, oracle, ctx):
    for checkpoint, n in ((True, 1000), (True, 1), (False, 777), (True, 5000)):
        say("geometric", checkpoint, n)
        run_lockstep(smc, oracle, ctx, I.geometric_spec(checkpoint), n, 11)


def test_kalman_config_matches(smc, oracle, ctx):
    """1-D linear-Gaussian filter: T = 100, N = 2^16, FP32 state."""
    y = I.lgssm_data(100, 2000)
    say("lgssm T=100 N=65536")
    run_lockstep(smc, oracle, ctx, I.lgssm_spec(y, 32), 1 << 16, 1, check_every=9)


def test_ssm_eq2_fp64_matches(smc, oracle, ctx):
    y = I.lgssm_data(20, 123, a=1.0, b=2.0, q=1.0, r=5.0, m0=0.0, s0=100.0)
    say("ssm eq2")
    run_lockstep(smc, oracle, ctx, I.lgssm_spec(y, 64, a=1.0, b=2.0, q=1.0, r=5.0, m0=0.0, s0=100.0), 3001, 4)


def test_crbd_small_config_matches(smc, oracle, ctx):
    """CRBD on a 20-tip Yule tree, N = 1000, FP64 throughout."""
    tree = I.yule_tree(20, 1000)
    say("crbd 20 tips N=1000")
    run_lockstep(smc, oracle, ctx, I.crbd_spec(tree, precision=64), 1000, 1)


def test_crbd_fp32_ragged_matches(smc, oracle, ctx):
    tree = I.yule_tree(48, 3000)
    say("crbd fp32 48 tips N=5000")
    run_lockstep(smc, oracle, ctx, I.crbd_spec(tree, precision=32), 5000, 7, check_every=5)


def test_crbd_caps_and_degenerate_match(smc, oracle, ctx):
    tree = I.yule_tree(6, 3)
    say("crbd caps")
    run_lockstep(smc, oracle, ctx, I.crbd_spec(tree, fixed_lambda=6.0, fixed_mu=6.0, max_events=3, max_depth=2),
                 2048, 2)
    say("crbd degenerate")
    lz, ref = run_lockstep(smc, oracle, ctx, I.crbd_spec(tree, fixed_lambda=50.0, fixed_mu=0.0), 64, 1)
    assert ref.status == oracle.DEGENERATE and lz == -math.inf


def test_clads_matches(smc, oracle, ctx):
    tree = I.yule_tree(40, 4001)
    say("clads 40 tips N=4096")
    run_lockstep(smc, oracle, ctx, I.clads_spec(tree, precision=32), 4096, 3, check_every=3)
    say("clads fp64 fixed")
    run_lockstep(smc, oracle, ctx, I.clads_spec(I.yule_tree(12, 5), precision=64, fixed_l0=2.0, fixed_eps=0.3,
                                                fixed_alpha=1.0, fixed_sigma=0.0), 1500, 9)


def test_run_to_end_and_call_order(smc, oracle, ctx):
    tree = I.yule_tree(20, 1000)
    spec = I.crbd_spec(tree, precision=64)
    model = smc.Model(ctx, spec)
    r = smc.Run(model, 1000, 1)
    with pytest.raises(smc.SMCError) as e:
        r.resample()
    assert e.value.code == smc.ERR_STATE
    r.step()
    with pytest.raises(smc.SMCError) as e:
        r.step()
    assert e.value.code == smc.ERR_STATE
    r.resample()
    st = r.run_to_end()
    ref = oracle.Run(spec, 1000, 1)
    ref.run_to_end()
    assert st == smc.FINISHED
    assert abs(r.log_z() - ref.log_z) <= LOGZ_RTOL * abs(ref.log_z)
    assert r.stats()["block_steps"] == 1000 * 39
    r.close()
    with pytest.raises(smc.SMCError):
        smc.Run(model, 0, 1)
    with pytest.raises(smc.SMCError):
        smc.Run(model, (1 << 24) + 1, 1)
    model.close()


def test_batch_matches_runs_alone(smc, oracle, ctx):
    """Runs of different sizes and models advanced together give the same
    log Z (and, being deterministic, the same ancestors) as alone."""
    specs = [I.crbd_spec(I.yule_tree(20 + 3 * i, 50 + i), precision=32) for i in range(3)]
    specs += [I.clads_spec(I.yule_tree(16 + 5 * i, 70 + i), precision=32) for i in range(3)]
    ns = [1000, 4096, 3000, 2048, 1025, 5000]
    models = [smc.Model(ctx, s) for s in specs]
    b = smc.Batch(ctx)
    slots = [b.add(m, n, 100 + i) for i, (m, n) in enumerate(zip(models, ns))]
    say("batch of", len(slots))
    for _ in range(200):
        b.tick(4)
        done, lz, st, steps = b.poll()
        if done.all():
            break
    assert done.all()
    for i, (s, n) in enumerate(zip(specs, ns)):
        ref = oracle.Run(s, n, 100 + i)
        ref.run_to_end()
        assert st[slots[i]] == ref.status
        assert abs(lz[slots[i]] - ref.log_z) <= LOGZ_RTOL * abs(ref.log_z), (i, lz[slots[i]], ref.log_z)
        assert steps[slots[i]] == ref.block_steps
    for s in slots:
        b.retire(s)
    b.close()
    for m in models:
        m.close()


def test_graph_replays_match_eager_runs(smc, oracle, ctx):
    """run_to_end replays one captured graph; each replay after a reset (with
    eager runs and synchronisations in between) equals an eager run and the
    oracle for that seed."""
    tree = I.yule_tree(30, 77)
    spec = I.crbd_spec(tree, precision=32)
    model = smc.Model(ctx, spec)
    replayed = smc.Run(model, 3000, 1)
    for seed in (5, 6, 7, 5):
        replayed.reset(seed)
        assert replayed.run_to_end() == smc.FINISHED
        eager = smc.Run(model, 3000, seed)
        while True:
            eager.step()
            eager.resample()
            done, st = eager.done()
            if done:
                break
        ref = oracle.Run(spec, 3000, seed)
        ref.run_to_end()
        a, b = replayed.stats(), eager.stats()
        assert a["log_z"] == b["log_z"] and a["block_steps"] == b["block_steps"] == ref.block_steps
        assert abs(a["log_z"] - ref.log_z) <= LOGZ_RTOL * abs(ref.log_z)
        assert np.array_equal(replayed.field(0, np.float32), eager.field(0, np.float32))
        eager.close()
    replayed.close()
    model.close()


def test_crbd_deep_recursion_matches(smc, oracle, ctx):
    """Critical birth-death rates make hidden lineages recurse well past the
    register-held frames, so many particles take the deep-stack pass."""
    tree = I.yule_tree(8, 5)
    say("crbd deep recursion fp64")
    run_lockstep(smc, oracle, ctx, I.crbd_spec(tree, fixed_lambda=10.0, fixed_mu=10.0), 2048, 1)
    say("crbd deep recursion fp32 priors")
    run_lockstep(smc, oracle, ctx, I.crbd_spec(tree, precision=32, scale_lambda=8.0, scale_mu=8.0), 3000, 2)


def test_clads_deep_side_lineages_match(smc, oracle, ctx):
    tree = I.yule_tree(8, 6)
    say("clads deep side lineages")
    run_lockstep(smc, oracle, ctx, I.clads_spec(tree, precision=64, fixed_l0=8.0, fixed_eps=0.95, fixed_alpha=1.0,
                                                fixed_sigma=0.0), 2048, 3)
    run_lockstep(smc, oracle, ctx, I.clads_spec(tree, precision=32, fixed_l0=6.0, fixed_eps=0.9), 2048, 4)


def test_large_run_fold_kernel_path_matches(smc, oracle, ctx):
    """Above 2^20 particles the propagation partials are folded by separate
    one-work-group kernels; ragged size, round-by-round parity."""
    y = I.lgssm_data(6, 31)
    say("lgssm N=2^20+4097")
    run_lockstep(smc, oracle, ctx, I.lgssm_spec(y, 32), (1 << 20) + 4097, 12, check_every=2)
