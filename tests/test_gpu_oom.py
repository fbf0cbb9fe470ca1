"""Allocation failures through the context's allocator callback.

The callback is part of the C interface (the caller's allocator supplies every
device buffer). A callback that returns NULL must turn into SMC_ERR_OOM with
nothing leaked; a batch whose tick could not allocate its tables must rebuild
them on the next tick and still give every run's own result; the serving loop
must postpone an admission that does not fit and retry it after retirements.
Failures are forced from the host: no kernel runs on a partial allocation.
"""
import sys

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


class FailingAllocator:
    """torch's caching allocator behind a switch: fails the call with index
    `fail_at` (0-based, counted from `arm()`), or every allocation of at least
    `cap_min` bytes that would take the live total above `cap` bytes (a device
    with less particle memory than the caller's budget; small control
    allocations still succeed). Tracks the live allocations."""

    def __init__(self):
        import torch
        self.torch = torch
        self.live = {}
        self.calls = 0
        self.fail_at = None
        self.cap = None
        self.cap_min = 0
        self.failures = 0

    def arm(self, fail_at=None, cap=None, cap_min=0):
        self.calls = 0
        self.fail_at = fail_at
        self.cap = cap
        self.cap_min = cap_min

    def alloc(self, nbytes):
        k = self.calls
        self.calls += 1
        if self.fail_at is not None and k == self.fail_at:
            self.failures += 1
            return None
        if self.cap is not None and nbytes >= self.cap_min and sum(self.live.values()) + nbytes > self.cap:
            self.failures += 1
            return None
        p = self.torch.cuda.caching_allocator_alloc(int(nbytes), 0, self.torch.cuda.current_stream(0))
        self.live[p] = int(nbytes)
        return p

    def free(self, p):
        assert p in self.live, "freed a pointer the allocator never handed out"
        del self.live[p]
        self.torch.cuda.caching_allocator_delete(p)


def test_init_oom_at_every_allocation_leaks_nothing(smc, oracle):
    tree = I.yule_tree(12, 21)
    spec = I.clads_spec(tree, precision=32)
    A = FailingAllocator()
    ctx = smc.Context(0, allocator=(A.alloc, A.free))
    model = smc.Model(ctx, spec)
    baseline = dict(A.live)
    A.arm()
    probe = smc.Run(model, 3000, 4)
    n_allocs = A.calls
    probe.close()
    assert A.live == baseline and n_allocs > 5
    for k in range(n_allocs):
        A.arm(fail_at=k)
        with pytest.raises(smc.SMCError) as e:
            smc.Run(model, 3000, 4)
        assert e.value.code == smc.ERR_OOM, (k, e.value)
        assert A.live == baseline, f"allocation {k}: leaked {len(A.live) - len(baseline)} buffers"
    A.arm()
    run = smc.Run(model, 3000, 4)
    assert run.run_to_end() == smc.FINISHED
    ref = oracle.Run(spec, 3000, 4)
    ref.run_to_end()
    assert abs(run.log_z() - ref.log_z) <= LOGZ_RTOL * abs(ref.log_z)
    run.close()
    model.close()
    assert A.live == {}
    ctx.close()


def test_model_register_oom_leaks_nothing(smc):
    spec = I.crbd_spec(I.yule_tree(30, 2), precision=32)
    A = FailingAllocator()
    ctx = smc.Context(0, allocator=(A.alloc, A.free))
    A.arm()
    m = smc.Model(ctx, spec)
    n_allocs = A.calls
    m.close()
    assert A.live == {}
    for k in range(n_allocs):
        A.arm(fail_at=k)
        with pytest.raises(smc.SMCError) as e:
            smc.Model(ctx, spec)
        assert e.value.code == smc.ERR_OOM
        assert A.live == {}
    ctx.close()


def test_batch_tick_oom_then_retry_gives_same_results(smc, oracle):
    """The tick's table allocation fails: the tick reports ERR_OOM and leaves
    no partial table behind; the next tick rebuilds the tables and every run
    finishes with its own result."""
    specs = [I.crbd_spec(I.yule_tree(14, 31), precision=32), I.clads_spec(I.yule_tree(10, 32), precision=32)]
    ns = [2000, 1500]
    A = FailingAllocator()
    ctx = smc.Context(0, allocator=(A.alloc, A.free))
    models = [smc.Model(ctx, s) for s in specs]
    b = smc.Batch(ctx)
    slots = [b.add(m, n, 50 + i) for i, (m, n) in enumerate(zip(models, ns))]
    for fail_at in (0, 1, 2):  # run table, reduction tile table, a propagation tile table
        A.arm(fail_at=fail_at)
        with pytest.raises(smc.SMCError) as e:
            b.tick(2)
        assert e.value.code == smc.ERR_OOM
    A.arm()
    for _ in range(100):
        b.tick(4)
        done, lz, st, steps = b.poll()
        if done.all():
            break
    assert done.all()
    for i, (s, n) in enumerate(zip(specs, ns)):
        ref = oracle.Run(s, n, 50 + i)
        ref.run_to_end()
        assert st[slots[i]] == ref.status
        assert abs(lz[slots[i]] - ref.log_z) <= LOGZ_RTOL * abs(ref.log_z)
        assert steps[slots[i]] == ref.block_steps
    # a run added after the failures joins cleanly
    extra = b.add(models[0], 700, 99)
    for _ in range(100):
        b.tick(4)
        done, lz, st, steps = b.poll()
        if done[extra]:
            break
    ref = oracle.Run(specs[0], 700, 99)
    ref.run_to_end()
    assert abs(lz[extra] - ref.log_z) <= LOGZ_RTOL * abs(ref.log_z)
    for s in slots + [extra]:
        b.retire(s)
    b.close()
    for m in models:
        m.close()
    assert A.live == {}
    ctx.close()


def test_serving_admission_waits_for_memory(smc):
    """A device that holds fewer runs than the memory budget admits: admissions
    that fail with ERR_OOM wait for retirements and are retried; every request
    ends with the log Z it has when served alone."""
    from paper_2112_00364_amd import serve as S
    reqs = []
    for i in range(8):
        tips = 16 + 3 * i
        tree = I.yule_tree(tips, 900 + i)
        r = {"id": i, "arrival": 0.0, "tips": tips, "seed": 10 + i, "rounds": 2 * tips - 1}
        if i % 2 == 0:
            r.update(kind="crbd", spec=I.crbd_spec(tree, precision=32), depth=0, n=1024)
        else:
            r.update(kind="clads", spec=I.clads_spec(tree, precision=32), depth=S.clads_stack_depth(tree), n=2048)
        r["block_steps"] = r["n"] * r["rounds"]
        r["bytes"] = S.footprint_bytes(r["kind"], r["n"], 32, r["depth"])
        reqs.append(r)
    A = FailingAllocator()
    ctx = smc.Context(0, allocator=(A.alloc, A.free))
    side_stack = 32 * 17 * 2048  # the largest allocation of a ClaDS request
    cap = int(2.5 * side_stack)
    A.arm(cap=cap, cap_min=16384)
    say("serving with a particle-memory cap of", cap, "bytes")
    out, _ = S.serve_batched(ctx, reqs, memory_budget=1 << 40, rounds_per_tick=8, honour_arrivals=False,
                             log_every=0)
    assert S.serve_batched.last_oom_waits > 0 and A.failures > 0
    A.arm()
    alone, _ = S.serve_one_at_a_time(ctx, reqs, honour_arrivals=False, log_every=0)
    a = {r["id"]: r for r in alone}
    assert len(out) == len(reqs)
    for r in out:
        ref = a[r["id"]]
        assert r["status"] == ref["status"] == smc.FINISHED
        assert abs(r["log_z"] - ref["log_z"]) <= LOGZ_RTOL * abs(ref["log_z"])
        assert r["block_steps"] == ref["block_steps"]
    assert A.live == {}
    ctx.close()
