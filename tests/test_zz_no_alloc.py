"""The allocation-free resampling entry point (smc_resample_weights_noalloc)
against smc_resample_weights through the C interface: two calls in a row, the
second on a smaller input, each bit-exact in ancestors, log Z increment and
status; the device allocator is never asked for memory during the calls."""
import math
import sys

import numpy as np
import pytest

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


class CountingAllocator:
    def __init__(self):
        import torch
        self.torch = torch
        self.calls = 0
        self.live = {}

    def alloc(self, nbytes):
        self.calls += 1
        t = self.torch.empty(nbytes, dtype=self.torch.uint8, device="cuda")
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def free(self, p):
        self.live.pop(p, None)


def _weights(n, rng, kind):
    if kind == "wide":
        lw = rng.normal(0, 30, n)
        lw[rng.random(n) < 0.3] = -np.inf
        lw[rng.integers(n)] = 5.0
        return lw
    return rng.normal(0, 3, n) - 50.0


def _one_call(smc, ctx_ref, ctx_na, alloc, lw, seed, rnd):
    import torch
    n = len(lw)
    st_ref, anc_ref, inc_ref = ctx_ref.resample_weights(lw, seed, rnd)
    lw_dev = torch.as_tensor(lw, dtype=torch.float64, device="cuda")
    anc_dev = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    inc_dev = torch.full((1,), math.nan, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    before = alloc.calls
    st = ctx_na.resample_weights_noalloc(lw_dev, anc_dev, inc_dev, seed, rnd)
    assert alloc.calls == before, "the allocation-free entry point asked for device memory"
    assert st == st_ref
    if st == smc.OK:
        assert np.array_equal(anc_dev.cpu().numpy().view(np.uint32), anc_ref)
    inc = float(inc_dev.cpu()[0])
    assert np.float64(inc).view(np.uint64) == np.float64(inc_ref).view(np.uint64), (inc, inc_ref)


@pytest.mark.parametrize("sizes", [((1 << 20) + 4097, 5000), ((1 << 24), (1 << 20) - 3), (3000, 1)])
def test_noalloc_matches_resample_weights(smc, sizes):
    alloc = CountingAllocator()
    ctx_ref = smc.Context(0)
    ctx_na = smc.Context(0, allocator=(alloc.alloc, alloc.free))
    rng = np.random.default_rng(sizes[0] % 1000003)
    try:
        for i, n in enumerate(sizes):
            say("noalloc call", i, "n", n)
            lw = _weights(n, rng, "wide" if i else "normal")
            _one_call(smc, ctx_ref, ctx_na, alloc, lw, int(rng.integers(1 << 62)), int(rng.integers(1 << 20)))
    finally:
        ctx_na.close()
        ctx_ref.close()


def test_noalloc_statuses_and_limits(smc):
    import torch
    alloc = CountingAllocator()
    ctx_ref = smc.Context(0)
    ctx_na = smc.Context(0, allocator=(alloc.alloc, alloc.free))
    try:
        say("noalloc degenerate / nan")
        _one_call(smc, ctx_ref, ctx_na, alloc, np.full(5000, -np.inf), 1, 0)
        lw = np.zeros(3000)
        lw[1234] = np.nan
        _one_call(smc, ctx_ref, ctx_na, alloc, lw, 1, 0)
        # after a failed call the next one starts clean
        _one_call(smc, ctx_ref, ctx_na, alloc, np.random.default_rng(2).normal(0, 1, 4096), 7, 3)
        small = torch.zeros(16, dtype=torch.float64, device="cuda")
        anc = torch.zeros(16, dtype=torch.int32, device="cuda")
        L = smc.lib()
        import ctypes
        st = L.smc_resample_weights_noalloc(ctx_na._h, ctypes.c_void_p(small.data_ptr()), (1 << 24) + 1, 1, 0,
                                            ctypes.c_void_p(anc.data_ptr()), ctypes.c_void_p(small.data_ptr()))
        assert st == smc.ERR_INVALID
        st = L.smc_resample_weights_noalloc(ctx_na._h, ctypes.c_void_p(small.data_ptr()), 0, 1, 0,
                                            ctypes.c_void_p(anc.data_ptr()), ctypes.c_void_p(small.data_ptr()))
        assert st == smc.ERR_INVALID
        assert alloc.calls == 0
    finally:
        ctx_na.close()
        ctx_ref.close()
