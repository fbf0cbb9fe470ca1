"""Host-side scheduling helpers of the serving loop (no GPU needed)."""
import numpy as np

from paper_2112_00364_amd import inputs as I
from paper_2112_00364_amd import serve as S


def test_request_stream_shape():
    reqs = I.request_stream(2000, 5000, rate_per_s=10.0)
    kinds = [r["kind"] for r in reqs]
    assert 0.45 < kinds.count("crbd") / len(kinds) < 0.55
    tips = np.array([r["tips"] for r in reqs])
    assert tips.min() >= 16 and tips.max() <= 512
    n = np.array([r["n"] for r in reqs])
    assert set(np.log2(n).astype(int)) <= set(range(10, 19))
    arr = np.array([r["arrival"] for r in reqs])
    assert np.all(np.diff(arr) > 0)
    assert abs(len(reqs) / arr[-1] - 10.0) < 1.0


def test_clads_stack_depth_matches_oracle(oracle):
    for n, seed in ((32, 1), (77, 2), (128, 3)):
        tree = I.yule_tree(n, seed)
        r = oracle.Run(I.clads_spec(tree), 1, 0)
        assert S.clads_stack_depth(tree) == r.max_stack


def test_footprint_counts_double_buffered_state():
    a = S.footprint_bytes("crbd", 1 << 20, 32)
    b = S.footprint_bytes("crbd", 1 << 20, 64)
    assert b - a == (1 << 20) * 2 * 2 * 4  # two real fields, two buffers, 4 extra bytes
    c = S.footprint_bytes("clads", 4096, 32, stack_depth=10)
    assert c > S.footprint_bytes("clads", 4096, 32, stack_depth=1)


def test_rescaled_arrivals_rate():
    reqs = I.request_stream(4000, 1, rate_per_s=1.0)
    S.rescale_arrivals(reqs, 50.0, 2)
    t = np.array([r["arrival"] for r in reqs])
    assert abs(len(t) / t[-1] - 50.0) < 3.0
