"""Host-side scheduling helpers of the serving loop (no GPU needed)."""
import numpy as np
import pytest

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


def test_launch_cache_keys_and_round_trip(tmp_path):
    """Run shapes are keyed by kind, precision and the powers of two above the
    particle count and tree size; the cache file round-trips."""
    from paper_2112_00364_amd import autotune as A
    assert A.shape_key("clads", 32, 4096, 100) == "clads/fp32/n4096/tips128"
    assert A.shape_key("crbd", 64, 1000, 20) == "crbd/fp64/n1024/tips32"
    assert A.shape_key("lgssm", 32, 65536, 0) == "lgssm/fp32/n65536/tips0"
    c = A.LaunchCache(str(tmp_path / "sub" / "launch.json"))
    assert c.get("x") is None
    c.put("x", {"lanes": 256, "ms": {"lanes128": 2.0, "lanes256": 1.0}})
    d = A.LaunchCache(str(tmp_path / "sub" / "launch.json"))
    assert d.get("x")["lanes"] == 256
    (tmp_path / "bad.json").write_text("{not json")
    assert A.LaunchCache(str(tmp_path / "bad.json")).entries == {}


def test_batch_launch_choice_is_applied_and_cached(tmp_path):
    """A cached launch choice is returned without timing anything, an owned
    choice calls set_owned and a segmented one set_workgroup, and a cache entry
    written before owning existed (no "owned" field) is not taken as a choice."""
    from paper_2112_00364_amd import autotune as A
    c = A.LaunchCache(str(tmp_path / "launch.json"))
    key = A.shape_key("crbd", 32, 256, 40)
    c.put(key, {"lanes": 256, "owned": True, "ms": {"lanes128": 3.0, "lanes256": 2.0, "owned": 1.0}})
    # no device is touched: the model and context are never used on a cache hit
    assert A.batch_launch(c, None, None, "crbd", 32, 256, 40) == {"lanes": 256, "owned": True}

    class FakeBatch:
        def __init__(self):
            self.calls = []

        def set_owned(self, slot, owned=True):
            self.calls.append(("owned", slot, owned))

        def set_workgroup(self, slot, lanes):
            self.calls.append(("lanes", slot, lanes))

    b = FakeBatch()
    A.apply_batch_launch(b, 3, {"lanes": 256, "owned": True})
    A.apply_batch_launch(b, 4, {"lanes": 128, "owned": False})
    assert b.calls == [("owned", 3, True), ("lanes", 4, 128)]
    # an entry without "owned" would be re-tuned: with no device that fails
    old = A.shape_key("clads", 32, 4096, 100)
    c.put(old, {"lanes": 128, "ms": {"lanes128": 1.0, "lanes256": 2.0}})
    with pytest.raises(Exception):
        A.batch_launch(c, None, None, "clads", 32, 4096, 100)


def test_fifo_replay_queues_measured_service_times():
    """One-at-a-time FIFO from measured service times: a request starts when it
    has arrived and the previous one is done, and takes its own service time."""
    from paper_2112_00364_amd import serve as S
    served = [{"id": 0, "start": 0.0, "done": 2.0, "log_z": -1.0, "status": 1, "block_steps": 10},
              {"id": 1, "start": 2.0, "done": 2.5, "log_z": -2.0, "status": 1, "block_steps": 20},
              {"id": 2, "start": 2.5, "done": 5.5, "log_z": -3.0, "status": 1, "block_steps": 30}]
    reqs = [{"id": 0, "arrival": 1.0}, {"id": 1, "arrival": 1.5}, {"id": 2, "arrival": 10.0}]
    out, makespan = S.fifo_replay(served, reqs)
    by = {r["id"]: r for r in out}
    assert (by[0]["start"], by[0]["done"]) == (1.0, 3.0)      # idle server: starts on arrival
    assert (by[1]["start"], by[1]["done"]) == (3.0, 3.5)      # queued behind request 0
    assert (by[2]["start"], by[2]["done"]) == (10.0, 13.0)    # server idle again
    assert makespan == 13.0
    assert by[1]["log_z"] == -2.0 and by[2]["block_steps"] == 30
    lat = S.summarize(out, makespan)
    assert lat["requests"] == 3 and lat["failed"] == 0
