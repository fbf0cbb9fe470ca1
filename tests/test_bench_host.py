"""Host-side logic of bench.py: the algorithmic byte counts the roofline divides
by, the rule that ties a counter record to the kernel sources, the refusal of
more than one GPU, and the all-cores oracle sample of the batched leg."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_algorithmic_bytes_per_round():
    # Per particle and round: propagate reads anc 4 + block 1 + (lambda, mu) 8 and
    # writes block 1 + (lambda, mu) 8 + lw 8 = 30 B (round 0 has nothing to gather:
    # 17 B); reduce reads lw 8 (+16 B per 1024-particle tile); scan reads lw 8 and
    # writes anc 4, except in the final round.
    n, rounds = 1 << 20, 511
    run_total = bench.bytes_per_launch("propagate", n, rounds) * rounds
    assert run_total == pytest.approx(n * (17 + 30 * (rounds - 1)), rel=1e-12)
    assert bench.bytes_per_launch("reduce", n, rounds) == n * 8 + (n // 1024) * 16
    assert bench.bytes_per_launch("scan_anc", n, rounds) * rounds == pytest.approx(n * 12 * (rounds - 1), rel=1e-12)
    # the headline figure quoted with the roofline: 31.4 MB per propagation step
    assert bench.bytes_per_launch("propagate", n, rounds) == pytest.approx(31.43e6, rel=1e-3)
    # single-pass resampling reads lw 8 and writes anc 4, except in the final round
    assert bench.bytes_per_launch("resample", n, rounds) * rounds == pytest.approx(n * (8 * rounds + 4 * (rounds - 1)),
                                                                                  rel=1e-12)
    # a split propagation's two launches make one step
    assert bench.STEPS["propagate"] == ("propagate", "hidden")


def test_clads_run_bytes_counts_the_live_stack():
    # Three-tip tree in preorder: root 0 -> (1, 4); node 1 -> (2, 3). The walk
    # visits nodes 1..4 with 1, 2, 1, 0 pending rates below them (one left at
    # the root; internal node 1 pushes one; each tip pops one).
    tree = {"left": [1, 2, -1, -1, -1]}
    n = 10
    per = 29                              # round 0: block 1 + state 16 + level 0 4 + lw 8
    per += 46 + 8 * 1 + 4                 # node 1, internal, sp = 1
    per += 46 + 8 * 2                     # node 2, tip, sp = 2
    per += 46 + 8 * 1                     # node 3, tip, sp = 1
    per += 46 + 8 * 0                     # node 4, tip, sp = 0
    per += 20 * 4 + 8                     # four resampling rounds, the last one only reads lw
    assert bench.clads_run_bytes(tree, n) == n * per


def test_traffic_record_only_for_current_kernels(tmp_path, monkeypatch):
    """Traffic per round of a step: every dispatch of the step's kernels in the
    profiled runs, over runs x rounds; only while the record's kernel sources
    are the current ones."""
    os.makedirs(tmp_path / "profiles")
    rec = {"kernels": {"propagate": {"hbm_bytes_total": 1000.0}, "hidden": {"hbm_bytes_total": 230.0}},
           "source_sha": "aaaa", "runs": 2}
    (tmp_path / "profiles" / "t.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "aaaa")
    assert bench.measured_traffic("propagate", 5, "t.json") == pytest.approx(1230.0 / 10)
    assert bench.measured_traffic("reduce", 5, "t.json") is None      # kernel not in the record
    assert bench.measured_traffic("propagate", 5, "none.json") is None  # no record
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "bbbb")
    assert bench.measured_traffic("propagate", 5, "t.json") is None   # kernels changed since


def test_kernel_source_hash_ignores_host_engine():
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_batched_leg_cpu_sample(oracle):
    out = bench.batched_clads_cpu(runs_per_worker=1, n=256, max_workers=2)
    assert out["kind"] == "oracle" and out["unit"] == "particle-block-steps/s"
    assert 1 <= out["cores"] <= 2 and out["value"] > 0
    assert "one oracle process per run" in out["sample"]
    assert 0 <= out["finished_runs"] <= 2
