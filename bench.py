#!/usr/bin/env python3
"""Throughput of SMC over a PCFG on one MI355X: CRBD on a 256-tip tree, 2^20 particles.

One step is one complete SMC run (Algorithm 1: initialisation, 511 rounds of
propagation + resampling, final log Z) on the constant-rate birth-death model
of the paper's appendix, conditioned on a synthetic 256-tip Yule tree, with
FP32 particle state and FP64 log-weights and scan. The tree lives in device
memory before timing starts and every run's buffers are allocated beforehand.
Printed: one JSON line with canonical particle-block-steps/s (block executions
excluding b_stop, per second of wall time of the timed runs), the dominant
kernel's achieved bandwidth against MI355X's HBM peak, and the CPU oracle's
throughput on a bounded sample of the same workload. Beside the headline: the
same workload at 2^24 particles (buffers beyond the Infinity Cache), 512
batched ClaDS runs of 4096 particles, and a serving stream (one-at-a-time vs
continuous batching, p50/p99 latency), the headline workload with
ESS-triggered resampling, the same tree with delayed sampling and ESS-triggered
resampling (the paper's CRBD experiment with variance-reducing techniques), and
the vector-borne disease (SEIR) model.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-block-steps/s at 2^20 CRBD particles; batched p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
TIPS, TREE_SEED, N_PARTICLES = 256, 3000, 1 << 20

# Algorithmic bytes per launch (FP32 state: lambda, mu), per particle unless noted.
#  propagate:  the propagation step (both phases when it is split): anc 4 + gathered block 1 +
#              gathered state 8 read; block 1 + state 8 + lw 8 written (round 0 only writes: 17).
#              The hidden-event queue between the phases is the implementation's own traffic.
#  reduce:     lw 8 read (+ 16 B of tile sums written per 1024-particle tile)
#  scan_anc:   lw 8 read, anc 4 written (the final round only updates log Z)
#  resample:   single pass: lw 8 read, anc 4 written (the final round only reads)
def bytes_per_launch(kernel: str, n: int, rounds: int) -> float:
    if kernel == "propagate":
        return n * (17 + 30 * (rounds - 1)) / rounds
    if kernel == "reduce":
        return n * 8.0 + n / 1024 * 16
    if kernel == "resample":
        return n * (8.0 + 4.0 * (rounds - 1) / rounds)
    return n * 12.0 * (rounds - 1) / rounds


# Kernels that make up one step of a round: the roofline is taken per step.
STEPS = {"propagate": ("propagate", "hidden"), "resample": ("resample",), "reduce": ("reduce",),
         "scan_anc": ("scan_anc",), "bucket": ("bucket",)}


def kernel_source_hash() -> str:
    """Hash of the device code's sources (kernels.hip and the headers it
    includes); the host engine (capi.hip) does not change what a kernel moves,
    so counter records stay valid across host-only changes."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2112_00364_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f == "kernels.hip" or f.endswith(".hpp"):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(step: str, rounds: int, record: str = "traffic_crbd_yule256_n2p20.json"):
    """HBM bytes per round of one step (all its kernels' dispatches over a
    run, divided by the run's rounds) from a committed rocprofv3 counter
    summary of one complete run, if it was taken on the current kernel
    sources; else None."""
    path = os.path.join(ROOT, "profiles", record)
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    ks = d.get("kernels", {})
    parts = [k for k in STEPS.get(step, (step,)) if k in ks]
    if d.get("source_sha") != kernel_source_hash() or not parts or any("hbm_bytes_total" not in ks[k] for k in parts):
        return None
    runs = d.get("runs", 1)
    return sum(ks[k]["hbm_bytes_total"] for k in parts) / (runs * rounds)


def cpu_baseline(spec, n: int):
    from oracle import oracle as O
    O.build()
    t0 = time.perf_counter()
    r = O.Run(spec, n, 7)
    st = r.run_to_end()
    dt = time.perf_counter() - t0
    assert st == O.FINISHED
    return {"value": r.block_steps / dt, "unit": "particle-block-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"CRBD, {TIPS}-tip Yule tree (seed {TREE_SEED}), {n} particles, all {r.round + 1} rounds, "
                      f"single thread, {dt:.1f} s"}


def clads_run_bytes(tree, n: int) -> float:
    """Algorithmic HBM bytes of one complete ClaDS run of n particles (FP32
    state). Round 0 writes block 1 + state 16 + stack level 0 4 + lw 8. A
    branch round at node r with sp pending rates below it: anc 4 + gathered
    block 1 + state 16 + the sp live stack levels 4 sp read; block 1 + state 16
    + the carried levels 4 sp (+ the new level 4 at an internal node) + lw 8
    written. Every round but the last resamples: lw 8 read twice, anc 4
    written (the reduction's tile sums aside)."""
    left = tree["left"]
    total = 29.0
    cur = 1
    for node in range(1, len(left)):
        internal = left[node] >= 0
        total += 46 + 8 * cur + (4 if internal else 0)
        cur = cur + 1 if internal else max(cur - 1, 0)
    rounds = len(left)
    total += 20.0 * (rounds - 1) + 8.0
    return n * total


def batched_clads(ctx, smc, I, runs=512, n=4096, rounds_per_tick=16, tune=True, cache_path=None):
    """512 independent ClaDS runs (trees of 32-128 tips, seeds 4000 + r), 4096
    particles each, advanced together by the batch API. Before the timed
    region the batch autotuner picks each run shape's launch option -- the
    propagation work-group size of the segmented launches, or one work-group
    owning each run -- cached in a JSON file, tuned on a probe batch the first
    time."""
    import numpy as np
    import torch
    from paper_2112_00364_amd import autotune as A
    rng = np.random.default_rng(4000)
    tips = rng.integers(32, 129, size=runs)
    trees = [I.yule_tree(int(t), 4000 + r) for r, t in enumerate(tips)]
    models = [smc.Model(ctx, I.clads_spec(tr, precision=32)) for tr in trees]
    alg_bytes = sum(clads_run_bytes(tr, n) for tr in trees)
    lanes = {}
    tune_s = 0.0
    cache = A.LaunchCache(cache_path)
    if tune:
        t0 = time.perf_counter()
        for r, t in enumerate(tips):
            key = A.shape_key("clads", 32, n, int(t))
            if key not in lanes:
                lanes[key] = A.batch_launch(cache, ctx, models[r], "clads", 32, n, int(t))
        tune_s = time.perf_counter() - t0
    b = smc.Batch(ctx)
    for r, m in enumerate(models):
        slot = b.add(m, n, 40000 + r)
        if tune:
            A.apply_batch_launch(b, slot, lanes[A.shape_key("clads", 32, n, int(tips[r]))])
    b.tick(0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ticks = 0
    while True:
        b.tick(rounds_per_tick)
        ticks += 1
        done, lz, st, steps = b.poll()
        if ticks % 4 == 0:
            print(f"batched: tick {ticks}, {int(done.sum())}/{runs} done", file=sys.stderr, flush=True)
        if done.all():
            break
    dt = time.perf_counter() - t0
    total = int(steps.sum())
    ok = int((st == smc.FINISHED).sum())
    b.close()
    for m in models:
        m.close()
    return {"workload": f"clads_batch_{runs}x{n}", "runs": runs, "particles_per_run": n,
            "tips": [int(tips.min()), int(tips.max())], "seconds": dt, "block_steps": total,
            "block_steps_per_s": total / dt, "finished_runs": ok, "rounds_per_tick": rounds_per_tick,
            "launch_choice": lanes, "autotune": {key: cache.get(key) for key in lanes},
            "autotune_seconds": tune_s,
            # the whole leg (every launch of every tick) against HBM: the batch is bound by its
            # longest dependent chains, not by memory
            "roofline": {"bound": "hbm", "achieved": round(alg_bytes / dt / 1e9, 3), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(alg_bytes / dt / 1e9 / HBM_PEAK_GBS, 6), "traffic": None,
                         "kernel": "all launches of the leg", "alg_bytes": alg_bytes}}


def owned_point(ctx, smc, I, rounds_per_tick=16):
    """Whole batches run to the end with segmented launches and with every run
    owned by one work-group (smc_batch_set_owned): seconds each and whether the
    log Z bits agree. Trees of 32-128 tips (seed 5), seeds 40000 + r."""
    import numpy as np
    import torch

    def whole(models, ns, owned):
        b = smc.Batch(ctx)
        slots = [b.add(m, n, 40000 + i) for i, (m, n) in enumerate(zip(models, ns))]
        for s in slots:
            if owned:
                b.set_owned(s)
        b.tick(0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        while True:
            b.tick(rounds_per_tick)
            done, lz, st, steps = b.poll()
            if done.all():
                break
        dt = time.perf_counter() - t0
        b.close()
        return dt, [float(x) for x in lz[:len(slots)]], int(steps.sum())

    out = {}
    rng = np.random.default_rng(5)
    for name, kind, count, n in (("crbd_16x256", "crbd", 16, 256), ("crbd_256x1024", "crbd", 256, 1024),
                                 ("crbd_64x4096", "crbd", 64, 4096), ("clads_128x1024", "clads", 128, 1024),
                                 ("clads_512x4096", "clads", 512, 4096)):
        tips = rng.integers(32, 129, size=count)
        make = I.crbd_spec if kind == "crbd" else I.clads_spec
        models = [smc.Model(ctx, make(I.yule_tree(int(t), 4000 + r), precision=32)) for r, t in enumerate(tips)]
        seg = whole(models, [n] * count, False)
        own = whole(models, [n] * count, True)
        for m in models:
            m.close()
        out[name] = {"segmented_s": seg[0], "owned_s": own[0], "block_steps": seg[2],
                     "same_log_z": seg[1] == own[1]}
        print(f"owned: {name} segmented {seg[0]:.3f} s, owned {own[0]:.3f} s", file=sys.stderr, flush=True)
    return out


def _clads_oracle_run(job):
    """One run of the ClaDS batch (run index r, tips) on the CPU oracle, in a worker process."""
    r, tips, n = job
    from oracle import oracle as O
    from paper_2112_00364_amd import inputs as I
    run = O.Run(I.clads_spec(I.yule_tree(tips, 4000 + r), precision=32), n, 40000 + r)
    st = run.run_to_end()
    return st == O.FINISHED, run.block_steps


def batched_clads_cpu(runs_per_worker: int = 8, n: int = 4096, max_workers: int = 16):
    """The batched ClaDS workload on the host: its first runs (same trees and seeds),
    each an independent oracle process, on every host core available to this
    process (at most `max_workers`). Aggregate block-steps/s over the wall time."""
    import multiprocessing as mp
    import numpy as np
    from oracle import oracle as O
    O.build()
    workers = max(1, min(max_workers, len(os.sched_getaffinity(0))))
    tips = np.random.default_rng(4000).integers(32, 129, size=512)
    jobs = [(r, int(tips[r]), n) for r in range(workers * runs_per_worker)]
    t0 = time.perf_counter()
    # fresh interpreters (not forks of this process, which holds a GPU context)
    with mp.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_clads_oracle_run, jobs, chunksize=1)
    dt = time.perf_counter() - t0
    steps = sum(s for _, s in res)
    return {"value": steps / dt, "unit": "particle-block-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"runs 0-{len(jobs) - 1} of the ClaDS batch ({n} particles each), one oracle process "
                      f"per run, {workers} processes, {dt:.1f} s",
            "finished_runs": sum(1 for ok, _ in res if ok)}


def serving_contexts(smc, ctx):
    """The per-kind server's contexts: one per model kind, each on its own HIP
    stream (default priority), and an idle one on which models are registered."""
    import torch
    kinds = {k: smc.Context(ctx.device, stream=torch.cuda.Stream(device=ctx.device)) for k in ("crbd", "clads")}
    return kinds, smc.Context(ctx.device, stream=torch.cuda.Stream(device=ctx.device))


def serving(ctx, smc, n_requests: int, budget_bytes: int, multipliers, alone_path=None, save_alone=None,
            mode: str = "by-kind"):
    """Serving stream: every request served alone once, back to back (plain
    runs, FIFO), which gives its service time, its log Z and the
    one-at-a-time service rate; then for each multiplier m the same requests
    arrive (Poisson) at m x that rate and are served (a) one at a time, FIFO:
    latencies from the measured service times, and (b) by continuous
    batching, in real time: one batch for all requests (mode "single") or one
    batch per model kind, each on its own stream (mode "by-kind"). The
    back-to-back pass can be saved to a JSON file (save_alone) and read back
    (alone_path), so that the arrival rates of one stream can be measured in
    separate processes against one pass."""
    from paper_2112_00364_amd import serve as S
    reqs = S.make_requests(n_requests, 5000, rate_per_s=1.0)
    if alone_path:
        rec = json.load(open(alone_path))
        assert rec["requests"] == n_requests and rec["stream_seed"] == 5000, "pass of another stream"
        alone, t_alone = rec["served"], rec["seconds"]
    else:
        alone, t_alone = S.serve_one_at_a_time(ctx, reqs, honour_arrivals=False)
        if save_alone:
            with open(save_alone, "w") as f:
                json.dump({"requests": n_requests, "stream_seed": 5000, "seconds": t_alone, "served": alone}, f)
    rate = len(reqs) / t_alone
    out = {"requests": n_requests, "one_at_a_time_service_rate_per_s": rate, "memory_budget_bytes": budget_bytes,
           "one_at_a_time_latencies": "FIFO over the measured service times of the back-to-back pass",
           "one_at_a_time_pass": alone_path or "measured in this process", "batched_mode": mode,
           "by_arrival_rate": []}
    by_kind = serving_contexts(smc, ctx) if mode == "by-kind" else None
    for m in multipliers:
        arr = m * rate
        S.rescale_arrivals(reqs, arr, 5001)
        print(f"serving: one-at-a-time rate {rate:.2f}/s, arrivals at {arr:.2f}/s", file=sys.stderr, flush=True)
        base, t_base = S.fifo_replay(alone, reqs)
        if by_kind:
            bat, t_bat = S.serve_batched_by_kind(by_kind[0], by_kind[1], reqs, budget_bytes)
        else:
            bat, t_bat = S.serve_batched(ctx, reqs, budget_bytes)
        same = {r["id"]: r["log_z"] for r in base}
        worst = max(abs(r["log_z"] - same[r["id"]]) / max(1.0, abs(same[r["id"]])) for r in bat)
        identical = all(r["log_z"] == same[r["id"]] for r in bat)
        out["by_arrival_rate"].append({"multiplier": m, "arrival_rate_per_s": arr,
                                       "one_at_a_time": S.summarize(base, t_base),
                                       "batched": S.summarize(bat, t_bat),
                                       "max_rel_logz_diff_batched_vs_alone": worst,
                                       "identical_log_z_batched_vs_alone": identical})
    if by_kind:
        for c in list(by_kind[0].values()) + [by_kind[1]]:
            c.close()
    return out


def ess_point(smc, ctx, spec, n: int, tau: float = 0.5, runs: int = 3):
    """The headline workload with ESS-triggered resampling (threshold tau):
    rounds whose effective sample size stays above tau N keep their weights
    and skip the ancestor pass."""
    import torch
    model = smc.Model(ctx, dict(spec, ess_threshold=tau))
    run = smc.Run(model, n, 91)
    run.run_to_end()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(ctx.stream)
    for i in range(runs):
        run.reset(92 + i)
        assert run.run_to_end() == smc.FINISHED
    end.record(ctx.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / runs
    s = run.stats()
    run.close()
    model.close()
    return {"ess_threshold": tau, "particles": n, "runs": runs, "ms_per_run": ms,
            "rounds": s["round"] + 1, "resampled_rounds": s["resamples"],
            "block_steps_per_s": s["block_steps"] / (ms / 1e3), "log_z_last": s["log_z"]}


def seir_point(smc, ctx, I, n: int = 1 << 18, days: int = 100, runs: int = 3, cpu: bool = True):
    """The vector-borne disease (SEIR) model of the paper's second experiment
    on a synthetic 100-day outbreak (the dengue data is not available), with
    the listing's priors: complete runs on the GPU, and the oracle on a
    bounded sample for scale."""
    import torch
    y = I.seir_data(days, 6000)
    spec = I.seir_spec(y, 32)
    model = smc.Model(ctx, spec)
    run = smc.Run(model, n, 61)
    run.run_to_end()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(ctx.stream)
    for i in range(runs):
        run.reset(62 + i)
        run.run_to_end()
    end.record(ctx.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / runs
    s = run.stats()
    run.close()
    # per particle and round, FP32 state (6 reals, 9 counts: 60 B): anc 4 + gathered block 1 +
    # gathered state 60 read, block 1 + state 60 + lw 8 written (round 0 writes only: 69);
    # resampling as in every model
    byte_model = {"propagate": lambda R: n * (69 + 134 * (R - 1)) / R,
                  "reduce": n * 8.0 + n / 1024 * 16, "scan_anc": lambda R: n * 12.0 * (R - 1) / R}
    kernels, roofline = profile_steps(smc, model, n, 4343, ms, byte_model)
    model.close()
    out = {"workload": f"seir_synthetic{days}d_n{n}", "particles": n, "days": days, "runs": runs,
           "ms_per_run": ms, "status": s["status"], "log_z_last": s["log_z"],
           "block_steps_per_s": s["block_steps"] / (ms / 1e3), "roofline": roofline, "kernels": kernels}
    if cpu:
        from oracle import oracle as O
        m = 1 << 12
        t0 = time.perf_counter()
        r = O.Run(spec, m, 61)
        r.run_to_end()
        dt = time.perf_counter() - t0
        out["cpu_oracle_block_steps_per_s"] = r.block_steps / dt
        out["cpu_oracle_sample"] = f"{m} particles, all {days} days, single thread, {dt:.1f} s"
    return out


def program_point(smc, ctx, I, n: int = 1 << 20, T: int = 100, runs: int = 2, cpu: bool = True,
                  tail: bool = True):
    """A compiled program (Sec. 4): eq. (2)'s state-space model written as a
    recursive CorePPL-style function, compiled by Algorithm 2 and run by the
    bytecode interpreter, beside the hand-written built-in block table on the
    same data (both FP64 state; they give the same bits). Every observation
    adds one frame of `step` to the particle's stack, so at the start of round
    t the live stack holds F_main + t F_step words and the live-prefix gather
    moves 16 (F_main + t F_step) bytes per particle: the leg measures that copy
    against HBM."""
    import torch
    from paper_2112_00364_amd import ppl
    y = I.lgssm_data(T, 2000)
    img = ppl.compile_program(I.lgssm_program(y), stack_words=8 * T + 8)
    f_main, f_step = img.frames["main"], img.frames["step"]
    out = {"workload": f"lgssm_program_T{T}_n{n}", "particles": n, "observations": T, "runs": runs,
           "stack_words": img.stack_words, "frame_words": dict(img.frames), "blocks": img.n_blocks,
           "instructions": int(len(img.code))}

    def timed(model, seed):
        run = smc.Run(model, n, seed)
        run.run_to_end()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(ctx.stream)
        for i in range(runs):
            run.reset(seed + 1 + i)
            run.run_to_end()
        end.record(ctx.stream)
        torch.cuda.synchronize()
        return run, start.elapsed_time(end) / runs

    model = smc.Model(ctx, {"kind": "program", "precision": 64, "program": img})
    run, ms = timed(model, 81)
    s = run.stats()
    lz_program = s["log_z"]
    run.reset(81 + runs)
    run.profile(True)
    run.run_to_end()
    kt = run.kernel_times()
    run.profile(False)
    run.close()
    model.close()
    # the same model written with a self tail call: constant stack, so no growing gather
    tms = lz_tail = None
    if tail:
        timg = ppl.compile_program(I.lgssm_program(y, tail=True), stack_words=16)
        tmodel = smc.Model(ctx, {"kind": "program", "precision": 64, "program": timg})
        trun, tms = timed(tmodel, 81)
        lz_tail = trun.stats()["log_z"]
        trun.close()
        tmodel.close()
    builtin = smc.Model(ctx, I.lgssm_spec(y, 64))
    brun, bms = timed(builtin, 81)
    lz_builtin = brun.stats()["log_z"]
    brun.close()
    builtin.close()
    ms_prop, launches = kt["propagate"]
    # run_to_end checks termination every 16 rounds, so a run also makes a few
    # launches after its last round (they return at once): rate the propagation
    # by its summed time per run, i.e. per round of the run.
    us = 1e3 * ms_prop / T
    # per particle and round: anc 4 + block 1 + sp 4 read, block 1 + sp 4 + lw 8 written,
    # plus the live prefix read and written (the stores of the running block are not counted)
    words = sum(f_main + f_step * t for t in range(1, T))
    per_round = n * (22.0 * T + 16.0 * words) / T
    out.update({"ms_per_run": ms, "builtin_ms_per_run": bms, "tail_call_ms_per_run": tms,
                "tail_call_same_log_z": None if lz_tail is None else lz_tail == lz_builtin,
                "status": s["status"],
                "block_steps_per_s": s["block_steps"] / (ms / 1e3),
                "same_log_z_as_builtin": lz_program == lz_builtin,
                "propagate_us_per_round": us, "propagate_launches_per_run": launches,
                "roofline": {"bound": "hbm", "kernel": "propagate (interpreter + live-prefix gather)",
                             "achieved": round(per_round / us / 1e3, 1), "peak": 8000.0, "unit": "GB/s",
                             "frac": round(per_round / us / 1e3 / 8000.0, 4),
                             "algorithmic_bytes_per_round": per_round,
                             "traffic": measured_traffic("propagate_program", T,
                                                         "traffic_program_lgssm100_n2p20.json")}})
    if cpu:
        from oracle import ppl_oracle as PO
        m = 512
        t0 = time.perf_counter()
        r = PO.ProgramRun(I.lgssm_program(y), m, 81)
        r.run_to_end()
        dt = time.perf_counter() - t0
        out["cpu_oracle_particle_rounds_per_s"] = m * T / dt
        out["cpu_oracle_sample"] = f"{m} particles, all {T} observations, source-level oracle, one thread, {dt:.1f} s"
    return out


def crbd_program_point(smc, ctx, I, tree, n: int = 1 << 20, runs: int = 2):
    """The Appendix CRBD model compiled from source (Sec. 4's path: static
    analysis, Alg. 2, frames, bytecode) on the headline tree, to set beside the
    built-in block table (the hand-written counterpart, as the paper sets
    compiled CorePPL beside RootPPL). Same model, other draws: the two log Z
    estimates agree within Monte Carlo error."""
    import torch
    from paper_2112_00364_amd import ppl
    img = ppl.compile_program(I.crbd_program(tree), stack_words=1024)
    model = smc.Model(ctx, {"kind": "program", "precision": 64, "program": img})
    run = smc.Run(model, n, 101)
    run.run_to_end()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(ctx.stream)
    zs = []
    for i in range(runs):
        run.reset(102 + i)
        run.run_to_end()
        zs.append(run.log_z())
    end.record(ctx.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / runs
    s = run.stats()
    run.reset(110)
    run.profile(True)
    run.run_to_end()
    kt = run.kernel_times()
    run.profile(False)
    run.close()
    model.close()
    return {"workload": f"crbd_program_yule{len(tree['age']) // 2 + 1}_n{n}", "particles": n, "runs": runs,
            "blocks": img.n_blocks, "instructions": int(len(img.code)), "frame_words": dict(img.frames),
            "stack_words": img.stack_words, "ms_per_run": ms, "status": s["status"], "rounds": s["round"],
            "log_z": zs, "kernel_ms_per_run": {k: round(v[0], 3) for k, v in kt.items()}}


def seir_program_point(smc, ctx, I, n: int = 1 << 16, days: int = 100, runs: int = 2):
    """The vector-borne disease model compiled from source, beside the built-in
    SEIR block table at FP64 state on the same data and seed (same bits)."""
    import torch
    from paper_2112_00364_amd import ppl
    y = I.seir_data(days, 6000)
    img = ppl.compile_program(I.seir_program(y), stack_words=2800)
    out = {"workload": f"seir_program_synthetic{days}d_n{n}", "particles": n, "days": days, "runs": runs,
           "blocks": img.n_blocks, "frame_words": dict(img.frames)}
    zs = {}
    for key, spec in (("program", {"kind": "program", "precision": 64, "program": img}),
                      ("builtin", I.seir_spec(y, 64))):
        model = smc.Model(ctx, spec)
        run = smc.Run(model, n, 61)
        run.run_to_end()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(ctx.stream)
        for i in range(runs):
            run.reset(62 + i)
            run.run_to_end()
        end.record(ctx.stream)
        torch.cuda.synchronize()
        out[f"{key}_ms_per_run"] = start.elapsed_time(end) / runs
        zs[key] = run.stats()["log_z"]
        run.close()
        model.close()
    out["same_log_z"] = zs["program"] == zs["builtin"]
    out["log_z"] = zs["program"]
    return out


def bucketing_point(smc, ctx, I, n: int = 1 << 20, T: int = 12, runs: int = 2):
    """Block bucketing on a program whose particles resume at two different
    blocks every round (regime_program: resampling inside the branch of a
    random regime, 24 Gamma draws of work per branch): complete runs without
    and with bucketing, and the autotuner's choice from a few timed rounds."""
    import torch
    from paper_2112_00364_amd import autotune, ppl
    img = ppl.compile_program(I.regime_program(I.branching_observations(T, 9)), stack_words=256)
    model = smc.Model(ctx, {"kind": "program", "precision": 64, "program": img})
    run = smc.Run(model, n, 91)
    out = {"workload": f"regime_program_T{T}_n{n}", "particles": n, "observations": T, "runs": runs}
    zs = {}
    for on in (False, True):
        run.set_bucketing(on)
        run.reset(91)
        run.run_to_end()
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        end = torch.cuda.Event(enable_timing=True)
        start.record(ctx.stream)
        for i in range(runs):
            run.reset(92 + i)
            run.run_to_end()
        end.record(ctx.stream)
        torch.cuda.synchronize()
        key = "on" if on else "off"
        out[f"ms_per_run_bucketing_{key}"] = start.elapsed_time(end) / runs
        zs[key] = run.stats()["log_z"]
        run.reset(95)
        run.profile(True)
        run.run_to_end()
        kt = run.kernel_times()
        run.profile(False)
        out[f"kernel_ms_per_run_bucketing_{key}"] = {k: round(v[0], 3) for k, v in kt.items()}
    out["same_log_z"] = zs["on"] == zs["off"]
    out["autotuner"] = autotune.choose_launch(run, 96, rounds=4, repeats=2)
    run.close()
    model.close()
    return out


def crbd_ds_point(smc, ctx, I, tree, n: int, tau: float = 0.5, runs: int = 3):
    """The paper's CRBD experiment with variance-reducing techniques: the
    headline tree with static delayed sampling (rates marginalised) and
    ESS-triggered resampling."""
    import torch
    model = smc.Model(ctx, dict(I.crbd_ds_spec(tree, precision=32), ess_threshold=tau))
    run = smc.Run(model, n, 71)
    run.run_to_end()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(ctx.stream)
    zs = []
    for i in range(runs):
        run.reset(72 + i)
        run.run_to_end()
    end.record(ctx.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / runs
    s = run.stats()
    run.close()
    model.close()
    return {"workload": f"crbd_ds_yule{TIPS}_n{n}", "ess_threshold": tau, "particles": n, "runs": runs,
            "ms_per_run": ms, "status": s["status"], "resampled_rounds": s["resamples"], "rounds": s["round"] + 1,
            "block_steps_per_s": s["block_steps"] / (ms / 1e3), "log_z_last": s["log_z"]}


def profile_steps(smc, model, n: int, seed: int, ms_per_run: float, byte_model: dict):
    """One profiled complete run (HIP events on the run's stream around every
    launch). Each bracketed launch pays a fixed event cost that the graph replay
    of the timed runs does not; it is estimated live as (bracketed time of the
    run - timed time per run) / launches and taken off every launch (the raw
    figures are kept beside). Returns the per-launch table, the per-step table
    (a split propagation is two launches per round) and the roofline of the
    dominant step; byte_model maps a step to its algorithmic bytes per round
    (a number, or a function of the run's round count)."""
    prof = smc.Run(model, n, seed)
    prof.profile(True)
    prof.run_to_end()
    times = prof.kernel_times()
    prof.close()
    launched = {k: v for k, v in times.items() if v[1] > 0}
    bracketed_ms = sum(ms for ms, _ in launched.values())
    n_launches = sum(c for _, c in launched.values())
    overhead_ms = max(0.0, (bracketed_ms - ms_per_run) / n_launches)
    kernels = {}
    for k, (ms, launches) in launched.items():
        raw_ms = ms / launches
        avg_ms = max(raw_ms - overhead_ms, 1e-6)
        kernels[k] = {"avg_us": avg_ms * 1e3, "bracketed_avg_us": raw_ms * 1e3,
                      "bracket_overhead_us": overhead_ms * 1e3, "launches": launches}
    steps = {}
    for step, parts in STEPS.items():
        got = [kernels[p] for p in parts if p in kernels]
        if not got:
            continue
        rounds_run = got[0]["launches"]
        avg_us = sum(g["avg_us"] * g["launches"] for g in got) / rounds_run
        entry = {"kernels": [p for p in parts if p in kernels], "avg_us_per_round": avg_us, "rounds": rounds_run}
        if step in byte_model:
            b = byte_model[step]
            b = b(rounds_run) if callable(b) else b
            entry.update({"alg_bytes_per_round": b, "achieved_GBs": b / (avg_us * 1e-6) / 1e9})
        steps[step] = entry
    dom = max((k for k in steps if "achieved_GBs" in steps[k]),
              key=lambda k: steps[k]["avg_us_per_round"] * steps[k]["rounds"])
    kd = steps[dom]
    roofline = {"bound": "hbm", "achieved": round(kd["achieved_GBs"], 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(kd["achieved_GBs"] / HBM_PEAK_GBS, 5), "traffic": None, "kernel": dom,
                "launches_per_round": kd["kernels"], "avg_launch_us": round(kd["avg_us_per_round"], 3)}
    return {"launches": kernels, "steps": steps}, roofline


def kalman_evidence(y, a=0.9, b=0.0, q=1.0, r=0.5, m0=0.0, s0=None) -> float:
    """Exact log evidence of the 1-D linear-Gaussian model by the Kalman
    filter (the reference the filter's log Z estimate approaches)."""
    if s0 is None:
        s0 = math.sqrt(q * q / (1.0 - a * a))
    m, P, lz = m0, s0 * s0, 0.0
    for yt in y:
        m, P = a * m + b, a * a * P + q * q
        S = P + r * r
        lz += -0.5 * (math.log(2.0 * math.pi * S) + (yt - m) ** 2 / S)
        K = P / S
        m, P = m + K * (yt - m), (1.0 - K) * P
    return lz


def kalman_point(smc, ctx, I, n: int = 1 << 16, T: int = 100, runs: int = 20):
    """The linear-Gaussian configuration: T = 100 observations simulated from
    the model (data seed 2000), 2^16 particles, FP32 state, FP64 log-weights,
    resampling every step. Complete runs replayed from a captured graph; log Z
    next to the exact Kalman evidence; the roofline of the dominant step."""
    import torch
    y = I.lgssm_data(T, 2000)
    model = smc.Model(ctx, I.lgssm_spec(y, 32))
    run = smc.Run(model, n, 1)
    run.run_to_end()
    for i in range(3):
        run.reset(300 + i)
        run.run_to_end()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(ctx.stream)
    for i in range(runs):
        run.reset(1 + i)
        run.run_to_end()
    end.record(ctx.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / runs
    s = run.stats()
    run.close()
    # per particle and round: anc 4 + gathered block 1 + gathered x 4 read, block 1 + x 4 + lw 8
    # written (round 0 writes only: 13); resampling reads lw 8 and writes anc 4 (not in the last round)
    byte_model = {"propagate": n * (13 + 22 * (T - 1)) / T, "resample": n * (8.0 + 4.0 * (T - 1) / T),
                  "reduce": n * 8.0 + n / 1024 * 16, "scan_anc": n * 12.0 * (T - 1) / T}
    kernels, roofline = profile_steps(smc, model, n, 4242, ms, byte_model)
    model.close()
    exact = kalman_evidence(y)
    return {"workload": f"lgssm_T{T}_n{n}", "particles": n, "observations": T, "runs": runs, "ms_per_run": ms,
            "block_steps_per_run": s["block_steps"], "block_steps_per_s": s["block_steps"] / (ms / 1e3),
            "log_z_last": s["log_z"], "kalman_log_evidence": exact, "roofline": roofline, "kernels": kernels}


def small_crbd_point(smc, ctx, I, runs: int = 50, cpu: bool = True):
    """The small CRBD configuration: 20-tip Yule tree (seed 1000), 1000
    particles, FP64 throughout: GPU run time and the oracle's time for the same
    run (single thread, same seed; the two log Z agree)."""
    import torch
    tree = I.yule_tree(20, 1000)
    spec = I.crbd_spec(tree, precision=64)
    model = smc.Model(ctx, spec)
    run = smc.Run(model, 1000, 1)
    run.run_to_end()
    run.reset(1)
    run.run_to_end()
    lz_gpu = run.stats()["log_z"]
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(ctx.stream)
    for i in range(runs):
        run.reset(1 + i)
        run.run_to_end()
    end.record(ctx.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / runs
    steps = run.stats()["block_steps"]
    run.close()
    model.close()
    out = {"workload": "crbd_yule20_n1000_fp64", "particles": 1000, "rounds": 39, "ms_per_run": ms,
           "block_steps_per_s": steps / (ms / 1e3), "log_z_seed1": lz_gpu}
    if cpu:
        from oracle import oracle as O
        t0 = time.perf_counter()
        ref = O.Run(spec, 1000, 1)
        ref.run_to_end()
        dt = time.perf_counter() - t0
        out.update({"cpu_oracle_ms_per_run": dt * 1e3, "cpu_oracle_block_steps_per_s": ref.block_steps / dt,
                    "cpu_oracle_log_z_seed1": ref.log_z, "cpu_oracle_cores": 1})
    return out


def large_point(smc, model, n: int, runs: int = 2, rounds: int = 2 * TIPS - 1, profile: bool = True):
    """Complete runs at a particle count whose buffers exceed the 256 MB
    Infinity Cache, so every round streams from HBM; with the roofline of the
    dominant step (the resampling takes the three-kernel form above 2^20)."""
    import torch
    run = smc.Run(model, n, 77)
    run.run_to_end()
    torch.cuda.synchronize()
    stream = model.ctx.stream
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for i in range(runs):
        run.reset(78 + i)
        assert run.run_to_end() == smc.FINISHED
    end.record(stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(end) / runs
    s = run.stats()
    run.close()
    out = {"particles": n, "runs": runs, "ms_per_run": ms, "block_steps_per_run": s["block_steps"],
           "block_steps_per_s": s["block_steps"] / (ms / 1e3)}
    if profile:
        byte_model = {k: bytes_per_launch(k, n, rounds) for k in ("propagate", "resample", "reduce", "scan_anc")}
        kernels, roofline = profile_steps(smc, model, n, 79, ms, byte_model)
        roofline["traffic"] = measured_traffic(roofline["kernel"], rounds, "traffic_crbd_yule256_n2p24.json")
        out.update({"roofline": roofline, "kernels": kernels})
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed SMC runs")
    ap.add_argument("--warmup", type=int, default=2, help="untimed SMC runs first")
    ap.add_argument("--cpu-particles", type=int, default=1 << 16,
                    help="particles in the CPU oracle's bounded sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event pass")
    ap.add_argument("--no-batched", action="store_true", help="skip the 512-run batched ClaDS leg")
    ap.add_argument("--serving-requests", type=int, default=250,
                    help="requests in the serving leg (0 skips it; the full stream is 2000)")
    ap.add_argument("--serving-rates", default="0.9",
                    help="arrival rates as multiples of the one-at-a-time service rate, comma-separated")
    ap.add_argument("--no-large", action="store_true", help="skip the 2^24-particle point")
    ap.add_argument("--no-kalman", action="store_true", help="skip the linear-Gaussian (Kalman) configuration")
    ap.add_argument("--no-small", action="store_true", help="skip the small CRBD configuration (and its oracle time)")
    ap.add_argument("--no-ess", action="store_true", help="skip the ESS-triggered point")
    ap.add_argument("--no-seir", action="store_true", help="skip the vector-borne disease (SEIR) point")
    ap.add_argument("--seir-particles", type=int, default=1 << 18,
                    help="particles of the SEIR point (2^16 puts one wavefront on each SIMD)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched leg: keep the default work-group size (no probe batches)")
    ap.add_argument("--no-program", action="store_true", help="skip the compiled-program point")
    ap.add_argument("--no-bucketing", action="store_true", help="skip the block-bucketing point")
    ap.add_argument("--no-crbd-program", action="store_true", help="skip the compiled CRBD point")
    ap.add_argument("--no-tail-call", action="store_true",
                    help="compiled-program point: skip the tail-call form (profiles of the stack-growing form)")
    ap.add_argument("--serving-budget-gb", type=float, default=32.0)
    ap.add_argument("--serving-mode", choices=["single", "by-kind"], default="by-kind",
                    help="serving leg: one batch for all requests, or one batch per model kind on its own stream")
    ap.add_argument("--serving-alone-out", default=None,
                    help="serving leg: write the back-to-back one-at-a-time pass to this JSON file")
    ap.add_argument("--serving-alone-in", default=None,
                    help="serving leg: take the one-at-a-time pass from this JSON file instead of measuring it")
    ap.add_argument("--only", choices=["ess", "crbd_ds", "seir", "seir_program", "bucketing", "large", "kalman",
                                       "small", "batched", "serving", "owned"],
                    help="run this one leg alone (no headline runs) and print its record: "
                         "for kernel traces that hold one workload")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first copy 256 MiB device-to-device 3 times (a known-size kernel for HBM counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the SMC path here runs on a single MI355X; "
              "independent runs shard across GPUs without communication", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2112_00364_amd import inputs as I
    from paper_2112_00364_amd import smc

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    tree = I.yule_tree(TIPS, TREE_SEED)
    spec = I.crbd_spec(tree, precision=32)
    rounds = 2 * TIPS - 1
    ctx = smc.Context(0)
    if args.only:
        rates = [float(x) for x in args.serving_rates.split(",") if x]
        legs = {"ess": lambda: ess_point(smc, ctx, spec, N_PARTICLES),
                "crbd_ds": lambda: crbd_ds_point(smc, ctx, I, tree, N_PARTICLES),
                "seir": lambda: seir_point(smc, ctx, I, n=args.seir_particles, cpu=False),
                "seir_program": lambda: seir_program_point(smc, ctx, I),
                "bucketing": lambda: bucketing_point(smc, ctx, I),
                "large": lambda: large_point(smc, smc.Model(ctx, spec), 1 << 24, runs=1, profile=not args.no_profile),
                "kalman": lambda: kalman_point(smc, ctx, I),
                "small": lambda: small_crbd_point(smc, ctx, I, cpu=not args.no_cpu_baseline),
                "batched": lambda: batched_clads(ctx, smc, I, tune=not args.no_autotune),
                "owned": lambda: owned_point(ctx, smc, I),
                "serving": lambda: serving(ctx, smc, args.serving_requests, int(args.serving_budget_gb * 2**30),
                                           rates, args.serving_alone_in, args.serving_alone_out,
                                           args.serving_mode)}
        print(f"{args.only} leg alone", file=sys.stderr, flush=True)
        print(json.dumps({"leg": args.only, args.only: legs[args.only]()}), flush=True)
        return
    model = smc.Model(ctx, spec)
    stream = ctx.stream
    # One run's buffers, reused: smc_reset re-initialises them on the device and
    # smc_run_to_end replays the captured graph of all rounds.
    run = smc.Run(model, N_PARTICLES, 1)
    torch.cuda.synchronize()
    for i in range(args.warmup):
        run.reset(1000 + i)
        run.run_to_end()
    torch.cuda.synchronize()

    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    steps_total = 0
    log_zs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start.record(stream)
    for i in range(args.steps):
        run.reset(1 + i)
        st = run.run_to_end()
        assert st == smc.FINISHED, st
    end.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = start.elapsed_time(end)
    # every timed run executed all its blocks: N particles x 511 canonical blocks
    for i in range(args.steps):
        steps_total += N_PARTICLES * rounds
    s = run.stats()
    assert s["status"] == smc.FINISHED and s["block_steps"] == N_PARTICLES * rounds, s
    log_zs.append(s["log_z"])
    run.close()
    ms_per_step = gpu_ms / args.steps
    value = steps_total / (gpu_ms / 1e3)

    roofline = None
    kernels = None
    if not args.no_profile:
        byte_model = {k: bytes_per_launch(k, N_PARTICLES, rounds) for k in ("propagate", "resample", "reduce",
                                                                             "scan_anc")}
        kernels, roofline = profile_steps(smc, model, N_PARTICLES, 12345, ms_per_step, byte_model)
        roofline["traffic"] = measured_traffic(roofline["kernel"], rounds)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-block-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "particle_rounds_per_s": N_PARTICLES * rounds * args.steps / (gpu_ms / 1e3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"crbd_yule{TIPS}_n2^20", "tips": TIPS, "tree_seed": TREE_SEED,
                   "particles": N_PARTICLES, "rounds_per_run": rounds, "state": "f32",
                   "log_weights": "f64", "step": "one complete SMC run"},
        "roofline": roofline,
        "kernels": kernels,
        "wall_s_timed": wall,
        "log_z": log_zs,
    }
    if not args.no_kalman:
        print("linear-Gaussian configuration", file=sys.stderr, flush=True)
        out["kalman"] = kalman_point(smc, ctx, I)
    if not args.no_small:
        print("small CRBD configuration", file=sys.stderr, flush=True)
        out["small"] = small_crbd_point(smc, ctx, I, cpu=not args.no_cpu_baseline)
    if not args.no_ess:
        print("ESS-triggered point", file=sys.stderr, flush=True)
        out["ess"] = ess_point(smc, ctx, spec, N_PARTICLES)
    if not args.no_ess:
        print("delayed-sampling CRBD point", file=sys.stderr, flush=True)
        out["crbd_ds"] = crbd_ds_point(smc, ctx, I, tree, N_PARTICLES)
    if not args.no_seir:
        print("SEIR point", file=sys.stderr, flush=True)
        out["seir"] = seir_point(smc, ctx, I, n=args.seir_particles, cpu=not args.no_cpu_baseline)
    if not args.no_program:
        print("compiled-program point", file=sys.stderr, flush=True)
        out["program"] = program_point(smc, ctx, I, cpu=not args.no_cpu_baseline, tail=not args.no_tail_call)
    if not args.no_seir and not args.no_program:
        print("compiled SEIR point", file=sys.stderr, flush=True)
        out["seir_program"] = seir_program_point(smc, ctx, I)
    if not args.no_crbd_program:
        print("compiled CRBD point", file=sys.stderr, flush=True)
        out["crbd_program"] = crbd_program_point(smc, ctx, I, tree)
        out["crbd_program"]["builtin_ms_per_run"] = ms_per_step
        out["crbd_program"]["builtin_log_z"] = log_zs
    if not args.no_bucketing:
        print("block-bucketing point", file=sys.stderr, flush=True)
        out["bucketing"] = bucketing_point(smc, ctx, I)
    if not args.no_large:
        print("2^24-particle point", file=sys.stderr, flush=True)
        out["large"] = large_point(smc, model, 1 << 24)
    if not args.no_batched:
        print("batched leg", file=sys.stderr, flush=True)
        out["batched"] = batched_clads(ctx, smc, I, tune=not args.no_autotune)
    if args.serving_requests > 0:
        print("serving leg", file=sys.stderr, flush=True)
        rates = [float(x) for x in args.serving_rates.split(",") if x]
        out["serving"] = serving(ctx, smc, args.serving_requests, int(args.serving_budget_gb * 2**30), rates,
                                 args.serving_alone_in, args.serving_alone_out, args.serving_mode)
    if not args.no_cpu_baseline:
        print("cpu baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(spec, args.cpu_particles)
        if "batched" in out:
            print("cpu baseline of the batched leg (all cores)", file=sys.stderr, flush=True)
            out["batched"]["cpu_oracle_all_cores"] = batched_clads_cpu()
    print(json.dumps(out))
    model.close()
    ctx.close()


if __name__ == "__main__":
    main()
