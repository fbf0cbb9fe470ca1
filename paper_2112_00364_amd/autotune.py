"""Launch-option autotuning by measurement (host side).

Two launch options of a single run change no result, only the time:
* the propagation work-group size (smc_set_workgroup: 128 or 256 lanes);
  smaller groups schedule divergent blocks more finely, larger ones amortise
  the per-group work and suit long uniform blocks;
* block bucketing (smc_set_bucketing), which sorts the particle slots by the
  block each resumes at before every propagation: it pays off when the
  particles of a wavefront would otherwise run different blocks, and costs
  three small launches per round when they would not.
Which choice wins is a property of the model, its data and the particle
count, so it is made by timing: the first rounds of the run are executed
under each candidate (the run is reset in between, so all see the same
particles), and the fastest is kept.
"""
from __future__ import annotations

import json
import math
import os


def _time_rounds(run, seed: int, rounds: int) -> float:
    import torch
    stream = run.model.ctx.stream
    run.reset(seed)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(rounds):
        run.step()
        run.resample()
    end.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(end)


def _apply(run, option):
    lanes, bucketing = option
    if lanes is not None:
        run.set_workgroup(lanes)
    run.set_bucketing(bucketing)


def choose_launch(run, seed: int, rounds: int = 6, repeats: int = 2,
                  lanes=(128, 256), bucketing=(False, True)) -> dict:
    """Times `rounds` rounds of `run` (from a reset with `seed`) under every
    (work-group lanes, bucketing) candidate, `repeats` times each (the best
    counts), leaves the fastest setting on and the run reset to `seed`.
    Returns the chosen option and every measurement (ms)."""
    times = {}
    for l in lanes:
        for b in bucketing:
            _apply(run, (l, b))
            _time_rounds(run, seed, 1)  # first use of the setting: allocation, code load
            times[(l, b)] = min(_time_rounds(run, seed, rounds) for _ in range(repeats))
    best = min(times, key=times.get)
    _apply(run, best)
    run.reset(seed)
    return {"lanes": best[0], "bucketing": best[1], "rounds": rounds,
            "ms": {f"lanes{l}_bucketing_{'on' if b else 'off'}": t for (l, b), t in times.items()}}


def choose_bucketing(run, seed: int, rounds: int = 6, repeats: int = 2) -> dict:
    """Bucketing alone, at the run's current work-group size."""
    r = choose_launch(run, seed, rounds, repeats, lanes=(None,))
    return {"bucketing": r["bucketing"], "ms_off": r["ms"]["lanesNone_bucketing_off"],
            "ms_on": r["ms"]["lanesNone_bucketing_on"], "rounds": rounds}


# --- batches -----------------------------------------------------------------------------

def shape_key(kind: str, precision: int, n: int, tips: int) -> str:
    """Cache key of a run shape: model kind, precision, particle count (power
    of two above) and tree size (power of two above; 0 without a tree)."""
    n2 = 1 << max(0, math.ceil(math.log2(max(n, 1))))
    t2 = 1 << max(0, math.ceil(math.log2(tips))) if tips else 0
    return f"{kind}/fp{precision}/n{n2}/tips{t2}"


class LaunchCache:
    """Chosen launch options per run shape, kept in a JSON file: {key:
    {"lanes": 128|256, "ms": {...}}}. A shape not in the file is timed once
    (choose_batch_workgroup) and the choice written back."""

    def __init__(self, path: str | None = None):
        self.path = path or os.path.join(os.path.expanduser("~"), ".cache", "pcfgsmc_launch.json")
        self.entries = {}
        if os.path.exists(self.path):
            try:
                self.entries = json.load(open(self.path))
            except (OSError, ValueError):
                self.entries = {}

    def get(self, key: str):
        return self.entries.get(key)

    def put(self, key: str, entry: dict):
        self.entries[key] = entry
        d = os.path.dirname(self.path)
        if d:
            os.makedirs(d, exist_ok=True)
        tmp = f"{self.path}.{os.getpid()}.tmp"
        with open(tmp, "w") as f:
            json.dump(self.entries, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def choose_batch_workgroup(ctx, model, n: int, seeds, rounds: int = 8, ticks: int = 2,
                           lanes=(128, 256), owned: bool = False) -> dict:
    """Times a probe batch of len(seeds) runs of `model` (n particles each)
    advanced `ticks` ticks of `rounds` rounds under each launch option -- each
    propagation work-group size of the segmented launches and, with `owned`,
    one work-group owning each run -- from the same initial particles every
    time (fresh batches, same seeds); the fastest option wins. The probe's
    results are discarded."""
    import torch
    from . import smc
    options = [(f"lanes{l}", l, False) for l in lanes] + ([("owned", 256, True)] if owned else [])
    times = {}
    for name, l, own in options:
        best = None
        for _ in range(2):
            b = smc.Batch(ctx)
            slots = [b.add(model, n, s) for s in seeds]
            for slot in slots:
                if own:
                    b.set_owned(slot)
                else:
                    b.set_workgroup(slot, l)
            b.tick(0)  # tables
            torch.cuda.synchronize()
            start = torch.cuda.Event(enable_timing=True)
            end = torch.cuda.Event(enable_timing=True)
            start.record(ctx.stream)
            for _ in range(ticks):
                b.tick(rounds)
            end.record(ctx.stream)
            torch.cuda.synchronize()
            t = start.elapsed_time(end)
            best = t if best is None else min(best, t)
            b.close()
        times[name] = best
    choice = min(times, key=times.get)
    lanes_of = {name: l for name, l, _ in options}
    return {"lanes": lanes_of[choice], "owned": choice == "owned", "rounds": rounds, "ticks": ticks,
            "runs": len(seeds), "ms": times}


# Largest run one work-group may own (smc_batch_set_owned).
OWNED_MAX_PARTICLES = 4096


def batch_launch(cache: LaunchCache, ctx, model, kind: str, precision: int, n: int, tips: int,
                 probe_runs: int = 8) -> dict:
    """The cached launch option for this run shape, tuned on first use:
    {"lanes": 128 or 256, "owned": bool}. Owning by a work-group is tried for
    built-in models of at most OWNED_MAX_PARTICLES particles."""
    key = shape_key(kind, precision, n, tips)
    hit = cache.get(key)
    if hit is None or "owned" not in hit:
        can_own = kind != "program" and n <= OWNED_MAX_PARTICLES
        hit = choose_batch_workgroup(ctx, model, n, seeds=list(range(90001, 90001 + probe_runs)), owned=can_own)
        cache.put(key, hit)
    return {"lanes": int(hit["lanes"]), "owned": bool(hit["owned"])}


def apply_batch_launch(batch, slot: int, choice: dict):
    """Applies a batch_launch choice to one run of a batch."""
    if choice["owned"]:
        batch.set_owned(slot)
    else:
        batch.set_workgroup(slot, choice["lanes"])


def batch_workgroup(cache: LaunchCache, ctx, model, kind: str, precision: int, n: int, tips: int,
                    probe_runs: int = 8) -> int:
    """The cached work-group size of the segmented launches for this run shape."""
    return batch_launch(cache, ctx, model, kind, precision, n, tips, probe_runs)["lanes"]
