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
