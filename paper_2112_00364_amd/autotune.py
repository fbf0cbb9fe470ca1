"""Launch-option autotuning by measurement (host side).

Block bucketing (smc_set_bucketing) sorts a run's particle slots by the block
each resumes at before every propagation. It changes no result, only the
time: it pays off when the particles of a wavefront would otherwise run
different blocks, and costs three small launches per round when they would
not. Which case holds is a property of the program and its data, so the
choice is made by timing: the first rounds of the run are executed with and
without bucketing (the run is reset in between, so both see the same
particles), and the faster setting is kept. Work-group sizes per model kind
were chosen the same way, offline, and are fixed in the library.
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


def choose_bucketing(run, seed: int, rounds: int = 6, repeats: int = 2) -> dict:
    """Times `rounds` rounds of `run` (from a reset with `seed`) without and with
    bucketing, `repeats` times each (the best counts), leaves the faster setting
    on and the run reset to `seed`. Returns the measurements and the choice."""
    times = {}
    for on in (False, True):
        run.set_bucketing(on)
        _time_rounds(run, seed, 1)  # first use of the setting: allocation, code load
        times[on] = min(_time_rounds(run, seed, rounds) for _ in range(repeats))
    best = times[True] < times[False]
    run.set_bucketing(best)
    run.reset(seed)
    return {"bucketing": best, "ms_off": times[False], "ms_on": times[True], "rounds": rounds}
