"""Serving loop: continuous batching of SMC inference requests on one GPU.

Requests (a model specification, a particle count and a seed) arrive over
time. The server admits a request when its particle memory fits the budget,
adds it to the device-resident batch (smc_batch_add), advances every live run
by a few rounds per tick (one launch per kernel for all runs), retires runs as
they finish and records latency = completion - arrival. The one-at-a-time
baseline serves the same requests first-come first-served, each as a plain
smc_init + smc_run_to_end on the same kernels.

All SMC work runs in libpcfgsmc.so; this module is host-side scheduling only.
"""
from __future__ import annotations

import collections
import sys
import time

import numpy as np

from . import inputs as I
from . import smc


def footprint_bytes(kind: str, n: int, precision: int, stack_depth: int = 0) -> int:
    """Device bytes of one run: double-buffered block + state (+ ClaDS rate
    stack), log-weights, ancestors, the propagation's group slots and the
    reduction's tile sums (+ ClaDS side-lineage stacks: 32 levels of 17 bytes
    per particle)."""
    real = {"geometric": 0, "lgssm": 1, "crbd": 2, "clads": 4, "seir": 6}[kind]
    ints = {"geometric": 1, "seir": 9}.get(kind, 0)
    rb = 4 if precision == 32 else 8
    per = 2 * (1 + real * rb + 4 * ints + (stack_depth * rb if kind == "clads" else 0)) + 8 + 4
    if kind == "clads":
        per += 32 * 17
    return n * per + 1024 + (n + 1023) // 1024 * 24 + 512


def clads_stack_depth(tree) -> int:
    cur = deepest = 1
    left = tree["left"]
    for node in range(1, len(left)):
        cur = cur + 1 if left[node] >= 0 else max(cur - 1, 0)
        deepest = max(deepest, cur)
    return deepest + 1


def make_requests(n_requests: int, seed: int, rate_per_s: float, precision: int = 32):
    """The serving workload with its trees built up front (inputs, not serving work)."""
    reqs = I.request_stream(n_requests, seed, rate_per_s)
    for r in reqs:
        tree = I.yule_tree(r["tips"], r["tree_seed"])
        if r["kind"] == "crbd":
            r["spec"] = I.crbd_spec(tree, precision=precision)
            r["depth"] = 0
        else:
            r["spec"] = I.clads_spec(tree, precision=precision)
            r["depth"] = clads_stack_depth(tree)
        r["rounds"] = 2 * r["tips"] - 1
        r["block_steps"] = r["n"] * r["rounds"]
        r["bytes"] = footprint_bytes(r["kind"], r["n"], precision, r["depth"])
    return reqs


def rescale_arrivals(reqs, rate_per_s: float, seed: int):
    """Same requests, Poisson arrivals at a new rate."""
    rng = np.random.default_rng(seed)
    t = 0.0
    for r in reqs:
        t += rng.exponential(1.0 / rate_per_s)
        r["arrival"] = t
    return reqs


def _progress(msg: str):
    print(msg, file=sys.stderr, flush=True)


def serve_one_at_a_time(ctx: smc.Context, reqs, honour_arrivals=True, log_every=100):
    """FIFO, one plain run at a time."""
    import torch
    out = []
    t0 = time.perf_counter()
    for k, r in enumerate(reqs):
        if log_every and k % log_every == 0:
            _progress(f"one-at-a-time: request {k}/{len(reqs)} at {time.perf_counter() - t0:.1f} s")
        now = time.perf_counter() - t0
        if honour_arrivals and r["arrival"] > now:
            time.sleep(r["arrival"] - now)
        start = time.perf_counter() - t0
        model = smc.Model(ctx, r["spec"])
        run = smc.Run(model, r["n"], r["seed"])
        st = run.run_to_end()
        lz = run.log_z()
        done = time.perf_counter() - t0
        steps = run.stats()["block_steps"]
        run.close()
        model.close()
        out.append({"id": r["id"], "arrival": r["arrival"], "start": start, "done": done, "log_z": lz,
                    "status": st, "block_steps": steps})
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def fifo_replay(served, reqs):
    """One-at-a-time FIFO latencies of a stream from measured service times.
    `served` holds each request served alone back to back (serve_one_at_a_time
    with honour_arrivals=False: start and done of its plain run on the GPU);
    with the arrivals now in `reqs`, request i starts at max(arrival_i,
    done_{i-1}) and takes its measured service time. This is the real-time
    FIFO replay without the idle waits, so one measured pass serves every
    arrival rate. Returns (results, makespan)."""
    service = {r["id"]: (r["done"] - r["start"], r) for r in served}
    out = []
    free_at = 0.0
    for q in sorted(reqs, key=lambda x: x["arrival"]):
        dt, r = service[q["id"]]
        start = max(q["arrival"], free_at)
        free_at = start + dt
        out.append(dict(r, arrival=q["arrival"], start=start, done=free_at))
    return out, free_at


def serve_batched(ctx: smc.Context, reqs, memory_budget: int, rounds_per_tick: int = 8,
                  max_live: int = 256, honour_arrivals=True, log_every=100):
    """Continuous batching: admit while memory and slots allow, tick, retire.
    An admission whose allocation fails (SMC_ERR_OOM) waits for the next
    retirement and is tried again; serve_batched.last_oom_waits counts them."""
    pending = collections.deque(sorted(reqs, key=lambda r: r["arrival"]))
    batch = smc.Batch(ctx)
    live = {}       # slot -> (request, model, admitted time)
    used = 0
    oom_waits = 0   # admissions postponed because an allocation failed
    out = []
    t0 = time.perf_counter()
    while pending or live:
        now = time.perf_counter() - t0
        # admission: arrived requests in order while their particle memory fits
        while pending and (not honour_arrivals or pending[0]["arrival"] <= now):
            r = pending[0]
            if live and (used + r["bytes"] > memory_budget or len(live) >= max_live):
                break
            model = None
            try:
                model = smc.Model(ctx, r["spec"])
                slot = batch.add(model, r["n"], r["seed"])
            except smc.SMCError as e:
                if model is not None:
                    model.close()
                # the device is fuller than the budget says: wait for live runs
                # to retire and try again (a request that fails alone cannot fit)
                if e.code != smc.ERR_OOM or not live:
                    raise
                oom_waits += 1
                break
            pending.popleft()
            live[slot] = (r, model, time.perf_counter() - t0)
            used += r["bytes"]
        if not live:
            if pending:
                time.sleep(max(0.0, pending[0]["arrival"] - (time.perf_counter() - t0)))
            continue
        batch.tick(rounds_per_tick)
        done, lz, st, steps = batch.poll()
        now = time.perf_counter() - t0
        for slot in list(live):
            if done[slot]:
                r, model, admitted = live.pop(slot)
                out.append({"id": r["id"], "arrival": r["arrival"], "start": admitted, "done": now,
                            "log_z": float(lz[slot]), "status": int(st[slot]), "block_steps": int(steps[slot])})
                batch.retire(slot)
                model.close()
                used -= r["bytes"]
                if log_every and len(out) % log_every == 0:
                    _progress(f"batched: {len(out)}/{len(reqs)} done, {len(live)} live at {now:.1f} s")
    batch.close()
    serve_batched.last_oom_waits = oom_waits
    return out, time.perf_counter() - t0


def serve_batched_by_kind(ctxs: dict, reg_ctx, reqs, memory_budget: int, rounds_per_tick: int = 8,
                          max_live: int = 256, honour_arrivals=True, log_every=100):
    """Continuous batching with one batch per model kind, each on its own
    context (its own HIP stream): a tick of one batch does not wait for the
    other's, so requests of a light model are not held by a heavy one's long
    chains. A batch is ticked again as soon as its previous tick has finished
    (an event on its stream, queried without blocking); admission as in
    serve_batched, against one memory budget for both. ctxs maps a request kind
    to the Context its batch runs on; models are registered on reg_ctx, whose
    stream stays idle, so an admission never waits for a running tick."""
    import torch
    pending = collections.deque(sorted(reqs, key=lambda r: r["arrival"]))
    kinds = sorted(ctxs)
    batches = {k: smc.Batch(ctxs[k]) for k in kinds}
    live = {k: {} for k in kinds}      # kind -> slot -> (request, model, admitted time)
    in_flight = {k: None for k in kinds}  # kind -> event recorded after its last tick
    used = 0
    out = []
    t0 = time.perf_counter()
    while pending or any(live[k] for k in kinds):
        now = time.perf_counter() - t0
        n_live = sum(len(live[k]) for k in kinds)
        while pending and (not honour_arrivals or pending[0]["arrival"] <= now):
            r = pending[0]
            if n_live and (used + r["bytes"] > memory_budget or n_live >= max_live):
                break
            k = r["kind"]
            model = None
            try:
                model = smc.Model(reg_ctx, r["spec"])
                slot = batches[k].add(model, r["n"], r["seed"])
            except smc.SMCError as e:
                if model is not None:
                    model.close()
                if e.code != smc.ERR_OOM or not n_live:
                    raise
                break
            pending.popleft()
            live[k][slot] = (r, model, time.perf_counter() - t0)
            used += r["bytes"]
            n_live += 1
        progressed = False
        for k in kinds:
            ev = in_flight[k]
            if ev is not None:
                if not ev.query():
                    continue
                in_flight[k] = None
                done, lz, st, steps = batches[k].poll()
                now = time.perf_counter() - t0
                for slot in list(live[k]):
                    if done[slot]:
                        r, model, admitted = live[k].pop(slot)
                        out.append({"id": r["id"], "arrival": r["arrival"], "start": admitted, "done": now,
                                    "log_z": float(lz[slot]), "status": int(st[slot]),
                                    "block_steps": int(steps[slot])})
                        batches[k].retire(slot)
                        model.close()
                        used -= r["bytes"]
                        if log_every and len(out) % log_every == 0:
                            _progress(f"batched by kind: {len(out)}/{len(reqs)} done at {now:.1f} s")
                progressed = True
            if live[k] and in_flight[k] is None:
                batches[k].tick(rounds_per_tick)
                ev = torch.cuda.Event()
                ev.record(ctxs[k].stream)
                in_flight[k] = ev
                progressed = True
        if not progressed:
            if not any(live[k] for k in kinds) and pending:
                time.sleep(max(0.0, pending[0]["arrival"] - (time.perf_counter() - t0)))
            else:
                time.sleep(0.0002)
    for k in kinds:
        batches[k].close()
    return out, time.perf_counter() - t0


def summarize(results, makespan: float) -> dict:
    lat = np.array([r["done"] - r["arrival"] for r in results])
    steps = sum(r["block_steps"] for r in results)
    return {"requests": len(results), "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)), "mean_latency_s": float(lat.mean()),
            "makespan_s": makespan, "block_steps": int(steps), "block_steps_per_s": steps / makespan,
            "failed": int(sum(1 for r in results if r["status"] != smc.FINISHED))}
