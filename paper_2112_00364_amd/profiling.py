"""Summaries of rocprofv3 output for the library's kernels (host-side tooling).

rocprofv3 writes an SQLite database per run (``<dir>/<name>_results.db``).
This module turns one into the short text records kept with the benchmark:

* ``trace``: per-kernel launch count and durations from a ``--kernel-trace``
  run, as a markdown table;
* ``counters``: per-kernel means of every counter of one ``--pmc`` run, per
  dispatch and per wavefront, as a markdown table;
* ``traffic``: HBM bytes per launch from two ``--pmc`` runs (``FETCH_SIZE``,
  then ``WRITE_SIZE``, KiB per dispatch). Each counter is scaled by what it
  reads for a device-to-device copy of known size in the same run (the
  ``--calibrate-copy`` option of bench.py copies 256 MiB three times first),
  so the figures are bytes, whatever unit quirks the counters have.

Usage:
  python -m paper_2112_00364_amd.profiling trace DB OUT.md --cmd "COMMAND"
  python -m paper_2112_00364_amd.profiling counters DB OUT.md --cmd "COMMAND"
  python -m paper_2112_00364_amd.profiling traffic FETCH_DB WRITE_DB OUT.json \
      --cmd-fetch "COMMAND" --cmd-write "COMMAND" --source-sha SHA
"""
from __future__ import annotations

import argparse
import collections
import json
import sqlite3

# Kernel-name prefixes -> the names bench.py reports.
KERNELS = {
    "k_propagate_one<6": "propagate_program",
    "k_propagate": "propagate",
    "k_maxkey": "maxkey",
    "k_fold_sums": "fold_sums",
    "k_reduce": "reduce",
    "k_scan_anc": "scan_anc",
}
CALIBRATION_BYTES = 256 << 20
CALIBRATION_KERNEL = "__amd_rocclr_copyBuffer"


def short_name(kernel_name: str) -> str:
    """'void pcfg::k_propagate_one<2, float>(pcfg::RunDev)' -> 'k_propagate_one<2, float>'."""
    name = kernel_name.split("(")[0]
    if name.startswith("void "):
        name = name[5:]
    return name.replace("pcfg::", "")


def bench_kernel(kernel_name: str):
    s = short_name(kernel_name)
    for prefix, k in KERNELS.items():
        if s.startswith(prefix):
            return k
    return None


def trace_rows(db: str):
    con = sqlite3.connect(db)
    q = ("select name, count(*), avg(duration), min(duration), max(duration), sum(duration) "
         "from kernels group by name order by sum(duration) desc")
    return [(short_name(n), c, a, mn, mx, s) for n, c, a, mn, mx, s in con.execute(q)]


def trace_markdown(db: str, title: str, cmd: str) -> str:
    rows = trace_rows(db)
    total = sum(r[5] for r in rows) or 1.0
    out = [f"# rocprofv3 kernel trace: {title}", "", "Command (repository root):", "", "```", cmd, "```", "",
           "| kernel | launches | avg us | min us | max us | total ms | share |",
           "|---|---|---|---|---|---|---|"]
    for n, c, a, mn, mx, s in rows:
        out.append(f"| {n} | {c} | {a / 1e3:.2f} | {mn / 1e3:.2f} | {mx / 1e3:.2f} | {s / 1e6:.3f} | "
                   f"{100 * s / total:.1f}% |")
    return "\n".join(out) + "\n"


def counter_per_dispatch(db: str, counter: str):
    """[(dispatch id, kernel name, summed counter value)] in dispatch order."""
    con = sqlite3.connect(db)
    acc = collections.defaultdict(float)
    names = {}
    q = "select dispatch_id, kernel_name, value from counters_collection where counter_name = ?"
    for d, k, v in con.execute(q, (counter,)):
        acc[d] += v
        names[d] = k
    return [(d, names[d], acc[d]) for d in sorted(acc)]


def counters_markdown(db: str, title: str, cmd: str) -> str:
    """Mean of each counter per dispatch (and per wavefront when SQ_WAVES was
    collected) for the library's kernels."""
    con = sqlite3.connect(db)
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for d, k, c, v in con.execute("select dispatch_id, kernel_name, counter_name, value from counters_collection"):
        if bench_kernel(k) is None:
            continue
        per[d][c] += v
        names[d] = short_name(k)
    by_kernel = collections.defaultdict(list)
    for d in per:
        by_kernel[names[d]].append(per[d])
    counters = sorted({c for d in per for c in per[d]})
    out = [f"# rocprofv3 counters: {title}", "", "Command (repository root):", "", "```", cmd, "```", "",
           "Mean per dispatch (per wavefront in brackets when SQ_WAVES was collected).", "",
           "| kernel | dispatches | " + " | ".join(counters) + " |", "|---|---|" + "---|" * len(counters)]
    for name, ds in sorted(by_kernel.items()):
        mean = {c: sum(d.get(c, 0.0) for d in ds) / len(ds) for c in counters}
        waves = mean.get("SQ_WAVES", 0.0)
        cells = []
        for c in counters:
            cell = f"{mean[c]:.4g}"
            if waves > 0 and c.startswith("SQ_") and c not in ("SQ_WAVES", "SQ_BUSY_CYCLES"):
                cell += f" ({mean[c] / waves:.4g})"
            cells.append(cell)
        out.append(f"| {name} | {len(ds)} | " + " | ".join(cells) + " |")
    return "\n".join(out) + "\n"


def calibration_scale(rows) -> float:
    """Bytes per counter unit: the known copy size over the largest copy dispatch's reading."""
    copies = [v for _, k, v in rows if short_name(k) == CALIBRATION_KERNEL]
    if not copies or max(copies) <= 0:
        raise ValueError("no calibration copy in this run (use bench.py --calibrate-copy)")
    return CALIBRATION_BYTES / max(copies)


def _launch_stats(values):
    """Mean bytes over the launches that did work. A run driven by
    smc_run_to_end checks termination every few rounds, so it can end with
    launches that only read the run's status; dispatches below 1% of the
    kernel's median are counted apart as idle."""
    med = sorted(values)[len(values) // 2]
    busy = [v for v in values if v >= 0.01 * med]
    return {"launches": len(busy), "idle_launches": len(values) - len(busy),
            "bytes_per_launch": sum(busy) / len(busy), "bytes_total": sum(values)}


def traffic(fetch_db: str, write_db: str) -> dict:
    result = {}
    for counter, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        rows = counter_per_dispatch(db, counter)
        scale = calibration_scale(rows)
        per = collections.defaultdict(list)
        for _, k, v in rows:
            b = bench_kernel(k)
            if b is not None:
                per[b].append(v * scale)
        result[counter] = {"bytes_per_counter_unit": scale,
                           "kernels": {k: _launch_stats(v) for k, v in per.items()}}
    kernels = {}
    for k in result["FETCH_SIZE"]["kernels"]:
        f = result["FETCH_SIZE"]["kernels"][k]["bytes_per_launch"]
        w = result["WRITE_SIZE"]["kernels"].get(k, {}).get("bytes_per_launch", 0.0)
        total = (result["FETCH_SIZE"]["kernels"][k]["bytes_total"] +
                 result["WRITE_SIZE"]["kernels"].get(k, {}).get("bytes_total", 0.0))
        kernels[k] = {"fetch_bytes_per_launch": f, "write_bytes_per_launch": w, "hbm_bytes_per_launch": f + w,
                      "hbm_bytes_total": total,
                      "launches": result["FETCH_SIZE"]["kernels"][k]["launches"],
                      "idle_launches": result["FETCH_SIZE"]["kernels"][k]["idle_launches"]}
    return {"kernels": kernels,
            "fetch_scale": result["FETCH_SIZE"]["bytes_per_counter_unit"],
            "write_scale": result["WRITE_SIZE"]["bytes_per_counter_unit"]}


def main(argv=None):
    ap = argparse.ArgumentParser(description="summaries of rocprofv3 databases")
    sub = ap.add_subparsers(dest="what", required=True)
    t = sub.add_parser("trace")
    t.add_argument("db")
    t.add_argument("out")
    t.add_argument("--cmd", required=True)
    t.add_argument("--title", default=None)
    c = sub.add_parser("counters")
    c.add_argument("db")
    c.add_argument("out")
    c.add_argument("--cmd", required=True)
    c.add_argument("--title", default=None)
    f = sub.add_parser("traffic")
    f.add_argument("fetch_db")
    f.add_argument("write_db")
    f.add_argument("out")
    f.add_argument("--cmd-fetch", required=True)
    f.add_argument("--cmd-write", required=True)
    f.add_argument("--source-sha", required=True)
    f.add_argument("--runs", type=int, default=1, help="complete runs the profiled command made")
    a = ap.parse_args(argv)
    if a.what in ("trace", "counters"):
        title = a.title or a.out.rsplit("/", 1)[-1].rsplit(".", 1)[0]
        make = trace_markdown if a.what == "trace" else counters_markdown
        text = make(a.db, title, a.cmd)
        open(a.out, "w").write(text)
        print(text)
    else:
        d = traffic(a.fetch_db, a.write_db)
        d.update({"source_sha": a.source_sha, "runs": a.runs, "commands": {"fetch": a.cmd_fetch, "write": a.cmd_write},
                  "calibration": f"{CALIBRATION_KERNEL} of {CALIBRATION_BYTES} bytes, largest dispatch"})
        open(a.out, "w").write(json.dumps(d, indent=1) + "\n")
        print(json.dumps(d, indent=1))


if __name__ == "__main__":
    main()
