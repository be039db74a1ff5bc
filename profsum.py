"""Text summaries of rocprofv3 output for profiles/.

    python profsum.py kernels <run_results.db> <steps> "<command>"
        kernel table of a --kernel-trace --stats run (durations from the trace)

    python profsum.py traffic <family> <kernel regex> <source file> \\
        <fetch.csv> <write.csv> <copy_fetch.csv> <copy_write.csv> <copy bytes> <algo bytes/launch> "<commands>" \\
        [<workload> [<method>]]
        per-launch HBM traffic of the kernels matching the regex: FETCH_SIZE and
        WRITE_SIZE (KiB per dispatch, from two --pmc passes) scaled by what the same
        counters read for a plain device copy of known size

    python profsum.py stage <name> <kernel regex> <steps> <fetch.csv> <write.csv> \\
        <copy_fetch.csv> <copy_write.csv> <copy bytes> <algo bytes/step> "<commands>" [<workload> [<source>]]
        the same scaled HBM traffic summed over every matching dispatch of a run of
        <steps> steps, per step (a stage made of many kernels)

    python profsum.py mfma <counters.csv> <kernel regex> <calls> <algo flops/call> "<command>"
        FP64 matrix-core work and busy cycles of the matching dispatches, per call

Reads only what rocprofv3 wrote; prints the summary on stdout.
"""
from __future__ import annotations

import csv
import hashlib
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.abspath(__file__))


def kernels(db: str, steps: float, cmd: str) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
    out = ["# rocprofv3 kernel summary (durations from the kernel trace)",
           "# command: " + cmd,
           f"# steps in the trace: {steps:g} (warmup + timed)",
           f"{'calls':>7} {'total_ms':>10} {'ms/step':>9} {'avg_us':>10} {'pct':>6}  kernel"]
    for name, calls, tot, avg, pct in rows[:40]:
        short = name.replace("tts::(anonymous namespace)::", "")
        if len(short) > 110:
            short = short[:110] + "..."
        out.append(f"{calls:7d} {tot / 1000:10.3f} {tot / 1000 / steps:9.3f} {avg:10.2f} {pct:6.2f}  {short}")
    return "\n".join(out)


def _counter(path: str, counter: str, regex: str | None):
    """(sum of the counter over matching dispatches, number of matching dispatches)."""
    total, seen = 0.0, set()
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            if regex and not re.search(regex, row.get("Kernel_Name", "")):
                continue
            total += float(row["Counter_Value"])
            seen.add(row.get("Dispatch_Id"))
    return total, len(seen)


def traffic(family, regex, source, fetch_csv, write_csv, cfetch_csv, cwrite_csv, copy_bytes, algo, cmds,
            workload=None, method="cps") -> str:
    f_sum, f_n = _counter(fetch_csv, "FETCH_SIZE", regex)
    w_sum, w_n = _counter(write_csv, "WRITE_SIZE", regex)
    cf_sum, cf_n = _counter(cfetch_csv, "FETCH_SIZE", r"copyBuffer")
    cw_sum, cw_n = _counter(cwrite_csv, "WRITE_SIZE", r"copyBuffer")
    if not (f_n and w_n and cf_n and cw_n):
        raise SystemExit("no matching dispatches")
    fetch_kib, write_kib = f_sum / f_n, w_sum / w_n
    kib = float(copy_bytes) / 1024.0
    ffac = kib / (cf_sum / cf_n)
    wfac = kib / (cw_sum / cw_n)
    tb = (fetch_kib * ffac + write_kib * wfac) * 1024.0
    with open(os.path.join(ROOT, source), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    lines = [f"# HBM traffic per launch of the '{family}' kernels (FETCH_SIZE + WRITE_SIZE, KiB per dispatch),",
             "# each scaled by the counter's reading for a plain device copy of known size.",
             "# commands:"] + [f"#   {c}" for c in cmds.split(" ;; ")] + (
             [f"workload: {workload}", f"method: {method}"] if workload else []) + [
             f"family: {family}",
             f"kernel_regex: {regex}",
             f"dispatches: {f_n}",
             f"fetch_kib_per_launch_raw: {fetch_kib:.3f}",
             f"write_kib_per_launch_raw: {write_kib:.3f}",
             f"copy_bytes: {int(copy_bytes)}",
             f"copy_fetch_factor: {ffac:.4f}",
             f"copy_write_factor: {wfac:.4f}",
             f"traffic_bytes_per_launch: {tb:.1f}",
             f"algorithmic_bytes_per_launch: {float(algo):.1f}",
             f"traffic_over_algorithmic: {tb / float(algo):.3f}" if float(algo) > 0 else "traffic_over_algorithmic: n/a",
             f"source: {source}",
             f"source_sha256: {sha}"]
    return "\n".join(lines)


def _counters(path: str, regex: str):
    """{counter: sum over matching dispatches}, number of matching dispatches."""
    tot, seen = {}, set()
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if not re.search(regex, row.get("Kernel_Name", "")):
                continue
            tot[row["Counter_Name"]] = tot.get(row["Counter_Name"], 0.0) + float(row["Counter_Value"])
            seen.add(row.get("Dispatch_Id"))
    return tot, len(seen)


def stage(name, regex, steps, fetch_csv, write_csv, cfetch_csv, cwrite_csv, copy_bytes, algo, cmds,
          workload=None, source=None) -> str:
    f_sum, f_n = _counter(fetch_csv, "FETCH_SIZE", regex)
    w_sum, w_n = _counter(write_csv, "WRITE_SIZE", regex)
    cf_sum, cf_n = _counter(cfetch_csv, "FETCH_SIZE", r"copyBuffer")
    cw_sum, cw_n = _counter(cwrite_csv, "WRITE_SIZE", r"copyBuffer")
    if not (f_n and w_n and cf_n and cw_n):
        raise SystemExit("no matching dispatches")
    steps = float(steps)
    kib = float(copy_bytes) / 1024.0
    ffac = kib / (cf_sum / cf_n)
    wfac = kib / (cw_sum / cw_n)
    tb = (f_sum * ffac + w_sum * wfac) * 1024.0 / steps
    lines = [f"# HBM traffic per step of the stage '{name}' (FETCH_SIZE + WRITE_SIZE summed over its",
             "# dispatches), each counter scaled by its reading for a plain device copy of known size.",
             "# commands:"] + [f"#   {c}" for c in cmds.split(" ;; ")] + (
             [f"workload: {workload}"] if workload else []) + [
             f"stage: {name}",
             f"kernel_regex: {regex}",
             f"steps: {steps:g}",
             f"dispatches_per_step: {f_n / steps:.1f}",
             f"fetch_kib_per_step_raw: {f_sum / steps:.1f}",
             f"write_kib_per_step_raw: {w_sum / steps:.1f}",
             f"copy_fetch_factor: {ffac:.4f}",
             f"copy_write_factor: {wfac:.4f}",
             f"traffic_bytes_per_step: {tb:.1f}",
             f"algorithmic_bytes_per_step: {float(algo):.1f}",
             f"traffic_over_algorithmic: {tb / float(algo):.3f}"]
    if source:
        with open(os.path.join(ROOT, source), "rb") as fh:
            lines += [f"source: {source}", f"source_sha256: {hashlib.sha256(fh.read()).hexdigest()}"]
    return "\n".join(lines)


def mfma(csv_path, regex, calls, algo, cmd) -> str:
    tot, n = _counters(csv_path, regex)
    calls = float(calls)
    flops = tot.get("SQ_INSTS_VALU_MFMA_MOPS_F64", 0.0) * 512.0 / calls
    busy = tot.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / calls
    gui = tot.get("GRBM_GUI_ACTIVE", 0.0) / calls
    lines = ["# FP64 matrix-core counters of the matching dispatches, per call",
             "# command: " + cmd,
             "# MFMA flops = SQ_INSTS_VALU_MFMA_MOPS_F64 x 512; busy fraction = SQ_VALU_MFMA_BUSY_CYCLES /",
             "# (GRBM_GUI_ACTIVE / 8 XCDs x 1024 SIMDs): GRBM_GUI_ACTIVE sums the 8 XCDs' clocks",
             f"kernel_regex: {regex}",
             f"dispatches_per_call: {n / calls:g}",
             f"mfma_f64_flops_per_call: {flops:.4e}",
             f"algorithmic_flops_per_call: {float(algo):.4e}",
             f"mfma_flops_over_algorithmic: {flops / float(algo):.3f}",
             f"mfma_busy_cycles_per_call: {busy:.4e}",
             f"gui_active_cycles_per_call: {gui:.4e}",
             f"mfma_busy_fraction: {busy / (gui / 8.0 * 1024.0):.3f}" if gui else "mfma_busy_fraction: n/a",
             f"lds_instructions_per_call: {tot.get('SQ_INSTS_LDS', 0.0) / calls:.4e}",
             f"lds_bank_conflict_cycles_per_call: {tot.get('SQ_LDS_BANK_CONFLICT', 0.0) / calls:.4e}"]
    return "\n".join(lines)


def main(argv):
    if len(argv) >= 4 and argv[0] == "kernels":
        print(kernels(argv[1], float(argv[2]), argv[3]))
    elif len(argv) >= 11 and argv[0] == "traffic":
        print(traffic(*argv[1:13]))
    elif len(argv) >= 11 and argv[0] == "stage":
        print(stage(*argv[1:13]))
    elif len(argv) >= 6 and argv[0] == "mfma":
        print(mfma(*argv[1:6]))
    else:
        print(__doc__)
        raise SystemExit(2)


if __name__ == "__main__":
    main(sys.argv[1:])
