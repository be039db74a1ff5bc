"""Text summaries of rocprofv3 output for profiles/.

    python -m paper_1908_02721_amd.profsum kernels <run_results.db> <steps> "<command>"
        kernel table of a --kernel-trace --stats run (durations from the trace)

    python -m paper_1908_02721_amd.profsum traffic <family> <kernel regex> <source file> \\
        <fetch.csv> <write.csv> <copy_fetch.csv> <copy_write.csv> <copy bytes> <algo bytes/launch> "<commands>"
        per-launch HBM traffic of the kernels matching the regex: FETCH_SIZE and
        WRITE_SIZE (KiB per dispatch, from two --pmc passes) scaled by what the same
        counters read for a plain device copy of known size

Reads only what rocprofv3 wrote; prints the summary on stdout.
"""
from __future__ import annotations

import csv
import hashlib
import os
import re
import sqlite3
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


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


def traffic(family, regex, source, fetch_csv, write_csv, cfetch_csv, cwrite_csv, copy_bytes, algo, cmds) -> str:
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
             "# commands:"] + [f"#   {c}" for c in cmds.split(" ;; ")] + [
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


def main(argv):
    if len(argv) >= 4 and argv[0] == "kernels":
        print(kernels(argv[1], float(argv[2]), argv[3]))
    elif len(argv) >= 11 and argv[0] == "traffic":
        print(traffic(*argv[1:11]))
    else:
        print(__doc__)
        raise SystemExit(2)


if __name__ == "__main__":
    main(sys.argv[1:])
