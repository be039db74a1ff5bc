"""Render the kernel table of a rocprofv3 --kernel-trace --stats run as text.

    python profiles/make_summary.py <run_results.db> <steps_profiled> "<command>" > profiles/<name>.txt
"""
import sqlite3
import sys

db, steps, cmd = sys.argv[1], float(sys.argv[2]), sys.argv[3]
con = sqlite3.connect(db)
rows = con.execute("select name, total_calls, total_duration, average, percentage from top_kernels").fetchall()
print("# rocprofv3 kernel summary (durations from the kernel trace)")
print("# command: " + cmd)
print(f"# steps in the trace: {steps:g} (warmup + timed)")
print(f"{'calls':>7} {'total_ms':>10} {'ms/step':>9} {'avg_us':>10} {'pct':>6}  kernel")
for name, calls, tot, avg, pct in rows[:40]:
    short = name.replace("tts::(anonymous namespace)::", "")
    if len(short) > 110:
        short = short[:110] + "..."
    print(f"{calls:7d} {tot / 1000:10.3f} {tot / 1000 / steps:9.3f} {avg:10.2f} {pct:6.2f}  {short}")
