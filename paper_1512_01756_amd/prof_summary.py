"""Summarize rocprofv3 output into short text tables.

usage: python -m paper_1512_01756_amd.prof_summary [--last N] <csv> <title> <command...>

<csv> is one of
  * a --stats kernel_stats.csv (per-kernel call counts and durations),
  * a --kernel-trace kernel_trace.csv (per-dispatch records, summarized per
    kernel like the stats file),
  * a --pmc counter_collection.csv (per-kernel mean counter value per
    dispatch, e.g. FETCH_SIZE / WRITE_SIZE in KiB).
With --last N (trace and counter files only) each kernel keeps only its last N
dispatches, e.g. the timed launches of a benchmark after the setup's own.
"""
import argparse
import csv
from collections import defaultdict


def short(name):
    return name.split("(")[0].replace("void ", "")


def stats_table(rows):
    out = [f"{'kernel':60s} {'calls':>6s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}"]
    for r in rows:
        out.append(f"{short(r['Name'])[:60]:60s} {int(r['Calls']):6d} {float(r['AverageNs'])/1e3:9.2f} "
                   f"{float(r['MinNs'])/1e3:8.2f} {float(r['MaxNs'])/1e3:8.2f} {float(r['Percentage']):6.2f}")
    return out


def trace_table(rows, last):
    per = defaultdict(list)           # kernel -> [(dispatch, ns)]
    for r in rows:
        per[short(r["Kernel_Name"])].append((int(r["Dispatch_Id"]),
                                             int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    if last:
        per = {k: sorted(v)[-last:] for k, v in per.items()}
    total = sum(ns for v in per.values() for _, ns in v)
    out = [f"{'kernel':60s} {'calls':>6s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(ns for _, ns in kv[1])):
        ns = [x for _, x in v]
        out.append(f"{k[:60]:60s} {len(ns):6d} {sum(ns)/len(ns)/1e3:9.2f} {min(ns)/1e3:8.2f} "
                   f"{max(ns)/1e3:8.2f} {100.0*sum(ns)/total:6.2f}")
    return out


def counter_table(rows, last):
    per = defaultdict(float)          # (kernel, dispatch, counter) -> value
    for r in rows:
        per[(short(r["Kernel_Name"]), int(r["Dispatch_Id"]), r["Counter_Name"])] += float(r["Counter_Value"])
    agg = defaultdict(list)           # (kernel, counter) -> [(dispatch, value)]
    for (k, d, c), v in per.items():
        agg[(k, c)].append((d, v))
    if last:
        agg = {kc: sorted(v)[-last:] for kc, v in agg.items()}
    out = [f"{'kernel':60s} {'counter':>12s} {'dispatches':>10s} {'mean/dispatch':>14s} {'min':>12s} {'max':>12s}"]
    for (k, c), dv in sorted(agg.items(), key=lambda kv: -sum(v for _, v in kv[1])):
        vs = [v for _, v in dv]
        out.append(f"{k[:60]:60s} {c:>12s} {len(vs):10d} {sum(vs)/len(vs):14.1f} {min(vs):12.1f} {max(vs):12.1f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--last", type=int, default=0)
    ap.add_argument("csv")
    ap.add_argument("title")
    ap.add_argument("command", nargs=argparse.REMAINDER)
    a = ap.parse_args()
    rows = list(csv.DictReader(open(a.csv)))
    print(f"# {a.title}")
    print(f"# command: {' '.join(a.command)}")
    if rows and "Counter_Name" in rows[0]:
        lines = counter_table(rows, a.last)
    elif rows and "Start_Timestamp" in rows[0]:
        lines = trace_table(rows, a.last)
    else:
        lines = stats_table(rows)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
