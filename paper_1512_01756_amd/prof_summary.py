"""Summarize rocprofv3 output into short text tables.

usage: python -m paper_1512_01756_amd.prof_summary <csv> <title> <command...>

<csv> is either a --stats kernel_stats.csv (per-kernel call counts and
durations) or a --pmc counter_collection.csv (per-kernel mean counter value
per dispatch, e.g. FETCH_SIZE / WRITE_SIZE in KiB).
"""
import csv
import sys
from collections import defaultdict


def short(name):
    return name.split("(")[0].replace("void ", "")


def stats_table(rows):
    out = [f"{'kernel':60s} {'calls':>6s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}"]
    for r in rows:
        out.append(f"{short(r['Name'])[:60]:60s} {int(r['Calls']):6d} {float(r['AverageNs'])/1e3:9.2f} "
                   f"{float(r['MinNs'])/1e3:8.2f} {float(r['MaxNs'])/1e3:8.2f} {float(r['Percentage']):6.2f}")
    return out


def counter_table(rows):
    per = defaultdict(float)          # (kernel, dispatch, counter) -> value
    for r in rows:
        per[(short(r["Kernel_Name"]), r["Dispatch_Id"], r["Counter_Name"])] += float(r["Counter_Value"])
    agg = defaultdict(list)           # (kernel, counter) -> values per dispatch
    for (k, _, c), v in per.items():
        agg[(k, c)].append(v)
    out = [f"{'kernel':60s} {'counter':>12s} {'dispatches':>10s} {'mean/dispatch':>14s} {'min':>12s} {'max':>12s}"]
    for (k, c), vs in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append(f"{k[:60]:60s} {c:>12s} {len(vs):10d} {sum(vs)/len(vs):14.1f} {min(vs):12.1f} {max(vs):12.1f}")
    return out


def main():
    path, title, cmd = sys.argv[1], sys.argv[2], " ".join(sys.argv[3:])
    rows = list(csv.DictReader(open(path)))
    print(f"# {title}")
    print(f"# command: {cmd}")
    lines = counter_table(rows) if rows and "Counter_Name" in rows[0] else stats_table(rows)
    print("\n".join(lines))


if __name__ == "__main__":
    main()
