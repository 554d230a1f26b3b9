"""Summarize a rocprofv3 --stats kernel_stats.csv into a short text table.

usage: python -m paper_1512_01756_amd.prof_summary <kernel_stats.csv> <title> <command...>
"""
import csv
import sys


def main():
    path, title, cmd = sys.argv[1], sys.argv[2], " ".join(sys.argv[3:])
    rows = list(csv.DictReader(open(path)))
    print(f"# {title}")
    print(f"# command: {cmd}")
    print(f"{'kernel':60s} {'calls':>6s} {'avg_us':>9s} {'min_us':>8s} {'max_us':>8s} {'pct':>6s}")
    for r in rows:
        name = r["Name"].split("(")[0].replace("void ", "")
        print(f"{name[:60]:60s} {int(r['Calls']):6d} {float(r['AverageNs'])/1e3:9.2f} "
              f"{float(r['MinNs'])/1e3:8.2f} {float(r['MaxNs'])/1e3:8.2f} {float(r['Percentage']):6.2f}")


if __name__ == "__main__":
    main()
