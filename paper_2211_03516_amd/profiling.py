"""Summaries of rocprofv3 CSV output for the profiles/ directory.

    python -m paper_2211_03516_amd.profiling stats <run_kernel_stats.csv> [--cmd "..."]
    python -m paper_2211_03516_amd.profiling counters <run_counter_collection.csv> [--cmd "..."]

`stats` prints the per-kernel table (calls, average / total milliseconds,
share of GPU time); `counters` prints per-kernel averages of each counter
over dispatches (FETCH_SIZE / WRITE_SIZE in KiB per dispatch, as rocprofv3
reports them).
"""
import argparse
import csv
import collections
import sys


def _short(name):
    name = name.strip('"')
    return name.split("(")[0].replace("void ", "")


def stats(path, out=sys.stdout):
    rows = list(csv.DictReader(open(path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    out.write("%-58s %6s %12s %12s %7s\n" % ("kernel", "calls", "avg_ms", "total_ms", "pct"))
    for r in rows:
        out.write("%-58s %6s %12.3f %12.3f %7.2f\n" % (
            _short(r["Name"])[:58], r["Calls"], float(r["AverageNs"]) / 1e6,
            float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))


def counters(path, out=sys.stdout):
    rows = list(csv.DictReader(open(path)))
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for r in rows:
        acc[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    out.write("%-58s %-22s %8s %16s\n" % ("kernel", "counter", "samples", "mean_per_dispatch"))
    for k in sorted(acc):
        for c in sorted(acc[k]):
            v = acc[k][c]
            out.write("%-58s %-22s %8d %16.6g\n" % (k[:58], c, len(v), sum(v) / len(v)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["stats", "counters"])
    ap.add_argument("path")
    ap.add_argument("--cmd", default=None, help="command that produced the CSV (written as a header)")
    a = ap.parse_args(argv)
    if a.cmd:
        sys.stdout.write("# command: %s\n" % a.cmd)
    {"stats": stats, "counters": counters}[a.what](a.path)


if __name__ == "__main__":
    main()
