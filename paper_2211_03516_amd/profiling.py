"""Summaries of rocprofv3 CSV output for the profiles/ directory.

    python -m paper_2211_03516_amd.profiling stats <run_kernel_stats.csv> [--cmd "..."]
    python -m paper_2211_03516_amd.profiling counters <run_counter_collection.csv> [--cmd "..."]
    python -m paper_2211_03516_amd.profiling traffic <fetch.csv> <write.csv> --copy-mib N [--out f.json]

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


KERNELS = {"deposit": "k_back_box", "forward": "k_forward_box"}


def kernel_source_hash(root):
    import hashlib
    import os
    h = hashlib.sha256()
    for f in ("project.hip", "boxes.hip", "vam_internal.h"):
        h.update(open(os.path.join(root, "paper_2211_03516_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def traffic(fetch_csv, write_csv, copy_mib, root, calls=None):
    """HBM bytes per call of the main kernels (a call = one operator pass,
    which may be several dispatches), with FETCH_SIZE and WRITE_SIZE each
    scaled by what they read for the largest copy kernel (a device copy of
    copy_mib MiB: reads and writes exactly that much).  `calls` maps each
    kernel to the number of operator passes in the profiled run."""
    calls = calls or {}
    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        copy = max((float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]), default=0.0)
        per = collections.defaultdict(list)
        for r in rows:
            for name, pat in KERNELS.items():
                if pat in r["Kernel_Name"]:
                    per[name].append(float(r["Counter_Value"]))
        return copy, per
    cf, fetch = load(fetch_csv, "FETCH_SIZE")
    cw, write = load(write_csv, "WRITE_SIZE")
    kib = copy_mib * 1024.0
    ff = kib / cf if cf else None
    fw = kib / cw if cw else None
    out = {"source_sha256": kernel_source_hash(root), "copy_mib": copy_mib,
           "fetch_scale": ff, "write_scale": fw,
           "note": "bytes per call; FETCH_SIZE and WRITE_SIZE (KiB) scaled by the copy calibration"}
    for name in KERNELS:
        if fetch.get(name) and write.get(name) and ff and fw:
            c = calls.get(name, 1)
            f = sum(fetch[name]) / c * ff * 1024
            w = sum(write[name]) / c * fw * 1024
            out[name] = {"fetch_bytes": f, "write_bytes": w, "dispatches_per_call": len(fetch[name]) / c}
    return out


def main(argv=None):
    import json
    import os
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["stats", "counters", "traffic"])
    ap.add_argument("path")
    ap.add_argument("path2", nargs="?")
    ap.add_argument("--cmd", default=None, help="command that produced the CSV (written as a header)")
    ap.add_argument("--copy-mib", type=float, default=1024.0)
    ap.add_argument("--calls", default="", help="operator passes per kernel in the run, e.g. forward=2,deposit=1")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    if a.what == "traffic":
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        calls = {k: int(v) for k, v in (kv.split("=") for kv in a.calls.split(",") if kv)}
        d = traffic(a.path, a.path2, a.copy_mib, root, calls)
        if a.cmd:
            d["command"] = a.cmd
        text = json.dumps(d, indent=1)
        if a.out:
            open(a.out, "w").write(text + "\n")
        print(text)
        return
    if a.cmd:
        sys.stdout.write("# command: %s\n" % a.cmd)
    {"stats": stats, "counters": counters}[a.what](a.path)


if __name__ == "__main__":
    main()
