"""Summaries of rocprofv3 CSV output for the profiles/ directory.

    python -m paper_2211_03516_amd.profiling stats <run_kernel_stats.csv> [--cmd "..."]
    python -m paper_2211_03516_amd.profiling counters <run_counter_collection.csv> [--cmd "..."]
    python -m paper_2211_03516_amd.profiling traffic <fetch.csv> <write.csv> --copy-mib N [--sq sq.csv] [--l2 l2.csv] [--out f.json]
    python -m paper_2211_03516_amd.profiling l2 <l2 counters.csv> <run_kernel_stats.csv> --copy-mib N --calls ...

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


def _sums(path, counters):
    """{kernel: {counter: (sum over dispatches, dispatches)}} for the main
    kernels, and {counter: largest value of a copy kernel dispatch}."""
    per = collections.defaultdict(lambda: collections.defaultdict(lambda: [0.0, 0]))
    copy = collections.defaultdict(float)
    for r in csv.DictReader(open(path)):
        c, v = r["Counter_Name"], float(r["Counter_Value"])
        if c not in counters:
            continue
        if "copyBuffer" in r["Kernel_Name"]:
            copy[c] = max(copy[c], v)
        for name, pat in KERNELS.items():
            if pat in r["Kernel_Name"]:
                per[name][c][0] += v
                per[name][c][1] += 1
    return per, copy


def traffic(fetch_csv, write_csv, copy_mib, root, calls=None, sq_csv=None, l2_csv=None):
    """HBM bytes per call of the main kernels (a call = one operator pass,
    which may be several dispatches), with FETCH_SIZE and WRITE_SIZE each
    scaled by what they read for the largest copy kernel (a device copy of
    copy_mib MiB: reads and writes exactly that much).  `calls` maps each
    kernel to the number of operator passes in the profiled run.  With
    sq_csv, also the VALU wave-instructions (SQ_INSTS_VALU), VALU thread
    cycles, LDS instructions and LDS bank-conflict cycles per call; with
    l2_csv (a run with the same copy), the L1 -> L2 read and write bytes per
    call (TCP_TCC_READ_REQ_sum / TCP_TCC_WRITE_REQ_sum times the copy's
    bytes per request)."""
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
    if sq_csv:
        per, _ = _sums(sq_csv, {"SQ_INSTS_VALU", "SQ_THREAD_CYCLES_VALU", "SQ_INSTS_LDS", "SQ_LDS_BANK_CONFLICT"})
        for name in KERNELS:
            if name in out and "SQ_INSTS_VALU" in per[name]:
                c = calls.get(name, 1)
                out[name]["valu_insts"] = per[name]["SQ_INSTS_VALU"][0] / c
                for key, counter in (("valu_thread_cycles", "SQ_THREAD_CYCLES_VALU"), ("lds_insts", "SQ_INSTS_LDS"),
                                     ("lds_bank_conflict_cycles", "SQ_LDS_BANK_CONFLICT")):
                    if counter in per[name]:
                        out[name][key] = per[name][counter][0] / c
    if l2_csv:
        per, copy = _sums(l2_csv, {"TCP_TCC_READ_REQ_sum", "TCP_TCC_WRITE_REQ_sum"})
        nbytes = copy_mib * 1048576.0
        rd = nbytes / copy["TCP_TCC_READ_REQ_sum"] if copy.get("TCP_TCC_READ_REQ_sum") else None
        wr = nbytes / copy["TCP_TCC_WRITE_REQ_sum"] if copy.get("TCP_TCC_WRITE_REQ_sum") else None
        for name in KERNELS:
            if name in out and rd and wr and "TCP_TCC_READ_REQ_sum" in per[name]:
                c = calls.get(name, 1)
                out[name]["l2_read_bytes"] = per[name]["TCP_TCC_READ_REQ_sum"][0] * rd / c
                out[name]["l2_write_bytes"] = per[name]["TCP_TCC_WRITE_REQ_sum"][0] * wr / c
    return out


def l2(counter_csv, stats_csv, copy_mib, calls=None, out=sys.stdout):
    """L1 -> L2 traffic per operator pass of the main kernels from
    TCP_TCC_READ_REQ_sum / TCP_TCC_WRITE_REQ_sum (bytes per request taken
    from the largest copy kernel: a device copy of copy_mib MiB reads and
    writes exactly that much), the L2 hit rate TCC_HIT / (TCC_HIT + TCC_MISS)
    and the read rate over the pass time of a kernel trace (AverageNs x
    dispatches per pass)."""
    calls = calls or {}
    rows = list(csv.DictReader(open(counter_csv)))
    acc = collections.defaultdict(lambda: collections.defaultdict(float))
    ndisp = collections.defaultdict(lambda: collections.defaultdict(int))
    copy = collections.defaultdict(float)
    for r in rows:
        c, v = r["Counter_Name"], float(r["Counter_Value"])
        if "copyBuffer" in r["Kernel_Name"]:
            copy[c] = max(copy[c], v)
        for name, pat in KERNELS.items():
            if pat in r["Kernel_Name"]:
                acc[name][c] += v
                ndisp[name][c] += 1
    nbytes = copy_mib * 1048576.0
    rd = nbytes / copy["TCP_TCC_READ_REQ_sum"] if copy.get("TCP_TCC_READ_REQ_sum") else None
    wr = nbytes / copy["TCP_TCC_WRITE_REQ_sum"] if copy.get("TCP_TCC_WRITE_REQ_sum") else None
    avg_ms = {}
    for r in csv.DictReader(open(stats_csv)):
        for name, pat in KERNELS.items():
            if pat in r["Name"]:
                avg_ms[name] = float(r["AverageNs"]) / 1e6
    out.write("# calibration (%g MiB copy): %.0f B per L1->L2 read request, %.0f B per write request\n"
              % (copy_mib, rd or 0, wr or 0))
    for name in KERNELS:
        if name not in acc or rd is None or wr is None:
            continue
        c = calls.get(name, 1)
        a = acc[name]
        reads = a["TCP_TCC_READ_REQ_sum"] * rd / c
        writes = a["TCP_TCC_WRITE_REQ_sum"] * wr / c
        hits, miss = a["TCC_HIT_sum"], a["TCC_MISS_sum"]
        per_pass = max(ndisp[name].values()) / c
        ms = avg_ms.get(name, 0.0) * per_pass
        rate = reads / (ms * 1e-3) / 1e12 if ms else 0.0
        out.write("%-8s L2 reads %.0f GB, writes %.0f GB per pass; %.2f TB/s read over %.0f ms; "
                  "L2 hit rate %.1f %%; requests %.3g\n"
                  % (name, reads / 1e9, writes / 1e9, rate, ms, 100.0 * hits / max(hits + miss, 1.0),
                     a["TCC_REQ_sum"] / c))


def main(argv=None):
    import json
    import os
    ap = argparse.ArgumentParser()
    ap.add_argument("what", choices=["stats", "counters", "traffic", "l2"])
    ap.add_argument("path")
    ap.add_argument("path2", nargs="?")
    ap.add_argument("--cmd", default=None, help="command that produced the CSV (written as a header)")
    ap.add_argument("--copy-mib", type=float, default=1024.0)
    ap.add_argument("--calls", default="", help="operator passes per kernel in the run, e.g. forward=2,deposit=1")
    ap.add_argument("--out", default=None)
    ap.add_argument("--sq", default=None, help="traffic: also SQ_INSTS_VALU from this counter CSV")
    ap.add_argument("--l2", default=None, help="traffic: also L1->L2 bytes from this counter CSV")
    a = ap.parse_args(argv)
    if a.what == "traffic":
        root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
        calls = {k: int(v) for k, v in (kv.split("=") for kv in a.calls.split(",") if kv)}
        d = traffic(a.path, a.path2, a.copy_mib, root, calls, sq_csv=a.sq, l2_csv=a.l2)
        if a.cmd:
            d["command"] = a.cmd
        text = json.dumps(d, indent=1)
        if a.out:
            open(a.out, "w").write(text + "\n")
        print(text)
        return
    if a.cmd:
        sys.stdout.write("# command: %s\n" % a.cmd)
    if a.what == "l2":
        calls = {k: int(v) for k, v in (kv.split("=") for kv in a.calls.split(",") if kv)}
        l2(a.path, a.path2, a.copy_mib, calls)
        return
    {"stats": stats, "counters": counters}[a.what](a.path)


if __name__ == "__main__":
    main()
