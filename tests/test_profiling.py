"""Host-side summaries of profiler output: the HBM traffic the benchmark line
reports and the L2 summary, on small hand-made CSV files whose answers are
worked out by hand below."""
import csv
import io
import json
import os

from paper_2211_03516_amd import profiling

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

DEP = "void vam::k_back_boxc<12, float, 1, 256, int>(vam::MarchParams, vam::BoxParams, float const*, double*)"
FWD = "void vam::k_forward_boxc<12, false>(vam::MarchParams, vam::BoxParams, float const*, float*, long, int)"
COPY = "__amd_rocclr_copyBuffer"


def _counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, c, v in rows:
            w.writerow({"Kernel_Name": k, "Counter_Name": c, "Counter_Value": v})


def test_traffic_scales_by_the_copy_calibration(tmp_path):
    # a 1 MiB copy reads as 512 KiB of FETCH_SIZE and 1024 KiB of WRITE_SIZE
    # (scales 2 and 1); the deposit's one dispatch fetches 100 KiB and writes
    # 10 KiB; the forward's four dispatches (two passes) fetch 3 KiB each
    f, w = tmp_path / "f.csv", tmp_path / "w.csv"
    _counters(f, [(COPY, "FETCH_SIZE", 512), (COPY, "FETCH_SIZE", 1), (DEP, "FETCH_SIZE", 100)]
              + [(FWD, "FETCH_SIZE", 3)] * 4)
    _counters(w, [(COPY, "WRITE_SIZE", 1024), (DEP, "WRITE_SIZE", 10)] + [(FWD, "WRITE_SIZE", 5)] * 4)
    d = profiling.traffic(str(f), str(w), 1.0, ROOT, {"forward": 2, "deposit": 1})
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    assert d["deposit"] == {"fetch_bytes": 100 * 2 * 1024, "write_bytes": 10 * 1024, "dispatches_per_call": 1.0}
    assert d["forward"] == {"fetch_bytes": 6 * 2 * 1024, "write_bytes": 10 * 1024, "dispatches_per_call": 2.0}
    assert d["source_sha256"] == profiling.kernel_source_hash(ROOT)


def test_l2_summary(tmp_path):
    # a 1 MiB copy makes 8192 read and 16384 write requests: 128 B and 64 B
    # per request.  One deposit dispatch of 2 ms: 1e6 read requests (128 MB
    # = 0.064 TB/s over 2 ms), 5e5 write requests (32 MB), 3 hits of 4.
    c, s = tmp_path / "l2.csv", tmp_path / "stats.csv"
    _counters(c, [(COPY, "TCP_TCC_READ_REQ_sum", 8192), (COPY, "TCP_TCC_WRITE_REQ_sum", 16384),
                  (DEP, "TCP_TCC_READ_REQ_sum", 1e6), (DEP, "TCP_TCC_WRITE_REQ_sum", 5e5),
                  (DEP, "TCC_HIT_sum", 3e6), (DEP, "TCC_MISS_sum", 1e6), (DEP, "TCC_REQ_sum", 4e6)])
    with open(s, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage"])
        w.writeheader()
        w.writerow({"Name": DEP, "Calls": 1, "TotalDurationNs": 2e6, "AverageNs": 2e6, "Percentage": 100})
    out = io.StringIO()
    profiling.l2(str(c), str(s), 1.0, {"deposit": 1}, out=out)
    lines = out.getvalue().splitlines()
    assert lines[0].startswith("# calibration (1 MiB copy): 128 B per L1->L2 read request, 64 B per write")
    assert lines[1] == ("deposit  L2 reads 0 GB, writes 0 GB per pass; 0.06 TB/s read over 2 ms; "
                        "L2 hit rate 75.0 %; requests 4e+06")


def test_committed_traffic_file_is_well_formed():
    d = json.load(open(os.path.join(ROOT, "profiles", "traffic_c2.json")))
    for k in ("deposit", "forward"):
        assert d[k]["fetch_bytes"] > 0 and d[k]["write_bytes"] > 0
    assert 1.9 < d["fetch_scale"] < 2.1 and 0.9 < d["write_scale"] < 1.1
    assert "rocprofv3 --pmc FETCH_SIZE" in d["command"] and "rocprofv3 --pmc WRITE_SIZE" in d["command"]


def test_traffic_with_valu_and_l2_counters(tmp_path):
    f, w, q, l = (tmp_path / n for n in ("f.csv", "w.csv", "sq.csv", "l2.csv"))
    _counters(f, [(COPY, "FETCH_SIZE", 512), (DEP, "FETCH_SIZE", 100)])
    _counters(w, [(COPY, "WRITE_SIZE", 1024), (DEP, "WRITE_SIZE", 10)])
    _counters(q, [(DEP, "SQ_INSTS_VALU", 7e9), (DEP, "SQ_LDS_BANK_CONFLICT", 5.0)])
    # a 1 MiB copy: 8192 read requests (128 B each), 16384 write requests (64 B)
    _counters(l, [(COPY, "TCP_TCC_READ_REQ_sum", 8192), (COPY, "TCP_TCC_WRITE_REQ_sum", 16384),
                  (DEP, "TCP_TCC_READ_REQ_sum", 1000), (DEP, "TCP_TCC_WRITE_REQ_sum", 10)])
    d = profiling.traffic(str(f), str(w), 1.0, ROOT, {"deposit": 1}, sq_csv=str(q), l2_csv=str(l))
    assert d["deposit"]["valu_insts"] == 7e9
    assert d["deposit"]["l2_read_bytes"] == 128000.0 and d["deposit"]["l2_write_bytes"] == 640.0
