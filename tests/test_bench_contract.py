"""Host-side parts of the benchmark contract: the multi-GPU refusal, the
secondary metric read from the committed learned-initialiser run, the
traffic figure's guard on the kernel sources and the oracle baseline's
sample of the workload."""
import json
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr or "single MI355X" in r.stderr


def test_learned_vs_plain_comes_from_the_committed_run():
    d = bench.learned_vs_plain()
    assert d is not None and d["source"] == "profiles/learned_c5.txt"
    assert d["commands"] and all(c.startswith("python -u -m paper_2211_03516_amd.learned") for c in d["commands"])
    assert d["timed_here"] is False
    assert 0 < d["learned_steps"] <= d["plain_steps"] and d["learned_s"] > 0 and d["plain_s"] > 0
    # the summary line in the file is the one reported
    summary = [json.loads(l) for l in open(os.path.join(ROOT, "profiles", "learned_c5.txt"))
               if '"phase": "summary"' in l]
    assert len(summary) == 1 and summary[0]["targets"] == d["targets"]


def test_traffic_only_for_the_profiled_sources(monkeypatch):
    t = json.load(open(os.path.join(ROOT, "profiles", "traffic_c2.json")))
    if t["source_sha256"] == bench.kernel_source_hash():
        got = bench.load_traffic("deposit")
        assert got == t["deposit"]["fetch_bytes"] + t["deposit"]["write_bytes"]
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "0" * 64)
    assert bench.load_traffic("deposit") is None


def test_counter_rates_follow_the_launch_time(monkeypatch):
    rec = {"fetch_bytes": 3e9, "write_bytes": 1e9, "valu_insts": 1024 * 2.4e9 / 2, "l2_read_bytes": 2e12}
    monkeypatch.setattr(bench, "load_counters", lambda kernel: rec)
    r = bench.counter_rates("deposit", 1000.0, 1024 * 2.4e9 * 64)     # one second
    assert r["hbm_GBps"] == 4.0 and r["hbm_frac"] == 4.0 / 8000.0
    assert r["l2_read_TBps"] == 2.0
    assert abs(r["valu_issue_busy"] - 1.0) < 1e-12   # one wave64 instruction per SIMD every 2 cycles
    assert abs(r["valu_lane_slots_per_sample"] - 0.5) < 1e-12
    monkeypatch.setattr(bench, "load_counters", lambda kernel: None)
    assert bench.counter_rates("deposit", 1000.0, 1) is None


def test_roofline_flop_count_matches_its_breakdown():
    # the per-sample FLOP counts (FMA = 2) are the sums their comment lists
    fwd = 6 + 3 + 7 * 3 + 2
    dep = 6 + 3 + 6 + 8 + 8 + 1
    assert bench.FLOP_PER_SAMPLE == {"forward": fwd, "deposit": dep}


def test_cpu_baseline_times_eight_evenly_spaced_angles():
    import oracle
    import synth
    p = synth.workload("c1")
    target, _ = synth.random_config1_target(p["nx"], p["r_inner"], seed=0)
    d = bench.cpu_baseline(p, target, 2)
    assert d["kind"] == "oracle" and d["cores"] == 2 and d["unit"] == "samples/s" and d["value"] > 0
    n = p["n_angles"]
    angles = [k * n // 8 for k in range(8)]
    assert d["sample"].startswith("forward + dose deposit of angles %s " % ", ".join(map(str, angles)))
    # forward and deposit of each of the 8 angles; every angle holds the
    # same samples (the resin lies inside the grid's inscribed cylinder)
    per_angle = oracle.count_samples(oracle.Geometry(p), a0=0, na=1, nthreads=2)
    assert "(%d samples" % (2 * 8 * per_angle) in d["sample"]
    assert d["full_pass_s_extrapolated"] > 0
    assert d["single_thread"]["value"] > 0 and "(%d samples" % per_angle in d["single_thread"]["sample"]
