"""Benchmark: ray-voxel samples/s of one forward projection plus one dose
deposit over all angles of the full-optics workload, on one GPU.

A step is one pass of the whole hot path over one synthetic target: the
forward projection of the 256^3 target for all 360 angles, then the dose
deposit of those projections.  Inputs are resident in HBM before the timed
region; the geometry (ray tracing) is set up once outside it.

Prints one JSON line (rank 0).  Only one GPU is used: --gpus above 1 exits
with a message.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic arithmetic of one ray-voxel sample, counting an FMA as 2 FLOP
# (the convention of the 157.3 TFLOP/s FP32 vector peak):
#   forward: position 3 FMA (6), fractional offsets 3, seven lerps of one
#            subtraction and one FMA (21), attenuated accumulation S r + v
#            (one FMA, 2) = 32;
#   deposit: position 3 FMA (6), fractional offsets 3, the z and y weight
#            splits (6), the x split of four weights (8), the eight corner
#            sums (8), the attenuation e r (1) = 32.
# (The same work counted in lane operations, an FMA once, is ~25-30 per
# sample.)
FLOP_PER_SAMPLE = {"forward": 32, "deposit": 32}
# Gather-byte model: the 8 FP32 corner values a sample reads (or updates).
GATHER_BYTES_PER_SAMPLE = 32
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_HBM_GBPS = 8000.0

WORKLOAD_NAMES = {
    "c2": ("c2: 256^3 target, 360 angles, 256x256 DMD, thin-lens projector "
           "(10 deg edge chief ray), 16 pupil samples (12.2 deg), refracting vial "
           "R_o 120 / R_i 112, n 1/1.47/1.49, alpha 0.005/voxel, step 0.5"),
    "c4": ("c4: 512^3 target, 360 angles, 512x512 DMD, thin-lens projector "
           "(15 deg edge chief ray), 8 pupil samples (12.2 deg), refracting vial "
           "R_o 240 / R_i 224, n 1/1.47/1.49, alpha 0.005/voxel, step 0.5"),
    "c5": ("c5: 128^3 target, 180 angles, 128x128 DMD, thin-lens projector "
           "(10 deg edge chief ray), 8 pupil samples, vial R_o 60 / R_i 56"),
    "c1": ("c1: 64^3 target, 90 angles, 64x64 DMD, telecentric chief rays, "
           "index-matched vial R 32, alpha 0.01/voxel"),
}


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("project.hip", "boxes.hip", "vam_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_2211_03516_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def load_counters(kernel):
    """The committed rocprofv3 counter record of a kernel per launch (HBM
    fetch / write bytes, VALU wave-instructions, L1->L2 bytes), or None when
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "traffic_c2.json")
    if not os.path.exists(path):
        return None
    try:
        d = json.load(open(path))
    except ValueError:
        return None
    if d.get("source_sha256") != kernel_source_hash() or kernel not in d:
        return None
    return d[kernel]


def load_traffic(kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, or None
    when the kernel source changed since they were taken."""
    k = load_counters(kernel)
    if k is None:
        return None
    return k.get("fetch_bytes", 0) + k.get("write_bytes", 0)


def counter_rates(kernel, launch_ms, samples):
    """HBM and L2 bandwidth and VALU use of a kernel: the committed rocprofv3
    counter totals per launch (taken on the same kernel sources, not in this
    run) over this run's launch time.  VALU issue busy = wave-instructions x
    2 cycles / (1024 SIMDs x 2.4 GHz x time), the rate at which MI355X issues
    one wave64 VALU instruction per SIMD every two cycles; VALU lane slots
    per sample = wave-instructions x 64 / samples."""
    k = load_counters(kernel)
    if k is None or not launch_ms:
        return None
    sec = launch_ms * 1e-3
    hbm = (k.get("fetch_bytes", 0) + k.get("write_bytes", 0)) / sec / 1e9
    out = {"kernel": kernel, "source": "committed rocprofv3 counters, profiles/traffic_c2.json",
           "hbm_GBps": hbm, "hbm_frac": hbm / PEAK_HBM_GBPS}
    if "l2_read_bytes" in k:
        out["l2_read_TBps"] = k["l2_read_bytes"] / sec / 1e12
    if "valu_insts" in k:
        out["valu_issue_busy"] = k["valu_insts"] * 2.0 / (1024 * 2.4e9 * sec)
        out["valu_lane_slots_per_sample"] = k["valu_insts"] * 64.0 / samples
    if "valu_thread_cycles" in k:
        out["valu_active_lane_cycles_per_sample"] = k["valu_thread_cycles"] / samples
    return out


def learned_vs_plain():
    """Secondary metric (seconds and steps to the plain method's dose error,
    learned vs plain start) from the committed c5 run of
    paper_2211_03516_amd.learned; it takes an hour of data generation and
    training, so it is not re-measured (nor timed) here."""
    path = os.path.join(ROOT, "profiles", "learned_c5.txt")
    if not os.path.exists(path):
        return None
    cmds, summary = [], None
    for line in open(path):
        if line.startswith("#   python"):
            cmds.append(line[1:].strip())
        elif '"phase": "summary"' in line:
            summary = json.loads(line)
    if summary is None:
        return None
    return {"metric": "s to target dose error (learned vs plain)", "unit": "s",
            "learned_s": summary["mean_learned_s"], "plain_s": summary["mean_plain_s"],
            "learned_steps": summary["mean_learned_steps"], "plain_steps": summary["mean_plain_steps"],
            "targets": summary["targets"], "reached": summary["reached"], "fallbacks": summary["fallbacks"],
            "workload": "c5: 128^3, 180 angles, 128^2 DMD, 8 pupil samples; 2000 training targets, "
                        "100-step labels",
            "timed_here": False, "source": "profiles/learned_c5.txt", "commands": cmds}


def cpu_baseline(p, target, threads):
    """The FP64 oracle on a bounded sample of the same workload: the forward
    and the dose deposit of 8 evenly spaced angles (every angle of the turn
    holds the same samples, by the rotational symmetry about z, so the full
    pass is these 8 scaled by n_angles / 8)."""
    import oracle
    og = oracle.Geometry(p)
    n_ang = p["n_angles"]
    angles = sorted({k * n_ang // 8 for k in range(8)})
    n_samples = 0
    t0 = time.perf_counter()
    for a in angles:
        P = oracle.forward(og, target, a0=a, na=1, nthreads=threads)
        oracle.adjoint(og, P, a0=a, na=1, nthreads=threads)
    dt = time.perf_counter() - t0
    for a in angles:
        n_samples += 2 * oracle.count_samples(og, a0=a, na=1, nthreads=threads)
    # the same oracle on one host thread: the forward of one angle
    n1 = oracle.count_samples(og, a0=angles[0], na=1, nthreads=threads)
    t1 = time.perf_counter()
    oracle.forward(og, target, a0=angles[0], na=1, nthreads=1)
    dt1 = time.perf_counter() - t1
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {
        "value": n_samples / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
        "sample": "forward + dose deposit of angles %s of the same workload " % ", ".join(map(str, angles)) +
                  "(%d samples, %.1f s wall, FP64 C++ std::thread)" % (n_samples, dt),
        "full_pass_s_extrapolated": dt * n_ang / len(angles),
        "single_thread": {"value": n1 / dt1, "unit": "samples/s",
                          "sample": "forward of angle %d on one thread (%d samples, %.1f s)" % (angles[0], n1, dt1)},
        "host": {"cpu_model": model, "logical_cpus": os.cpu_count()},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOAD_NAMES))
    ap.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16"],
                    help="storage type of the volume and projections (accumulation is FP32/FP64)")
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--adjoint-variant", type=int, default=0)
    ap.add_argument("--forward-variant", type=int, default=0)
    ap.add_argument("--box-edge", type=int, default=0, help="lab box edge: 8, 12 or 16")
    ap.add_argument("--seg-order", type=int, default=-1, help="segment order of the deposit")
    ap.add_argument("--seg-order-fwd", type=int, default=-1, help="segment order of the forward")
    ap.add_argument("--deposit-threads", type=int, default=0)
    ap.add_argument("--angle-block", default="", help="deposit[,forward] angle blocks of the XCD-aware work order")
    ap.add_argument("--forward-lanes", type=int, default=0, help="march mode of the box forward (1: one lane, 2: two lanes, 3: cached cell)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-sparse", action="store_true",
                    help="skip the extra timing of the deposit on the target's own (sparse) projections")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the projector pair is built and timed on a "
              "single MI355X (angle-block sharding across GPUs is a design note, not run).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_2211_03516_amd as vam
    import synth

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    p = synth.workload(args.workload)
    if args.workload == "c1":
        target, _ = synth.random_config1_target(p["nx"], p["r_inner"], seed=args.seed)
    else:
        target, _ = synth.random_config2_target(p["nx"], p["r_inner"], seed=args.seed)
    tdt = {"f32": torch.float32, "bf16": torch.bfloat16, "f16": torch.float16}[args.dtype]
    t_setup = time.perf_counter()
    g = vam.Geometry(p)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup
    g.set_adjoint_variant(args.adjoint_variant)
    g.set_forward_variant(args.forward_variant)
    if args.box_edge:
        g.set_box_edge(args.box_edge)
    if args.seg_order >= 0:
        g.set_segment_order(args.seg_order)
    if args.seg_order_fwd >= 0:
        g.set_segment_order(args.seg_order_fwd, forward=True)
    if args.deposit_threads:
        g.set_deposit_threads(args.deposit_threads)
    if args.forward_lanes:
        g.set_forward_lanes(args.forward_lanes)
    if args.angle_block:
        ab = [int(v) for v in args.angle_block.split(",")]
        g.set_angle_blocks(deposit=ab[0], forward=ab[1] if len(ab) > 1 else None)
    rays_hit, samples_per_pass = g.stats()
    vol = torch.from_numpy(target).to(dev, dtype=tdt)
    proj = torch.empty(g.proj_shape, device=dev, dtype=tdt)
    dose = torch.empty(g.vol_shape, device=dev)

    # The deposit skips rays whose projection value is 0 (their contribution
    # is exactly zero), so its speed depends on how much of each projection
    # is empty.  The headline step deposits a dense input -- the target's
    # projections plus a floor of 1e-3 of their maximum, computed once -- so
    # that every counted sample is processed; the target's own projections
    # (empty outside its shadow) are timed separately as `deposit_sparse_ms`.
    g.forward(vol, out=proj)
    dense = proj.float() + float(proj.float().max()) * 1e-3
    dense = dense.to(tdt)
    torch.cuda.synchronize()

    def step():
        g.forward(vol, out=proj)
        g.back(dense, out=dose)

    if args.copy_calibration:
        # a plain copy kernel of known size: reads and writes exactly n bytes,
        # so its FETCH_SIZE / WRITE_SIZE readings scale the counters to bytes
        n = args.copy_calibration << 20
        src = torch.ones(n // 4, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    fwd_ms, back_ms = [], []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
        # the library's per-kernel events are read after each step (one
        # synchronisation per ~0.6 s step)
        torch.cuda.synchronize()
        f, b = g.kernel_times()
        fwd_ms.append(f)
        back_ms.append(b)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    value = 2.0 * samples_per_pass * args.steps / (total_ms * 1e-3)

    f_avg, b_avg = float(np.mean(fwd_ms)), float(np.mean(back_ms))
    # deposit of the target's own projections (zero outside its shadow)
    sparse_ms, active = None, None
    if not args.no_sparse:
        g.forward(vol, out=proj)
        sparse_ms = []
        for _ in range(max(1, args.steps)):
            g.back(proj, out=dose)
            torch.cuda.synchronize()
            sparse_ms.append(g.kernel_times()[1])
        active = float((proj != 0).float().mean())
    dom, dom_ms = ("deposit", b_avg) if b_avg >= f_avg else ("forward", f_avg)
    flop = FLOP_PER_SAMPLE[dom] * samples_per_pass
    achieved = flop / (dom_ms * 1e-3) / 1e12
    profiled = (args.workload, args.dtype) == ("c2", "f32")
    traffic = load_traffic(dom) if profiled else None
    roofline = {
        "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
        "kernel": dom, "flop_per_sample": FLOP_PER_SAMPLE[dom], "flop_convention": "FMA = 2 FLOP",
        "launch_ms": dom_ms, "samples_per_launch": samples_per_pass,
    }
    gather_gbps = GATHER_BYTES_PER_SAMPLE * samples_per_pass / (dom_ms * 1e-3) / 1e9
    out = {
        "metric": "ray-voxel samples/s fwd+adj", "value": value, "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": args.dtype,
        "data": "synthetic (seeded union of spheres/boxes/tori, seed %d)" % args.seed,
        "config": {"workload": WORKLOAD_NAMES[args.workload], "samples_per_pass": samples_per_pass,
                   "rays_hit": rays_hit, "adjoint_variant": args.adjoint_variant,
                   "forward_variant": args.forward_variant, "box_edge": args.box_edge},
        "roofline": roofline,
        "kernels_ms": {"forward": f_avg, "deposit": b_avg,
                       "forward_median": float(np.median(fwd_ms)), "deposit_median": float(np.median(back_ms)),
                       "deposit_sparse_ms": float(np.mean(sparse_ms)) if sparse_ms else None,
                       "sparse_nonzero_pixel_fraction": active},
        "gather_model": {"bytes_per_sample": GATHER_BYTES_PER_SAMPLE, "kernel": dom,
                         "GBps": gather_gbps, "frac_of_hbm_peak": gather_gbps / PEAK_HBM_GBPS},
        "counters": counter_rates(dom, dom_ms, samples_per_pass) if profiled else None,
        "setup_s": t_setup, "wall_s": wall,
        "learned_vs_plain": learned_vs_plain(),
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        out["cpu_baseline"] = cpu_baseline(p, target, threads)
    g.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
