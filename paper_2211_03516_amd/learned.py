"""Learned initialiser for the projection optimisation.

Per angle, the network of include/vam_cnn.h maps two images -- the target's
parallel-beam projection and the filtered parallel-beam starting point of
the plain method (Sec. 2.3) -- to a starting point for the ray-traced
optimisation (Sec. 2.5-2.7); its output is a residual on the filtered
start.  It is trained on projections the plain optimisation produced for
seeded training targets, then judged on held-out targets by the ray-traced
projector: how many optimisation steps and seconds it takes to reach the
dose error the plain method reaches.  If the network's start has a worse
dose error than the plain start, the plain start is used (fallback).

    python -m paper_2211_03516_amd.learned --train 128 --test 16 --steps 40 --epochs 4

Large runs split the training targets into shards, one process each: shard
k generates its pairs, trains on them starting from the checkpoint of shard
k - 1 (parameters, Adam moments and step count, input scales and the
learning-rate schedule's position; a .npz file) and writes its own; the
evaluation then loads the last checkpoint:

    python -m paper_2211_03516_amd.learned --train 2000 --shards 5 --shard 0 --save ck0.npz ...
    python -m paper_2211_03516_amd.learned --train 2000 --shards 5 --shard 1 --resume ck0.npz --save ck1.npz ...
    python -m paper_2211_03516_amd.learned --eval --test 200 --resume ck4.npz ...

All numerical work runs in libvam's kernels (projector, Ram-Lak, dose error,
optimisation step, and the network's MFMA kernels); this module sequences
calls and moves batches between device buffers.
"""
import json
import sys
import time

import numpy as np
import torch

from . import Cnn, Geometry, dose_error, ramlak_filter
from .optim import parallel_beam_params, _first_step

DEV = "cuda:0"


def starts(target, geom, parallel):
    """(parallel-beam projections, plain filtered start) of one target; the
    start is scaled so that the mean dose over target voxels is 1."""
    sino = parallel.forward(target)
    g0 = ramlak_filter(sino, pitch=geom.p["pitch_u"], clip_negative=True)
    d = geom.back(g0)
    mask = target > 0.5
    mean_dose = float(d[mask].mean()) if bool(mask.any()) else float(d.mean())
    if mean_dose > 0:
        g0.mul_(1.0 / mean_dose)
    return sino, g0


def run_until(target, geom, proj, lr, steps, tol=None, threshold=0.8, sharpness=20.0):
    """Projected gradient steps with a fixed step size; stops once the dose
    error is at most tol.  Returns (projections, dose errors after each
    step, seconds elapsed after each step)."""
    proj = proj.contiguous()
    dose = torch.empty_like(target)
    errs, times = [], []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        geom.optimize_step(target, proj, threshold=threshold, sharpness=sharpness, lr=lr, dose=dose,
                           want_loss=False)
        e, _ = dose_error(dose, target, threshold, sharpness)   # synchronises
        errs.append(e)
        times.append(time.perf_counter() - t0)
        if tol is not None and e <= tol:
            break
    return proj, errs, times


def final_error(target, geom, proj, threshold=0.8, sharpness=20.0):
    """Dose error of the dose these projections deposit."""
    e, _ = dose_error(geom.back(proj), target, threshold, sharpness)
    return e


def make_dataset(p, seeds, steps, target_fn, log=None):
    """Inputs x [n_targets * n_angles][2][nv][nu] and optimised projections
    y [n_targets * n_angles][nv][nu] (device FP32) for the given seeds."""
    geom = Geometry(p)
    par = Geometry(parallel_beam_params(p))
    na, nv, nu = geom.proj_shape
    X = torch.empty((len(seeds) * na, 2, nv, nu), device=DEV)
    Y = torch.empty((len(seeds) * na, nv, nu), device=DEV)
    for i, s in enumerate(seeds):
        t, _ = target_fn(p["nx"], p["r_inner"], seed=s)
        tt = torch.from_numpy(t).to(DEV)
        sino, g0 = starts(tt, geom, par)
        X[i * na:(i + 1) * na, 0] = sino
        X[i * na:(i + 1) * na, 1] = g0
        lr = _first_step(tt, geom, g0, 0.8, 20.0)
        proj, errs, times = run_until(tt, geom, g0.clone(), lr, steps)
        Y[i * na:(i + 1) * na] = proj
        if log:
            log({"target_seed": s, "dose_error_start": errs[0] if errs else None,
                 "dose_error_end": errs[-1] if errs else None, "s": times[-1] if times else 0.0})
    geom.close()
    par.close()
    return X, Y


def train(net, X, Y, epochs, batch, lr=1e-3, seed=0, time_limit=None, log=None, step0=0, total_steps=None):
    """Adam on shuffled batches (seeded order) with a cosine decay of the
    step size over total_steps (default: this call's steps), starting at
    schedule position step0; returns (per-epoch mean loss, schedule position
    reached)."""
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    hist = []
    t0 = time.perf_counter()
    xb = torch.empty((batch,) + tuple(X.shape[1:]), device=X.device)
    yb = torch.empty((batch,) + tuple(Y.shape[1:]), device=Y.device)
    if total_steps is None:
        total_steps = step0 + epochs * (n // batch)
    step = step0
    for ep in range(epochs):
        order = torch.from_numpy(rng.permutation(n)).to(X.device)
        losses = []
        for b in range(n // batch):
            idx = order[b * batch:(b + 1) * batch]
            torch.index_select(X, 0, idx, out=xb)
            torch.index_select(Y, 0, idx, out=yb)
            want = (b % 20 == 0)
            loss = net.loss_grad(xb, yb, want_loss=want)
            if want:
                losses.append(loss)
            # cosine decay of the step size
            a = lr * 0.5 * (1.0 + np.cos(np.pi * step / max(1, total_steps)))
            net.adam_step(a)
            step += 1
            if time_limit and time.perf_counter() - t0 > time_limit:
                break
        hist.append(float(np.mean(losses)) if losses else None)
        if log:
            log({"epoch": ep, "loss": hist[-1], "s": time.perf_counter() - t0})
        if time_limit and time.perf_counter() - t0 > time_limit:
            break
    torch.cuda.synchronize()
    return hist, step


def infer(net, x, batch):
    """Network output for all angles of one target (x [na][2][nv][nu])."""
    out = torch.empty((x.shape[0],) + tuple(x.shape[2:]), device=x.device)
    for a0 in range(0, x.shape[0], batch):
        a1 = min(a0 + batch, x.shape[0])
        xs = x[a0:a1].contiguous()
        out[a0:a1] = net.forward(xs)
    return out


def evaluate(net, p, seeds, steps, target_fn, batch, log=None):
    """Steps and seconds to the plain method's final dose error, plain start
    vs learned start (with fallback), per held-out target."""
    geom = Geometry(p)
    par = Geometry(parallel_beam_params(p))
    rows = []
    # untimed warm-up on the first target: the first calls on a geometry
    # allocate its work buffers, which no timed step should pay for
    t, _ = target_fn(p["nx"], p["r_inner"], seed=seeds[0])
    tt = torch.from_numpy(t).to(DEV)
    sino, g0 = starts(tt, geom, par)
    run_until(tt, geom, g0.clone(), 1e-3, 1)
    infer(net, torch.stack([sino, g0], dim=1).contiguous(), batch)
    torch.cuda.synchronize()
    for s in seeds:
        t, _ = target_fn(p["nx"], p["r_inner"], seed=s)
        tt = torch.from_numpy(t).to(DEV)
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        sino, g0 = starts(tt, geom, par)
        torch.cuda.synchronize()
        t_plain_start = time.perf_counter() - t_start
        lr = _first_step(tt, geom, g0, 0.8, 20.0)
        t2 = time.perf_counter()
        e_plain0 = final_error(tt, geom, g0)     # needed by the fallback test only
        t_e0 = time.perf_counter() - t2
        _, errs_p, times_p = run_until(tt, geom, g0.clone(), lr, steps)
        target_err = errs_p[-1]
        # the plain method is charged up to the first step at which its dose
        # error reached its final value (the error need not fall
        # monotonically: it is not the loss being minimised)
        plain_steps = next(i for i, e in enumerate(errs_p) if e <= target_err) + 1
        # learned start: network inference on (sino, g0), fallback if worse
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x = torch.stack([sino, g0], dim=1).contiguous()
        gl = infer(net, x, batch)
        torch.cuda.synchronize()
        t_infer = time.perf_counter() - t1
        # the fallback test (two deposits and dose errors) is part of the
        # learned start's cost
        e_learn0 = final_error(tt, geom, gl)
        fallback = not (e_learn0 <= e_plain0)
        t_infer_check = time.perf_counter() - t1
        start = g0.clone() if fallback else gl
        _, errs_l, times_l = run_until(tt, geom, start, lr, steps, tol=target_err)
        reached = bool(errs_l) and errs_l[-1] <= target_err
        row = {"target_seed": s, "dose_error_plain_start": e_plain0, "dose_error_learned_start": e_learn0,
               "fallback": fallback, "target_dose_error": target_err,
               "plain_steps": plain_steps, "plain_s": t_plain_start + times_p[plain_steps - 1],
               "learned_steps": len(errs_l), "learned_reached": reached,
               "learned_s": t_plain_start + t_e0 + t_infer_check + times_l[-1], "inference_s": t_infer,
               "plain_dose_errors": errs_p}
        rows.append(row)
        if log:
            log(row)
    geom.close()
    par.close()
    return rows


def summarise(rows):
    ps = np.array([r["plain_steps"] for r in rows], dtype=float)
    ls = np.array([r["learned_steps"] for r in rows], dtype=float)
    pt = np.array([r["plain_s"] for r in rows])
    lt = np.array([r["learned_s"] for r in rows])
    return {"targets": len(rows), "mean_plain_steps": float(ps.mean()), "mean_learned_steps": float(ls.mean()),
            "mean_plain_s": float(pt.mean()), "mean_learned_s": float(lt.mean()),
            "reached": int(sum(r["learned_reached"] for r in rows)),
            "fallbacks": int(sum(r["fallback"] for r in rows)),
            "mean_dose_error_plain_start": float(np.mean([r["dose_error_plain_start"] for r in rows])),
            "mean_dose_error_learned_start": float(np.mean([r["dose_error_learned_start"] for r in rows]))}


def save_checkpoint(path, net, step, total_steps, s0, s1, meta):
    state, adam_t = net.get_state()
    np.savez(path, state=state, adam_steps=np.int64(adam_t), step=np.int64(step),
             total_steps=np.int64(total_steps), scales=np.array([s0, s1], dtype=np.float64),
             meta=np.frombuffer(json.dumps(meta).encode(), dtype=np.uint8))


def load_checkpoint(path):
    with np.load(path, allow_pickle=False) as z:
        return {"state": z["state"], "adam_steps": int(z["adam_steps"]), "step": int(z["step"]),
                "total_steps": int(z["total_steps"]), "s0": float(z["scales"][0]), "s1": float(z["scales"][1]),
                "meta": json.loads(bytes(z["meta"]).decode())}


def time_network(layers, channels, n, batch, steps, log):
    """Training steps (loss and gradients, then Adam) and forward passes per
    second of the network on seeded random batches of n x n images (no data
    loading): the network's own throughput."""
    import synth
    net = Cnn(layers, channels, n, n, max_batch=batch, in_scale=(0.05, 2.0))
    net.set_params(synth.cnninit.he_init(layers, channels, seed=0))
    gen = torch.Generator().manual_seed(0)
    x = torch.rand(batch, 2, n, n, generator=gen).to(DEV)
    t = torch.rand(batch, n, n, generator=gen).to(DEV)
    for _ in range(5):
        net.loss_grad(x, t, want_loss=False)
        net.adam_step(1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.loss_grad(x, t, want_loss=False)
        net.adam_step(1e-4)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    t1 = time.perf_counter()
    for _ in range(steps):
        net.forward(x)
    torch.cuda.synchronize()
    di = time.perf_counter() - t1
    log({"phase": "timing", "image": n, "batch": batch, "steps": steps,
         "train_images_per_s": steps * batch / dt, "train_ms_per_batch": 1e3 * dt / steps,
         "infer_ms_per_batch": 1e3 * di / steps})
    net.close()


def main(argv=None):
    import argparse
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c5")
    ap.add_argument("--train", type=int, default=128, help="training targets (over all shards)")
    ap.add_argument("--test", type=int, default=16)
    ap.add_argument("--steps", type=int, default=40, help="plain optimisation steps (labels and reference)")
    ap.add_argument("--epochs", type=int, default=4, help="epochs over each shard")
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--layers", type=int, default=6)
    ap.add_argument("--channels", type=int, default=64)
    ap.add_argument("--train-seconds", type=float, default=0.0)
    ap.add_argument("--scale", type=int, default=0, help="grid/DMD size override (0: the workload's)")
    ap.add_argument("--angles", type=int, default=0)
    ap.add_argument("--shards", type=int, default=1, help="split the training targets into this many shards")
    ap.add_argument("--shard", type=int, default=-1, help="generate and train on this shard only")
    ap.add_argument("--eval", action="store_true", help="only evaluate the network of --resume")
    ap.add_argument("--resume", default="", help="checkpoint to start from")
    ap.add_argument("--save", default="", help="checkpoint to write after training")
    ap.add_argument("--time-steps", type=int, default=0,
                    help="only time this many training steps and forward passes of the network")
    a = ap.parse_args(argv)

    def log(d):
        print(json.dumps(d), flush=True)

    p = synth.workload(a.workload)
    if a.time_steps:
        time_network(a.layers, a.channels, a.scale or p["nx"], a.batch, a.time_steps, log)
        return 0
    if a.scale or a.angles:
        n = a.scale or p["nx"]
        ratio = n / p["nx"]
        p = synth.configs.scaled(p, nx=n, ny=n, nz=n, nu=n, nv=n, n_angles=a.angles or p["n_angles"],
                                 r_outer=p["r_outer"] * ratio, r_inner=p["r_inner"] * ratio,
                                 focus=p["focus"] * ratio, pupil=p["pupil"] * ratio)
    fn = synth.random_config2_target
    ck = load_checkpoint(a.resume) if a.resume else None
    nv, nu, na = p["nv"], p["nu"], p["n_angles"]
    net = None
    if not a.eval:
        shards = range(a.shards) if a.shard < 0 else [a.shard]
        per = (a.train + a.shards - 1) // a.shards
        step = ck["step"] if ck else 0
        # the cosine schedule spans every shard's epochs
        total = ck["total_steps"] if ck else a.shards * a.epochs * ((per * na) // a.batch)
        for k in shards:
            seeds = list(range(1000 + k * per, 1000 + min((k + 1) * per, a.train)))
            t0 = time.perf_counter()
            X, Y = make_dataset(p, seeds, a.steps, fn, log=log)
            log({"phase": "data", "shard": k, "targets": len(seeds), "images": int(X.shape[0]),
                 "s": time.perf_counter() - t0})
            if net is None:
                if ck:
                    s0, s1 = ck["s0"], ck["s1"]
                else:
                    # input scales from the first shard, kept for all later ones
                    s0 = 1.0 / max(float(X[:, 0].abs().max()), 1e-30)
                    s1 = 1.0 / max(float(X[:, 1].abs().mean()), 1e-30)
                net = Cnn(a.layers, a.channels, nv, nu, max_batch=a.batch, in_scale=(s0, s1))
                if ck:
                    net.set_state(ck["state"], ck["adam_steps"])
                else:
                    net.set_params(synth.cnninit.he_init(a.layers, a.channels, seed=0))
            t1 = time.perf_counter()
            hist, step = train(net, X, Y, a.epochs, a.batch, lr=a.lr, seed=k,
                               time_limit=a.train_seconds or None, log=log, step0=step, total_steps=total)
            log({"phase": "train", "shard": k, "epochs": len(hist), "s": time.perf_counter() - t1,
                 "images_per_s": len(hist) * (X.shape[0] // a.batch) * a.batch / (time.perf_counter() - t1),
                 "schedule_step": step, "schedule_total": total})
            del X, Y
        if a.save:
            save_checkpoint(a.save, net, step, total, net.in_scale[0], net.in_scale[1],
                            {"workload": a.workload, "train": a.train, "shards": a.shards, "steps": a.steps,
                             "epochs": a.epochs, "last_shard": shards[-1]})
            log({"phase": "checkpoint", "path": a.save, "schedule_step": step})
    else:
        if not ck:
            raise SystemExit("--eval needs --resume")
        net = Cnn(a.layers, a.channels, nv, nu, max_batch=a.batch, in_scale=(ck["s0"], ck["s1"]))
        net.set_state(ck["state"], ck["adam_steps"])
    if a.test > 0 and (a.eval or a.shard < 0):
        rows = evaluate(net, p, list(range(5000, 5000 + a.test)), a.steps, fn, a.batch, log=log)
        log({"phase": "summary", **summarise(rows)})
    net.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
