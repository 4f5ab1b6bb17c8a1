"""Projection optimisation on top of the projector pair.

* `Project` / `Dose`: torch.autograd.Functions whose backward passes are the
  library's own transposed kernels (projection <-> dose deposit), so any
  torch loss on the dose can drive gradient descent on the projections.
* `plain_init`: the filtered parallel-beam initialisation of the paper's
  Radon baseline (Sec. 2.3): parallel-beam projection of the target with the
  same grid, DMD and angles, Ram-Lak filter along u, negatives clipped, then
  scaled so that the mean dose over target voxels is 1.
* `optimize`: repeated `vam_optimize_step` (projected gradient on the
  dose-threshold loss), stopping when the dose error of Sec. 2.7 falls below
  a tolerance.

Every numerical step runs in libvam's kernels; this module only sequences
calls.
"""
import time

import torch

from . import Geometry, dose_error, ramlak_filter, VAM_TELECENTRIC


class Project(torch.autograd.Function):
    """P = A V (forward projection); dL/dV = A^T dL/dP (dose deposit)."""

    @staticmethod
    def forward(ctx, vol, geom):
        ctx.geom = geom
        return geom.forward(vol.contiguous())

    @staticmethod
    def backward(ctx, grad_p):
        return ctx.geom.back(grad_p.contiguous().float()), None


class Dose(torch.autograd.Function):
    """D = A^T P (dose deposit); dL/dP = A dL/dD (forward projection)."""

    @staticmethod
    def forward(ctx, proj, geom):
        ctx.geom = geom
        return geom.back(proj.contiguous())

    @staticmethod
    def backward(ctx, grad_d):
        return ctx.geom.forward(grad_d.contiguous().float()), None


def project(vol, geom):
    return Project.apply(vol, geom)


def dose(proj, geom):
    return Dose.apply(proj, geom)


def parallel_beam_params(p):
    """Telecentric, chief-ray-only, index-matched version of a geometry on
    the same grid, DMD and angles (the Radon baseline's ray model)."""
    q = dict(p)
    q.update(projector=VAM_TELECENTRIC, pupil=0.0, n_pupil=1, pupil_xy=None,
             r_outer=p["r_inner"], r_inner=p["r_inner"], flags=0)
    return q


def plain_init(target, geom, parallel=None):
    """Filtered parallel-beam starting projections for `target` (device FP32
    volume), scaled so that the mean dose over target voxels is 1."""
    own = parallel is None
    if own:
        parallel = Geometry(parallel_beam_params(geom.p))
    try:
        sino = parallel.forward(target)
        g0 = ramlak_filter(sino, pitch=geom.p["pitch_u"], clip_negative=True)
    finally:
        if own:
            parallel.close()
    d = geom.back(g0)
    mask = target > 0.5
    mean_dose = float(d[mask].mean()) if bool(mask.any()) else float(d.mean())
    if mean_dose > 0:
        g0.mul_(1.0 / mean_dose)
    return g0


def optimize(target, geom, proj=None, steps=50, lr=None, threshold=0.8, sharpness=20.0,
             tol=None, check_every=1, log=None):
    """Projected gradient descent on the dose-threshold loss.  Returns
    (projections, history) where history holds per-step loss, dose error and
    voxel error rate.  lr=None picks the step by backtracking on the first
    step and keeps it fixed."""
    if proj is None:
        proj = plain_init(target, geom)
    proj = proj.contiguous()
    dose_buf = torch.empty_like(target)
    hist = []
    t0 = time.perf_counter()
    if lr is None:
        lr = _first_step(target, geom, proj, threshold, sharpness)
    for it in range(steps):
        loss = geom.optimize_step(target, proj, threshold=threshold, sharpness=sharpness, lr=lr,
                                  dose=dose_buf)
        rec = {"step": it, "loss": loss, "t": time.perf_counter() - t0}
        if check_every and (it % check_every == 0 or it == steps - 1):
            e, rate = dose_error(dose_buf, target, threshold, sharpness)
            rec.update(dose_error=e, voxel_error=rate)
            if tol is not None and e < tol:
                hist.append(rec)
                break
        hist.append(rec)
        if log:
            log(rec)
    return proj, hist


def optimize_stored(target, geom, proj, steps, lr, threshold=0.8, sharpness=20.0):
    """Projected gradient descent on projections stored in reduced precision
    (`proj` in bfloat16 or float16, updated in place): every step is one
    `vam_optimize_step` on the stored projections -- the deposit reads them
    as stored, the loss is reduced in FP64, the gradient is FP32 and the
    updated projections are rounded to the storage type by the library.
    Returns (proj, per-step losses)."""
    if proj.dtype not in (torch.bfloat16, torch.float16):
        raise TypeError("optimize_stored expects bfloat16 or float16 projections")
    hist = []
    for _ in range(steps):
        hist.append(geom.optimize_step(target, proj, threshold=threshold, sharpness=sharpness, lr=lr))
    return proj, hist


def _first_step(target, geom, proj, threshold, sharpness, lr0=None, shrink=0.5, tries=12):
    """Armijo backtracking on a copy of the projections for the first step."""
    base = geom.optimize_step(target, proj.clone(), threshold=threshold, sharpness=sharpness, lr=0.0)
    # scale of the gradient: one step with lr = 1 on a scratch copy
    lr = lr0 if lr0 is not None else 1.0 / max(base, 1e-12)
    for _ in range(tries):
        trial = proj.clone()
        geom.optimize_step(target, trial, threshold=threshold, sharpness=sharpness, lr=lr, want_loss=False)
        after = geom.optimize_step(target, trial.clone(), threshold=threshold, sharpness=sharpness, lr=0.0)
        if after < base:
            return lr
        lr *= shrink
    return lr


def _main(argv=None):
    """Batch optimisation experiment: seeded targets of a workload, plain
    initialisation, `steps` projected gradient steps; one JSON line per
    target with loss, dose error, voxel error rate and time per step."""
    import argparse
    import json
    import sys
    import numpy as np
    import synth
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--targets", type=int, default=8)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--seed0", type=int, default=0)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f16"],
                    help="projection storage; bf16/f16 keep the projections in that type in the library")
    a = ap.parse_args(argv)
    p = synth.workload(a.workload)
    g = Geometry(p)
    gen = synth.random_config3_target if a.workload == "c3" else synth.random_config2_target
    for i in range(a.targets):
        t, _ = gen(p["nx"], p["r_inner"], seed=a.seed0 + i)
        tt = torch.from_numpy(t).to("cuda:0")
        t0 = time.perf_counter()
        g0 = plain_init(tt, g)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        d0 = g.back(g0)
        e0, r0 = dose_error(d0, tt)
        t1 = time.perf_counter()
        if a.storage == "f32":
            proj, hist = optimize(tt, g, proj=g0, steps=a.steps, check_every=max(1, a.steps // 5))
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            last = [h for h in hist if "dose_error" in h][-1]
            rec = {"loss_first": hist[0]["loss"], "loss_last": hist[-1]["loss"],
                   "dose_error_last": last["dose_error"], "voxel_error_last": last["voxel_error"],
                   "steps": len(hist)}
        else:
            lr = _first_step(tt, g, g0, 0.8, 20.0)
            sdt = {"bf16": torch.bfloat16, "f16": torch.float16}[a.storage]
            proj, losses = optimize_stored(tt, g, g0.to(sdt), a.steps, lr)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t1
            e1, r1 = dose_error(g.back(proj), tt)
            rec = {"loss_first": losses[0], "loss_last": losses[-1], "dose_error_last": e1,
                   "voxel_error_last": r1, "steps": len(losses)}
        print(json.dumps({"workload": a.workload, "storage": a.storage, "target_seed": a.seed0 + i,
                          "init_s": t_init, "dose_error_init": e0, "voxel_error_init": r0, **rec,
                          "s_per_step": dt / rec["steps"]}), flush=True)
    g.close()
    return 0


if __name__ == "__main__":
    raise SystemExit(_main())
