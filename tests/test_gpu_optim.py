"""GPU tests of the optimisation layer: Ram-Lak kernel and dose error against
the oracle's numpy definitions, autograd through the hand-written adjoint
against the oracle's gradient, and a short plain-initialised optimisation."""
import math
import sys

import numpy as np
import pytest

import oracle
from oracle import ramlak
import synth
from synth.configs import scaled

torch = pytest.importorskip("torch")
import paper_2211_03516_amd as vam
from paper_2211_03516_amd import optim

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def relL2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


def test_ramlak_kernel_matches_definition():
    rng = synth.SplitMix64(31)
    for nu in (1, 7, 64, 257):
        rows = rng.uniform(5 * nu).reshape(5, nu) - 0.3
        say("ramlak nu", nu)
        for clip in (True, False):
            got = vam.ramlak_filter(torch.from_numpy(rows).float().to(DEV), pitch=0.8,
                                    clip_negative=clip).cpu().numpy()
            ref = ramlak.ramlak_filter(rows, 0.8, clip_negative=clip)
            assert np.abs(got - ref).max() <= 1e-5 * max(np.abs(ref).max(), 1.0)


def test_dose_error_matches_fp64_definition():
    rng = synth.SplitMix64(32)
    n = 100003
    d = rng.uniform(n) * 1.6
    t = (rng.uniform(n) > 0.6).astype(np.float64)
    e, rate = vam.dose_error(torch.from_numpy(d).float().to(DEV), torch.from_numpy(t).float().to(DEV), 0.8, 20.0)
    df = d.astype(np.float32).astype(np.float64)
    sig = 1.0 / (1.0 + np.exp(-20.0 * (df - np.float32(0.8))))
    assert e == pytest.approx(np.abs(sig - t).sum() / t.sum(), rel=1e-9)
    assert rate == pytest.approx(np.mean((df >= np.float32(0.8)) != (t >= 0.5)), abs=1e-12)


def _c1_like(n_angles=30):
    return scaled(synth.workload("c1"), n_angles=n_angles)


def test_autograd_dose_gradient_matches_oracle():
    p = _c1_like()
    og = oracle.Geometry(p)
    t, _ = synth.random_config1_target(64, 32.0, seed=5)
    P0 = oracle.forward(og, t)
    D0 = oracle.adjoint(og, P0)
    g0 = P0 / np.percentile(D0[t > 0], 50)
    _, _, grad_o = oracle.loss_grad(og, t, g0, 20.0, 0.8)
    g = vam.Geometry(p)
    gp = torch.from_numpy(g0).float().to(DEV).requires_grad_(True)
    tt = torch.from_numpy(t).to(DEV)
    d = optim.dose(gp, g)
    loss = ((torch.sigmoid(20.0 * (d - 0.8)) - tt) ** 2).mean()
    loss.backward()
    e = relL2(gp.grad.double().cpu().numpy(), grad_o)
    say("autograd gradient rel-L2 vs oracle %.3e" % e)
    assert e <= 1e-4
    # Project's backward is the deposit: <A x, y> = <x, A^T y> through autograd
    x = torch.from_numpy(t).to(DEV).requires_grad_(True)
    y = torch.rand(g.proj_shape, device=DEV)
    (optim.project(x, g) * y).sum().backward()
    ref = g.back(y)
    assert torch.allclose(x.grad, ref)
    g.close()


def test_plain_init_and_short_optimisation():
    p = scaled(synth.workload("c5"), n_angles=60)
    t, _ = synth.random_config2_target(128, p["r_inner"], seed=1)
    g = vam.Geometry(p)
    tt = torch.from_numpy(t).to(DEV)
    g0 = optim.plain_init(tt, g)
    d0 = g.back(g0)
    mean_t = float(d0[tt > 0.5].mean())
    say("plain init: mean target dose %.6f, min proj %.3e" % (mean_t, float(g0.min())))
    assert mean_t == pytest.approx(1.0, rel=1e-4)
    assert float(g0.min()) >= 0.0
    e0, r0 = vam.dose_error(d0, tt)
    proj, hist = optim.optimize(tt, g, proj=g0.clone(), steps=25)
    say("dose error %.4f -> %.4f, voxel error %.4f -> %.4f, loss %.5f -> %.5f" % (
        e0, hist[-1]["dose_error"], r0, hist[-1]["voxel_error"], hist[0]["loss"], hist[-1]["loss"]))
    assert hist[-1]["loss"] < hist[0]["loss"]
    assert hist[-1]["dose_error"] < e0
    assert float(proj.min()) >= 0.0
    g.close()


def test_equalize_u8_matches_definition():
    from oracle import export
    rng = synth.SplitMix64(41)
    x = (rng.uniform(360 * 64 * 64) ** 3 * 5.0).reshape(360, 64, 64)
    x[0, 0, :8] = -1.0
    xt = torch.from_numpy(x).float().to(DEV)
    q, st = vam.equalize_u8(xt)
    xf = x.astype(np.float32).astype(np.float64)   # the values as stored
    ref, (mean, sd, clip) = export.equalize_u8(xf)
    assert st[0] == pytest.approx(mean, rel=1e-12)
    assert st[1] == pytest.approx(sd, rel=1e-10)
    got = q.cpu().numpy()
    # a level is unique unless the scaled value sits at a half level within
    # the rounding of the FP64 statistics
    v = np.minimum(np.maximum(xf, 0), clip) * (255.0 / clip)
    ambiguous = np.abs(v - np.floor(v) - 0.5) < 1e-9
    assert np.array_equal(got[~ambiguous], ref[~ambiguous])
    assert np.all(np.abs(got[ambiguous].astype(int) - ref[ambiguous].astype(int)) <= 1)
    say("equalize: mean %.6f std %.6f clip %.6f, %d ambiguous" % (mean, sd, clip, int(ambiguous.sum())))


def test_bf16_storage_optimisation_tracks_fp32():
    # c3-style loop with the projections stored in BF16 inside the library:
    # same start, same step size, losses within a few percent of FP32
    p = scaled(synth.workload("c1"), n_angles=30)
    t, _ = synth.random_config1_target(64, 32.0, seed=6)
    g = vam.Geometry(p)
    tt = torch.from_numpy(t).to(DEV)
    g0 = optim.plain_init(tt, g)
    lr = 0.25 * optim._first_step(tt, g, g0, 0.8, 20.0)   # a step size that keeps descending
    p32, h32 = optim.optimize(tt, g, proj=g0.clone(), steps=15, lr=lr)
    p16, h16 = optim.optimize_stored(tt, g, g0.to(torch.bfloat16), 15, lr)
    say("FP32 loss %.5f -> %.5f, BF16 storage %.5f -> %.5f" % (h32[0]["loss"], h32[-1]["loss"], h16[0], h16[-1]))
    assert p16.dtype == torch.bfloat16
    assert h32[-1]["loss"] < h32[0]["loss"] and h16[-1] < h16[0]
    assert h16[0] == pytest.approx(h32[0]["loss"], rel=2e-2)
    assert h16[-1] == pytest.approx(h32[-1]["loss"], rel=5e-2)
    g.close()


@pytest.mark.parametrize("dt", ["bf16", "f16"])
def test_reduced_precision_step_matches_oracle(dt):
    # one vam_optimize_step on projections stored in BF16 / FP16, through the
    # C ABI: the FP64 loss and the dose of the stored values against the
    # oracle, and every updated value within one rounding of the oracle's
    # step g - lr grad taken from the same stored values.  One rounding to
    # nearest is within u of the value, or within half the subnormal spacing
    # below the format's smallest normal (FP16: 2^-25; BF16: 2^-134)
    tdt, u, sub = {"bf16": (torch.bfloat16, 2.0 ** -8, 2.0 ** -134),
                   "f16": (torch.float16, 2.0 ** -11, 2.0 ** -25)}[dt]
    p = scaled(synth.workload("c1"), n_angles=24)
    t, _ = synth.random_config1_target(64, 32.0, seed=8)
    og = oracle.Geometry(p)
    P0 = oracle.forward(og, t)
    D0 = oracle.adjoint(og, P0)
    g0 = torch.from_numpy(P0 * (1.0 / np.percentile(D0[t > 0], 50))).to(DEV, tdt)
    gs = g0.double().cpu().numpy()                       # the values as stored
    loss_o, dose_o, grad_o = oracle.loss_grad(og, t, gs, 20.0, 0.8)
    g = vam.Geometry(p)
    gp = g0.clone()
    dose = torch.empty(g.vol_shape, device=DEV)
    lr = 0.5
    loss = g.optimize_step(torch.from_numpy(t).to(DEV), gp, threshold=0.8, sharpness=20.0, lr=lr, dose=dose)
    want = np.maximum(gs - lr * grad_o, 0.0)
    got = gp.double().cpu().numpy()
    err = np.abs(got - want)
    tol = u * np.abs(want) + sub + 1e-4 * lr * np.abs(grad_o).max()
    say("%s step: loss gpu %.9e oracle %.9e; worst update error / tolerance %.3f"
        % (dt, loss, loss_o, float((err / tol).max())))
    assert loss == pytest.approx(loss_o, rel=1e-5)
    assert relL2(dose.cpu().numpy(), dose_o) <= 1e-5
    assert np.all(err <= tol)
    assert gp.dtype == tdt
    g.close()


def test_paper_pipeline_fin_stack_hex13_export():
    # the paper's chain at a small size: fin-stack target, 13-ray hexagonal
    # pupil, plain filtered start, optimisation, 8-bit export
    from oracle import export
    n = 64
    p = scaled(synth.workload("c5"), nx=n, ny=n, nz=n, nu=n, nv=n, n_angles=48, n_pupil=13,
               pupil_xy=synth.pupil_hex13(), r_outer=30.0, r_inner=28.0,
               focus=synth.workload("c5")["focus"] / 2, pupil=synth.workload("c5")["pupil"] / 2)
    t = synth.fin_stack_target(n, 0.4).astype(np.float32)
    assert t.sum() > 0
    og = oracle.Geometry(p)
    g = vam.Geometry(p)
    # forward parity with the hex-13 pupil table
    P = g.forward(torch.from_numpy(t).to(DEV)).cpu().numpy()
    assert relL2(P, oracle.forward(og, t)) <= 1e-5
    tt = torch.from_numpy(t).to(DEV)
    g0 = optim.plain_init(tt, g)
    e0, _ = vam.dose_error(g.back(g0), tt)
    proj, hist = optim.optimize(tt, g, proj=g0.clone(), steps=20)
    say("fin stack, hex-13 pupil: dose error %.4f -> %.4f" % (e0, hist[-1]["dose_error"]))
    assert hist[-1]["dose_error"] < e0
    q, (mean, sd, clip) = vam.equalize_u8(proj)
    ref, (rmean, rsd, rclip) = export.equalize_u8(proj.double().cpu().numpy())
    assert mean == pytest.approx(rmean, rel=1e-9) and clip == pytest.approx(rclip, rel=1e-9)
    v = np.minimum(np.maximum(proj.double().cpu().numpy(), 0), clip) * (255.0 / clip)
    tie = np.abs(v - np.floor(v) - 0.5) < 1e-9
    assert np.array_equal(q.cpu().numpy()[~tie], ref[~tie])
    assert int(q.min()) == 0 and int(q.max()) >= 128
    g.close()
