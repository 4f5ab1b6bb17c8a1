"""Error paths of the C ABI on the GPU: a device allocation that fails
(forced with vam_debug_fail_allocations) must leave every handle either
unchanged or refusing to run, never half-built, and the next call without
the failure must work."""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from synth.configs import scaled

torch = pytest.importorskip("torch")
import paper_2211_03516_amd as vam

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _p(n=32, n_angles=6):
    F = (n / 2) / math.tan(math.radians(10))
    return scaled(synth.workload("c2"), nx=n, ny=n, nz=n, nu=n, nv=n, focus=F,
                  pupil=F * math.tan(math.radians(6.1)), n_pupil=4, r_outer=0.47 * n,
                  r_inner=0.44 * n, alpha=0.02, n_angles=n_angles)


def _inputs(p, seed):
    rng = synth.SplitMix64(seed)
    n = p["nx"]
    x = torch.from_numpy(rng.uniform(n ** 3).reshape(n, n, n).astype(np.float32)).to(DEV)
    y = torch.from_numpy(rng.uniform(p["n_angles"] * n * n).reshape(p["n_angles"], n, n)
                         .astype(np.float32)).to(DEV)
    return x, y


@pytest.fixture(autouse=True)
def _hook_off():
    yield
    vam.debug_fail_allocations(0)


def test_failed_box_rebuild_refuses_then_recovers():
    p = _p()
    x, y = _inputs(p, 51)
    g = vam.Geometry(p)
    P0, D0 = g.forward(x), g.back(y)
    failed = 0
    for k in range(1, 40):
        say("rebuild with allocation %d failing" % k)
        vam.debug_fail_allocations(k)
        try:
            g.set_box_edge(8)
        except vam.VamError as e:
            vam.debug_fail_allocations(0)
            assert e.status == vam.VAM_ERR_OUT_OF_MEMORY
            failed += 1
            # no box decomposition now: both operators refuse, nothing runs
            with pytest.raises(vam.VamError):
                g.forward(x)
            with pytest.raises(vam.VamError):
                g.back(y)
            g.set_box_edge(12)
            assert torch.equal(g.forward(x), P0)
            assert float((g.back(y) - D0).abs().max()) <= 1e-6 * float(D0.abs().max())
            continue
        vam.debug_fail_allocations(0)
        break   # the rebuild makes fewer than k allocations
    say("%d rebuild allocations failed in turn" % failed)
    assert failed >= 8
    g.close()


def test_failed_setup_and_first_step_allocations():
    p = _p(24, n_angles=4)
    t = torch.zeros((24, 24, 24), device=DEV)
    t[8:16, 8:16, 8:16] = 1.0
    # every allocation of the set-up in turn: an error, and no handle
    for k in range(1, 40):
        vam.debug_fail_allocations(k)
        try:
            g = vam.Geometry(p)
        except vam.VamError as e:
            assert e.status == vam.VAM_ERR_OUT_OF_MEMORY
            continue
        finally:
            vam.debug_fail_allocations(0)
        break
    say("set-up succeeded once %d allocations were allowed to pass" % (k - 1))
    assert k > 5
    # the optimisation step's buffers: each of its four allocations in turn
    proj = g.forward(t)
    ref = proj.clone()
    g.optimize_step(t, ref, lr=0.1, want_loss=False)
    for k in range(1, 5):
        g2 = vam.Geometry(p)
        gp = proj.clone()
        vam.debug_fail_allocations(k)
        with pytest.raises(vam.VamError):
            g2.optimize_step(t, gp, lr=0.1)
        vam.debug_fail_allocations(0)
        assert torch.equal(gp, proj)          # nothing was launched
        g2.optimize_step(t, gp, lr=0.1)
        assert float((gp - ref).abs().max()) <= 1e-5 * float(ref.abs().max())
        g2.close()
    g.close()


def test_failed_first_forward_allocations():
    """The forward's first call allocates its 64-bit fixed-point projections
    and the volume maximum: either allocation failing is an error that writes
    nothing to the output, and the next call gives the same projections as
    a handle whose first call succeeded."""
    p = _p(24, n_angles=4)
    t = torch.zeros((24, 24, 24), device=DEV)
    t[6:18, 8:16, 5:19] = 1.0
    g0 = vam.Geometry(p)
    ref = g0.forward(t)
    g0.close()
    for k in (1, 2):
        g = vam.Geometry(p)
        out = torch.full_like(ref, 7.0)
        vam.debug_fail_allocations(k)
        try:
            with pytest.raises(vam.VamError) as e:
                g.forward(t, out=out)
            assert e.value.status == vam.VAM_ERR_OUT_OF_MEMORY
        finally:
            vam.debug_fail_allocations(0)
        torch.cuda.synchronize()
        assert bool((out == 7.0).all())
        assert torch.equal(g.forward(t), ref)
        g.close()
