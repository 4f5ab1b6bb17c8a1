"""The allocation-free deposit (vam_back_project_noalloc) through the C ABI:
the same dose as vam_back_project on two calls in a row, the second with a
smaller geometry, and a clear refusal of grids beyond its scratch array."""
import ctypes
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


def _p(n, n_angles):
    F = (n / 2) / math.tan(math.radians(10))
    return scaled(synth.workload("c2"), nx=n, ny=n, nz=n, nu=n, nv=n, focus=F,
                  pupil=F * math.tan(math.radians(6.1)), n_pupil=4, r_outer=0.47 * n,
                  r_inner=0.44 * n, alpha=0.02, n_angles=n_angles)


def _noalloc(g, y, out, accumulate=0, angle_begin=0):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return vam.lib().vam_back_project_noalloc(g.handle, y.data_ptr(), vam.VAM_F32, out.data_ptr(),
                                              int(accumulate), angle_begin, y.shape[0], s)


def test_noalloc_deposit_matches_the_allocating_entry_point():
    rng = synth.SplitMix64(71)
    for n, na in ((64, 24), (40, 10)):           # second call: a smaller input
        p = _p(n, na)
        say("noalloc deposit %d^3, %d angles" % (n, na))
        g = vam.Geometry(p)
        y = torch.from_numpy(rng.uniform(na * n * n).reshape(na, n, n).astype(np.float32)).to(DEV)
        ref = g.back(y)
        got = torch.full(g.vol_shape, 7.0, device=DEV)
        assert _noalloc(g, y, got) == vam.VAM_OK, vam.lib().vam_last_error()
        torch.cuda.synchronize()
        r, x = ref.double(), got.double()
        rel = float((x - r).norm() / r.norm())
        mx = float((x - r).abs().max() / r.abs().max())
        say("  vs vam_back_project: rel-L2 %.3e, max element %.3e" % (rel, mx))
        # the same kernels; only the free order of the FP64 atomic adds differs
        assert rel <= 1e-6 and mx <= 2.0 ** -22
        # and the oracle's bar
        Do = oracle.adjoint(oracle.Geometry(p), y.double().cpu().numpy())
        assert float(np.linalg.norm(x.cpu().numpy() - Do) / np.linalg.norm(Do)) <= 1e-5
        # accumulate into the result and an angle sub-range
        acc = got.clone()
        assert _noalloc(g, y[3:7].contiguous(), acc, accumulate=1, angle_begin=3) == vam.VAM_OK
        part = g.back(y[3:7].contiguous(), angle_begin=3)
        torch.cuda.synchronize()
        assert float((acc.double() - got.double() - part.double()).abs().max()) <= 1e-5 * float(part.abs().max())
        g.close()


def test_noalloc_deposit_refuses_large_grids_and_the_gather():
    p = dict(_p(16, 2), nx=258, ny=258, nz=258, nu=4, nv=4, r_outer=5.0, r_inner=4.5, n_pupil=1,
             pupil_xy=None)
    g = vam.Geometry(p)
    y = torch.ones((2, 4, 4), device=DEV)
    out = torch.empty(g.vol_shape, device=DEV)
    assert _noalloc(g, y, out) == vam.VAM_ERR_UNSUPPORTED
    assert b"scratch" in vam.lib().vam_last_error()
    g.close()
    g = vam.Geometry(_p(24, 3))
    g.set_adjoint_variant(vam.ADJ_GATHER)
    y = torch.ones((3, 24, 24), device=DEV)
    out = torch.empty(g.vol_shape, device=DEV)
    assert _noalloc(g, y, out) == vam.VAM_ERR_UNSUPPORTED
    g.set_adjoint_variant(vam.ADJ_RAY)
    assert _noalloc(g, y, out) == vam.VAM_OK
    torch.cuda.synchronize()
    ref = g.back(y)
    assert float((out - ref).abs().max()) <= 1e-6 * float(ref.abs().max())
    g.close()
