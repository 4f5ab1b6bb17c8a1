"""The C-ABI library loads and exports every function include/vam.h
declares; host-side argument checks fail cleanly without touching a GPU."""
import ctypes
import os

import pytest

import paper_2211_03516_amd as vam
import synth


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(vam.LIB_PATH):
        from paper_2211_03516_amd import build
        build.build()
    return vam.lib()


def test_exports_every_declared_function(L):
    names = vam.header_functions()
    assert len(names) >= 10
    for n in names:
        assert hasattr(L, n), n


def test_version_and_empty_error(L):
    assert L.vam_version() >= 10000
    assert L.vam_last_error() == b""


def test_null_and_invalid_descriptors_rejected_on_host(L):
    out = ctypes.c_void_p()
    assert L.vam_setup_geometry(None, None, ctypes.byref(out)) == vam.VAM_ERR_INVALID_ARG
    assert b"NULL" in L.vam_last_error()
    base = synth.workload("c1")
    bad_cases = [
        dict(nx=0), dict(nu=-3), dict(pitch_u=0.0), dict(n_angles=0), dict(projector=7),
        dict(n_pupil=0), dict(r_inner=0.0), dict(r_outer=10.0, r_inner=20.0),
        dict(step=0.0), dict(alpha=-1.0), dict(n_glass=0.5), dict(flags=8),
        dict(projector=1, focus=5.0, r_outer=32.0), dict(pupil=1.5),
        dict(n_pupil=2, pupil_xy=None),
        dict(n_pupil=1, pupil_xy=[[0.9, 0.9]]),
        dict(pitch_v=float("nan")),
    ]
    for kw in bad_cases:
        p = dict(base)
        p.update(kw)
        desc, keep = vam.make_desc(p)
        if "pupil_xy" in kw and kw["pupil_xy"] is None:
            desc.pupil_xy = ctypes.POINTER(ctypes.c_double)()
        st = L.vam_setup_geometry(ctypes.byref(desc), None, ctypes.byref(out))
        assert st == vam.VAM_ERR_INVALID_ARG, (kw, st)
        assert L.vam_last_error().startswith(b"invalid descriptor"), kw
        assert not out.value
    assert L.vam_setup_geometry(ctypes.byref(vam.make_desc(base)[0]), None, None) == vam.VAM_ERR_INVALID_ARG


def test_bad_handles_rejected(L):
    assert L.vam_destroy_geometry(None) == vam.VAM_OK
    a = ctypes.c_int64()
    assert L.vam_ray_table_stats(None, ctypes.byref(a), None) == vam.VAM_ERR_BAD_HANDLE
    assert L.vam_forward_project(None, None, 0, None, 0, 0, 1, None) == vam.VAM_ERR_BAD_HANDLE
    assert L.vam_back_project(None, None, 0, None, 0, 0, 1, None) == vam.VAM_ERR_BAD_HANDLE
    assert L.vam_optimize_step(None, None, None, 0, None, None, None, None) == vam.VAM_ERR_BAD_HANDLE
    assert L.vam_debug_fail_allocations(-1) == vam.VAM_ERR_INVALID_ARG
    assert L.vam_debug_fail_allocations(0) == vam.VAM_OK
    assert L.vam_export_rays(None, None) == vam.VAM_ERR_BAD_HANDLE
    assert L.vam_set_variant(None, 1, 0) == vam.VAM_ERR_BAD_HANDLE
    # a pointer to garbage is not a handle either
    junk = (ctypes.c_uint64 * 64)()
    assert L.vam_ray_table_stats(ctypes.cast(junk, ctypes.c_void_p), None, None) == vam.VAM_ERR_BAD_HANDLE


def test_struct_layouts_match_the_c_compiler(tmp_path):
    """Offsets of every ctypes mirror field equal the C compiler's offsetof
    for the structs declared in include/vam.h."""
    import subprocess
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#define __HIP_PLATFORM_AMD__',
             '#include "vam.h"', 'int main(void) {']
    for cname, mirror in (("vam_geometry_desc", vam.GeometryDesc), ("vam_opt_params", vam.OptParams)):
        lines.append('printf("%%zu\\n", sizeof(%s));' % cname)
        for f, _ in mirror._fields_:
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (cname, f))
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(vam.HEADER))
    subprocess.run(["gcc", "-I", inc, "-I", "/opt/rocm/include", str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = []
    for mirror in (vam.GeometryDesc, vam.OptParams):
        want.append(ctypes.sizeof(mirror))
        want += [getattr(mirror, f).offset for f, _ in mirror._fields_]
    assert got == want
