"""MI355X-native 3D ray-traced projector pair for tomographic VAM.

Thin ctypes binding over libvam.so (HIP, gfx950): argument marshalling only.
Every step of the projection, the dose deposit and the optimisation step runs
in the library's kernels; PyTorch supplies device memory and streams.  There
is no CPU fallback: importing works without a GPU (for inspection), but any
call needs the built library and a HIP device, and fails loudly otherwise.

Method: Webber et al., "Versatile volumetric additive manufacturing with 3D
ray tracing" -- projection (Sec. 2.4) and dose (Sec. 2.5) along rays traced
through the projector optics and the vial (Sec. 2.1).
"""
import ctypes
import os
import re

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libvam.so")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")
HEADER = os.path.join(INCLUDE, "vam.h")

VAM_OK, VAM_ERR_INVALID_ARG, VAM_ERR_UNSUPPORTED = 0, -1, -2
VAM_ERR_OUT_OF_MEMORY, VAM_ERR_HIP, VAM_ERR_BAD_HANDLE = -3, -4, -5
VAM_F32, VAM_BF16, VAM_F16 = 0, 1, 2
VAM_TELECENTRIC, VAM_THIN_LENS = 0, 1
VAM_NO_FRESNEL = 1
RAY_FIELDS = 12

# vam_set_variant operators and variants (include/vam.h)
OP_FORWARD, OP_DEPOSIT, OP_BOX_EDGE, OP_SEG_ORDER, OP_DEPOSIT_THREADS = 0, 1, 2, 4, 5
OP_SEG_ORDER_FWD, OP_ANGLE_BLOCK_DEPOSIT, OP_ANGLE_BLOCK_FORWARD, OP_FORWARD_LANES = 7, 8, 9, 10
FWD_DEFAULT, FWD_RAY, FWD_PARTIALS = 0, 1, 2
ADJ_DEFAULT, ADJ_RAY, ADJ_GATHER = 0, 1, 2
BOX_EDGES = (8, 12, 16)


class VamError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("libvam status %d: %s" % (status, msg))
        self.status = status


class GeometryDesc(ctypes.Structure):
    """Mirror of vam_geometry_desc (include/vam.h)."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("n_u", ctypes.c_int32), ("n_v", ctypes.c_int32),
        ("pitch_u", ctypes.c_double), ("pitch_v", ctypes.c_double),
        ("n_angles", ctypes.c_int32),
        ("angles_rad", ctypes.POINTER(ctypes.c_double)),
        ("projector", ctypes.c_int32),
        ("focus_distance", ctypes.c_double), ("pupil", ctypes.c_double),
        ("n_pupil", ctypes.c_int32),
        ("pupil_xy", ctypes.POINTER(ctypes.c_double)),
        ("r_outer", ctypes.c_double), ("r_inner", ctypes.c_double),
        ("n_air", ctypes.c_double), ("n_glass", ctypes.c_double),
        ("n_resin", ctypes.c_double), ("alpha", ctypes.c_double),
        ("step", ctypes.c_double), ("flags", ctypes.c_uint32),
    ]


class OptParams(ctypes.Structure):
    _fields_ = [("threshold", ctypes.c_double), ("sharpness", ctypes.c_double),
                ("lr", ctypes.c_double), ("clamp_nonneg", ctypes.c_int32)]


_lib = None
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64P = ctypes.POINTER(ctypes.c_int64)
_DP = ctypes.POINTER(ctypes.c_double)


def lib():
    """The loaded libvam.so.  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libvam.so is not built (run __graft_entry__.build() or "
                              "python paper_2211_03516_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "vam_setup_geometry": [ctypes.POINTER(GeometryDesc), _P, ctypes.POINTER(_P)],
            "vam_destroy_geometry": [_P],
            "vam_forward_project": [_P, _P, _I32, _P, _I32, _I32, _I32, _P],
            "vam_back_project": [_P, _P, _I32, _P, _I32, _I32, _I32, _P],
            "vam_back_project_noalloc": [_P, _P, _I32, _P, _I32, _I32, _I32, _P],
            "vam_optimize_step": [_P, _P, _P, _I32, _P, ctypes.POINTER(OptParams), _DP, _P],
            "vam_debug_fail_allocations": [_I32],
            "vam_ray_table_stats": [_P, _I64P, _I64P],
            "vam_export_rays": [_P, _DP],
            "vam_set_variant": [_P, _I32, _I32],
            "vam_kernel_times": [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)],
            "vam_ramlak_filter": [_P, _P, _I32, _I32, ctypes.c_double, _I32, _P],
            "vam_dose_error": [_P, _P, ctypes.c_int64, ctypes.c_double, ctypes.c_double, _DP, _P],
            "vam_equalize_u8": [_P, ctypes.c_int64, _P, _DP, _P],
            "vam_cnn_create": [_I32, _I32, _I32, _I32, _I32, ctypes.c_float, ctypes.c_float, ctypes.POINTER(_P)],
            "vam_cnn_destroy": [_P],
            "vam_cnn_set_params": [_P, _P],
            "vam_cnn_get_params": [_P, _P],
            "vam_cnn_get_grads": [_P, _P],
            "vam_cnn_get_state": [_P, _P, _I64P],
            "vam_cnn_set_state": [_P, _P, ctypes.c_int64],
            "vam_cnn_forward": [_P, _P, _I32, _P, _P],
            "vam_cnn_loss_grad": [_P, _P, _P, _I32, _DP, _P],
            "vam_cnn_adam_step": [_P, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = ctypes.c_int
            fn.argtypes = args
        L.vam_last_error.restype = ctypes.c_char_p
        L.vam_last_error.argtypes = []
        L.vam_version.restype = ctypes.c_int32
        L.vam_version.argtypes = []
        L.vam_cnn_param_count.restype = ctypes.c_int64
        L.vam_cnn_param_count.argtypes = [_P]
        _lib = L
    return _lib


def header_functions():
    """Names of the functions the headers under include/ declare."""
    names = set()
    for f in sorted(os.listdir(INCLUDE)):
        if f.endswith(".h"):
            text = re.sub(r"/\*.*?\*/", "", open(os.path.join(INCLUDE, f)).read(), flags=re.S)
            names.update(re.findall(r"\b(vam_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def _check(status):
    if status != VAM_OK:
        raise VamError(status, lib().vam_last_error().decode())


def _torch():
    import torch
    return torch


def _dtype_code(dtype):
    torch = _torch()
    codes = {torch.float32: VAM_F32, torch.bfloat16: VAM_BF16, torch.float16: VAM_F16}
    if dtype not in codes:
        raise TypeError("unsupported dtype %s (float32, bfloat16, float16)" % dtype)
    return codes[dtype]


def _stream_ptr(stream):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need_device_tensor(t, name, shape=None, dtypes=None):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a tensor on a HIP device" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if dtypes is not None and t.dtype not in dtypes:
        raise TypeError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtypes))


def make_desc(p):
    """vam_geometry_desc from a parameter dict (see synth.configs) plus the
    numpy arrays it points into (keep them alive while the desc is used)."""
    d = GeometryDesc()
    for k in ("nx", "ny", "nz"):
        setattr(d, k, int(p[k]))
    d.n_u, d.n_v = int(p["nu"]), int(p["nv"])
    d.pitch_u, d.pitch_v = float(p["pitch_u"]), float(p["pitch_v"])
    d.n_angles = int(p["n_angles"])
    keep = []
    if p.get("angles") is not None:
        ang = np.ascontiguousarray(p["angles"], dtype=np.float64)
        keep.append(ang)
        d.angles_rad = ang.ctypes.data_as(_DP)
    d.projector = int(p["projector"])
    d.focus_distance = float(p["focus"])
    d.pupil = float(p["pupil"])
    d.n_pupil = int(p["n_pupil"])
    if p.get("pupil_xy") is not None:
        pxy = np.ascontiguousarray(np.asarray(p["pupil_xy"], dtype=np.float64).reshape(-1, 2))
        keep.append(pxy)
        d.pupil_xy = pxy.ctypes.data_as(_DP)
    d.r_outer, d.r_inner = float(p["r_outer"]), float(p["r_inner"])
    d.n_air, d.n_glass, d.n_resin = float(p["n_air"]), float(p["n_glass"]), float(p["n_resin"])
    d.alpha, d.step = float(p["alpha"]), float(p["step"])
    d.flags = int(p.get("flags", 0))
    return d, keep


class Geometry:
    """A traced printer geometry (vam_setup_geometry) on the current device."""

    def __init__(self, params, stream=None):
        self.p = dict(params)
        desc, keep = make_desc(self.p)
        h = ctypes.c_void_p()
        _check(lib().vam_setup_geometry(ctypes.byref(desc), _stream_ptr(stream), ctypes.byref(h)))
        self._h = h
        self.vol_shape = (self.p["nz"], self.p["ny"], self.p["nx"])
        self.n_angles = self.p["n_angles"]
        self.proj_shape = (self.n_angles, self.p["nv"], self.p["nu"])

    @property
    def handle(self):
        if self._h is None:
            raise VamError(VAM_ERR_BAD_HANDLE, "geometry is closed")
        return self._h

    def close(self):
        if getattr(self, "_h", None) is not None:
            _check(lib().vam_destroy_geometry(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def stats(self):
        """(rays reaching the resin, samples per pass over all angles)."""
        a, b = ctypes.c_int64(), ctypes.c_int64()
        _check(lib().vam_ray_table_stats(self.handle, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def kernel_times(self):
        """(forward ms, dose-deposit ms) of the main kernel of the last calls;
        synchronise the stream first."""
        f, b = ctypes.c_float(), ctypes.c_float()
        _check(lib().vam_kernel_times(self.handle, ctypes.byref(f), ctypes.byref(b)))
        return f.value, b.value

    def export_rays(self):
        """FP64 resin segments, shape (n_pupil, nv, nu, 12)."""
        p = self.p
        out = np.zeros((p["n_pupil"], p["nv"], p["nu"], RAY_FIELDS))
        _check(lib().vam_export_rays(self.handle, out.ctypes.data_as(_DP)))
        return out

    def set_adjoint_variant(self, variant):
        _check(lib().vam_set_variant(self.handle, OP_DEPOSIT, int(variant)))

    def set_forward_variant(self, variant):
        _check(lib().vam_set_variant(self.handle, OP_FORWARD, int(variant)))

    def set_segment_order(self, order, forward=False):
        """Rebuild the box decomposition with segment order 0 (ray),
        1 (length), 2 (pixel parity class), 3, 4 (pixel class mod 3, 4),
        5 (hashed ray index), 6 (pixel, then pupil sample), 7, 8 (order 3
        with runs of 1024 / 2048 segments by length), 9 (pupil sample,
        column, row), 10 (pixel class u mod 3, v mod 2), 11, 12, 13
        (order 10 with runs of 1024 / 512 / 2048 segments by length) or 14,
        15, 16 (ray order with runs of 256 / 1024 segments / the whole box
        by length) for the deposit (or forward)."""
        _check(lib().vam_set_variant(self.handle, OP_SEG_ORDER_FWD if forward else OP_SEG_ORDER, int(order)))

    def set_forward_lanes(self, lanes):
        """March mode of the fixed-point box forward: 1 (one lane per
        segment), 2 (two lanes, alternate samples), 3 (one lane keeping the
        cell's LDS words in registers; the same bits as 1) or 0 (the default:
        3 for FP32/BF16 volumes, 1 for FP16)."""
        _check(lib().vam_set_variant(self.handle, OP_FORWARD_LANES, int(lanes)))

    def set_angle_blocks(self, deposit=None, forward=None):
        """Work order with the angles of a box in blocks (0: boxes fastest,
        1: all angles of a box on one XCD, A >= 2: blocks of A angles)."""
        if deposit is not None:
            _check(lib().vam_set_variant(self.handle, OP_ANGLE_BLOCK_DEPOSIT, int(deposit)))
        if forward is not None:
            _check(lib().vam_set_variant(self.handle, OP_ANGLE_BLOCK_FORWARD, int(forward)))

    def set_deposit_threads(self, n):
        _check(lib().vam_set_variant(self.handle, OP_DEPOSIT_THREADS, int(n)))

    def set_box_edge(self, edge):
        """Rebuild the lab-box decomposition with boxes of `edge` voxels
        (8, 12 or 16)."""
        _check(lib().vam_set_variant(self.handle, OP_BOX_EDGE, int(edge)))

    def forward(self, vol, out=None, angle_begin=0, angle_count=None, out_dtype=None, stream=None):
        """Projections [angle_count, nv, nu] of vol [nz, ny, nx]."""
        torch = _torch()
        _need_device_tensor(vol, "vol", self.vol_shape)
        na = self.n_angles - angle_begin if angle_count is None else angle_count
        if out is None:
            out = torch.empty((na, self.p["nv"], self.p["nu"]), device=vol.device,
                              dtype=out_dtype or torch.float32)
        _need_device_tensor(out, "out", (na, self.p["nv"], self.p["nu"]))
        _check(lib().vam_forward_project(self.handle, vol.data_ptr(), _dtype_code(vol.dtype),
                                         out.data_ptr(), _dtype_code(out.dtype), angle_begin, na,
                                         _stream_ptr(stream)))
        return out

    def back(self, proj, out=None, accumulate=False, angle_begin=0, stream=None):
        """Dose [nz, ny, nx] (FP32) deposited by proj [angle_count, nv, nu]."""
        torch = _torch()
        if not isinstance(proj, torch.Tensor) or proj.dim() != 3:
            raise ValueError("proj must be a 3-d tensor [angles, nv, nu]")
        na = proj.shape[0]
        _need_device_tensor(proj, "proj", (na, self.p["nv"], self.p["nu"]))
        if out is None:
            out = torch.empty(self.vol_shape, device=proj.device, dtype=torch.float32)
            accumulate = False
        _need_device_tensor(out, "out", self.vol_shape, (torch.float32,))
        _check(lib().vam_back_project(self.handle, proj.data_ptr(), _dtype_code(proj.dtype),
                                      out.data_ptr(), int(bool(accumulate)), angle_begin, na,
                                      _stream_ptr(stream)))
        return out

    def optimize_step(self, target, proj, threshold=0.8, sharpness=20.0, lr=1.0, clamp_nonneg=True,
                      dose=None, want_loss=True, stream=None):
        """One projected gradient step on the dose-threshold loss; updates
        proj (float32, bfloat16 or float16, as stored) in place and returns
        the loss before the update (or None)."""
        torch = _torch()
        _need_device_tensor(target, "target", self.vol_shape, (torch.float32,))
        _need_device_tensor(proj, "proj", self.proj_shape, (torch.float32, torch.bfloat16, torch.float16))
        if dose is not None:
            _need_device_tensor(dose, "dose", self.vol_shape, (torch.float32,))
        prm = OptParams(float(threshold), float(sharpness), float(lr), int(bool(clamp_nonneg)))
        loss = ctypes.c_double()
        _check(lib().vam_optimize_step(self.handle, target.data_ptr(), proj.data_ptr(), _dtype_code(proj.dtype),
                                       dose.data_ptr() if dose is not None else None,
                                       ctypes.byref(prm), ctypes.byref(loss) if want_loss else None,
                                       _stream_ptr(stream)))
        return loss.value if want_loss else None


def debug_fail_allocations(n):
    """Make the n-th following device allocation of the library fail (tests
    of the error paths); 0 switches this off."""
    _check(lib().vam_debug_fail_allocations(int(n)))


def ramlak_filter(proj, pitch=1.0, clip_negative=True, out=None, stream=None):
    """Ram-Lak filter along u of every row of proj [..., nu] (FP32, device),
    clipped at zero (the filtered back-projection step of the plain
    initialisation)."""
    torch = _torch()
    _need_device_tensor(proj, "proj", None, (torch.float32,))
    if out is None:
        out = torch.empty_like(proj)
    _need_device_tensor(out, "out", tuple(proj.shape), (torch.float32,))
    nu = proj.shape[-1]
    rows = proj.numel() // nu
    _check(lib().vam_ramlak_filter(proj.data_ptr(), out.data_ptr(), rows, nu, float(pitch),
                                   int(bool(clip_negative)), _stream_ptr(stream)))
    return out


def dose_error(dose, target, threshold=0.8, sharpness=20.0, stream=None):
    """(relative L1 error of the sigmoid-thresholded dose, voxel error rate),
    both reduced in FP64 on the device."""
    torch = _torch()
    _need_device_tensor(dose, "dose", None, (torch.float32,))
    _need_device_tensor(target, "target", tuple(dose.shape), (torch.float32,))
    out = (ctypes.c_double * 2)()
    _check(lib().vam_dose_error(dose.data_ptr(), target.data_ptr(), dose.numel(), float(threshold),
                                float(sharpness), ctypes.cast(out, _DP), _stream_ptr(stream)))
    return out[0], out[1]


def equalize_u8(proj, stream=None):
    """8-bit export of projections: (uint8 tensor, (mean, std, clip))."""
    torch = _torch()
    _need_device_tensor(proj, "proj", None, (torch.float32,))
    out = torch.empty(proj.shape, dtype=torch.uint8, device=proj.device)
    st = (ctypes.c_double * 3)()
    _check(lib().vam_equalize_u8(proj.data_ptr(), proj.numel(), out.data_ptr(), ctypes.cast(st, _DP),
                                 _stream_ptr(stream)))
    return out, (st[0], st[1], st[2])


def version():
    return lib().vam_version()


class Cnn:
    """Learned-initialiser network (include/vam_cnn.h): `layers` 3x3
    convolutions, `channels` hidden channels, H x W images, residual on the
    second input image.  Parameters are a flat FP32 numpy array in the
    library's layout (per layer W[c_out][3][3][c_in], then b[c_out])."""

    def __init__(self, layers=6, channels=64, height=128, width=128, max_batch=16, in_scale=(1.0, 1.0)):
        h = _P()
        _check(lib().vam_cnn_create(layers, channels, height, width, max_batch, float(in_scale[0]),
                                    float(in_scale[1]), ctypes.byref(h)))
        self.handle = h
        self.layers, self.channels, self.height, self.width = layers, channels, height, width
        self.max_batch = max_batch
        self.in_scale = (float(in_scale[0]), float(in_scale[1]))
        self.n_params = int(lib().vam_cnn_param_count(h))

    def close(self):
        if self.handle:
            lib().vam_cnn_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        a = np.ascontiguousarray(params, dtype=np.float32)
        if a.size != self.n_params:
            raise ValueError("expected %d parameters, got %d" % (self.n_params, a.size))
        _check(lib().vam_cnn_set_params(self.handle, a.ctypes.data))

    def get_params(self):
        a = np.empty(self.n_params, dtype=np.float32)
        _check(lib().vam_cnn_get_params(self.handle, a.ctypes.data))
        return a

    def get_state(self):
        """(parameters, Adam first moments, Adam second moments) as one FP32
        array of 3 * n_params, and the Adam step count: a checkpoint."""
        a = np.empty(3 * self.n_params, dtype=np.float32)
        t = ctypes.c_int64()
        _check(lib().vam_cnn_get_state(self.handle, a.ctypes.data, ctypes.byref(t)))
        return a, t.value

    def set_state(self, state, adam_steps):
        a = np.ascontiguousarray(state, dtype=np.float32)
        if a.size != 3 * self.n_params:
            raise ValueError("expected %d state values, got %d" % (3 * self.n_params, a.size))
        _check(lib().vam_cnn_set_state(self.handle, a.ctypes.data, int(adam_steps)))

    def grads(self):
        a = np.empty(self.n_params, dtype=np.float32)
        _check(lib().vam_cnn_get_grads(self.handle, a.ctypes.data))
        return a

    def _images(self, x, name, chans):
        torch = _torch()
        shape = (x.shape[0], chans, self.height, self.width) if chans else (x.shape[0], self.height, self.width)
        _need_device_tensor(x, name, shape, (torch.float32,))
        if not 1 <= x.shape[0] <= self.max_batch:
            raise ValueError("batch of %d outside [1, %d]" % (x.shape[0], self.max_batch))

    def forward(self, x, out=None, stream=None):
        """x [n][2][H][W] -> y [n][H][W] (device FP32)."""
        torch = _torch()
        self._images(x, "x", 2)
        if out is None:
            out = torch.empty((x.shape[0], self.height, self.width), device=x.device, dtype=torch.float32)
        self._images(out, "out", 0)
        _check(lib().vam_cnn_forward(self.handle, x.data_ptr(), x.shape[0], out.data_ptr(), _stream_ptr(stream)))
        return out

    def loss_grad(self, x, t, want_loss=True, stream=None):
        """Loss (scaled squared error) and gradients for one batch."""
        self._images(x, "x", 2)
        self._images(t, "t", 0)
        loss = ctypes.c_double(0.0)
        _check(lib().vam_cnn_loss_grad(self.handle, x.data_ptr(), t.data_ptr(), x.shape[0],
                                       ctypes.byref(loss) if want_loss else None, _stream_ptr(stream)))
        return loss.value if want_loss else None

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _check(lib().vam_cnn_adam_step(self.handle, float(lr), float(beta1), float(beta2), float(eps),
                                       _stream_ptr(stream)))
