"""ctypes binding of libosog.so: structures mirroring include/osog.h and the loader.

Argument marshalling only; every step of the renderer runs in the library's HIP
kernels.  ``load()`` loads the library on first use and raises if it is missing.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libosog.so")

OK, ERR_INVALID_ARGUMENT, ERR_UNSUPPORTED, ERR_WORKSPACE, ERR_HIP, ERR_NOT_INITIALIZED = range(6)
BRIGHTFIELD, DIC, OBLIQUE = 0, 1, 2
STAGES = ["binning", "raster", "pass1", "pass2", "pass3", "adj_pass3", "adj_pass2", "adj_pass1",
          "adj_raster", "batch"]

# Every symbol include/osog.h declares.
EXPORTS = [
    "osog_context_create", "osog_context_destroy", "osog_set_tiling", "osog_get_tiling",
    "osog_workspace_size", "osog_render", "osog_render_noalloc", "osog_render_multi", "osog_render_backward", "osog_batch_workspace_size",
    "osog_batch_render", "osog_batch_error", "osog_set_batch_group", "osog_set_size_tiling", "osog_set_size_radix", "osog_autotune", "osog_bin", "osog_band_info", "osog_philox4x32_10", "osog_profile_enable",
    "osog_profile_read", "osog_cnn_param_count", "osog_cnn_workspace_size", "osog_cnn_forward",
    "osog_cnn_train_step", "osog_conv3x3_workspace_size", "osog_conv3x3", "osog_status_string",
    "osog_last_error", "osog_spectral_workspace_size", "osog_spectral_target", "osog_spectral_loss",
    "osog_set_habits",
]


class Optics(ctypes.Structure):
    _fields_ = [
        ("mode", ctypes.c_int32),
        ("wavelength_um", ctypes.c_double),
        ("na", ctypes.c_double),
        ("n_medium", ctypes.c_double),
        ("pixel_um", ctypes.c_double),
        ("shear_angle_rad", ctypes.c_double),
        ("tilt_fx", ctypes.c_double),
        ("tilt_fy", ctypes.c_double),
        ("photons_mean", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("noise_frame", ctypes.c_uint32),
        ("absorption", ctypes.c_int32),
        ("read_noise", ctypes.c_double),
    ]


class Frame(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("soa", ctypes.c_void_p),
        ("n", ctypes.c_int64),
        ("ld", ctypes.c_int64),
        ("optics", Optics),
        ("globals", ctypes.c_void_p),
        ("opd_out", ctypes.c_void_p),
        ("intensity_out", ctypes.c_void_p),
    ]


class OsogError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__("%s failed: status %d (%s): %s" % (where, status, status_name(status), message))
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libosog.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libosog.so is not built (%s); run python -m paper_2606_21381_amd.build" % path)
    # torch first: the library links libamdhip64.so.7 and binds to the HIP runtime
    # already in the process, torch's; with the library loaded first the process
    # takes the system runtime instead, and torch then finds no GPU
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    sz = ctypes.c_size_t
    sig = {
        "osog_context_create": [ctypes.POINTER(vp), ctypes.c_int],
        "osog_context_destroy": [vp],
        "osog_set_tiling": [vp, i32, i32],
        "osog_get_tiling": [vp, ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "osog_workspace_size": [vp, i32, i32, i64, i32, i32, ctypes.POINTER(sz)],
        "osog_render": [vp, vp, i32, i32, vp, i64, i64, ctypes.POINTER(Optics), vp, vp, vp, vp, sz],
        "osog_render_noalloc": [vp, vp, i32, i32, vp, i64, i64, ctypes.POINTER(Optics), vp, vp, vp],
        "osog_render_multi": [vp, vp, i32, i32, vp, i64, i64, i32, ctypes.POINTER(Optics), vp,
                              ctypes.POINTER(vp), vp, vp, sz],
        "osog_render_backward": [vp, vp, i32, i32, vp, i64, i64, ctypes.POINTER(Optics), vp, vp, vp,
                                 vp, vp, vp, sz],
        "osog_batch_workspace_size": [vp, ctypes.POINTER(Frame), i32, i32, ctypes.POINTER(sz)],
        "osog_batch_render": [vp, vp, ctypes.POINTER(Frame), i32, vp, sz, vp],
        "osog_batch_error": [vp, vp, ctypes.POINTER(i32)],
        "osog_set_batch_group": [vp, i32],
        "osog_set_size_tiling": [vp, i32, i32, i32, i32],
        "osog_set_size_radix": [vp, i32, i32, i32],
        "osog_autotune": [vp, vp, i32, i32, vp, i64, i64, ctypes.POINTER(Optics), vp, vp, vp, sz, i32,
                          ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)],
        "osog_bin": [vp, vp, i32, i32, vp, i64, i64, vp, vp, i64, vp, vp, vp, vp, sz],
        "osog_philox4x32_10": [vp, vp, i64, u32, u32, vp],
        "osog_band_info": [vp, i32, i32, ctypes.POINTER(Optics), ctypes.POINTER(i32), ctypes.POINTER(i32)],
        "osog_profile_enable": [vp, i32],
        "osog_profile_read": [vp, vp, vp],
        "osog_cnn_param_count": [ctypes.POINTER(i64)],
        "osog_cnn_workspace_size": [i32, i32, i32, ctypes.POINTER(sz)],
        "osog_cnn_forward": [vp, vp, i32, i32, i32, vp, vp, vp, vp, sz],
        "osog_cnn_train_step": [vp, vp, i32, i32, i32, vp, vp, vp, vp, vp, i32, ctypes.c_float, vp, vp, vp, sz],
        "osog_conv3x3_workspace_size": [i32, i32, i32, i32, i32, i32, i32, ctypes.POINTER(sz)],
        "osog_conv3x3": [vp, vp, i32, i32, i32, i32, i32, i32, i32, vp, vp, vp, vp, vp, vp, vp, vp, sz],
        "osog_spectral_workspace_size": [i32, i32, ctypes.POINTER(sz)],
        "osog_set_habits": [vp, i32, vp, vp, vp, vp, vp, ctypes.c_uint64],
        "osog_spectral_target": [vp, vp, i32, i32, vp, ctypes.c_float, vp, vp, sz],
        "osog_spectral_loss": [vp, vp, i32, i32, vp, vp, ctypes.c_float, vp, vp, vp, sz],
        "osog_status_string": [ctypes.c_int],
        "osog_last_error": [],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_char_p if name in ("osog_status_string", "osog_last_error") else ctypes.c_int
    _lib = lib
    return lib


def status_name(status: int) -> str:
    names = ["OSOG_OK", "OSOG_ERR_INVALID_ARGUMENT", "OSOG_ERR_UNSUPPORTED", "OSOG_ERR_WORKSPACE",
             "OSOG_ERR_HIP", "OSOG_ERR_NOT_INITIALIZED"]
    return names[status] if 0 <= status < len(names) else "unknown"


def check(status: int, where: str):
    if status != OK:
        msg = load().osog_last_error()
        raise OsogError(status, where, msg.decode() if msg else "")


def make_optics(spec) -> Optics:
    """Optics from any object with the fields of ``workloads.OpticsSpec``."""
    o = Optics()
    o.mode = int(spec.mode)
    o.wavelength_um = float(spec.wavelength_um)
    o.na = float(spec.na)
    o.n_medium = float(spec.n_medium)
    o.pixel_um = float(spec.pixel_um)
    o.shear_angle_rad = float(spec.shear_angle_rad)
    o.tilt_fx = float(spec.tilt_fx)
    o.tilt_fy = float(spec.tilt_fy)
    o.photons_mean = float(spec.photons_mean)
    o.seed = int(spec.seed) & 0xFFFFFFFFFFFFFFFF
    o.noise_frame = int(getattr(spec, "noise_frame", 0)) & 0xFFFFFFFF
    o.absorption = 1 if getattr(spec, "absorption", 0) else 0
    o.read_noise = float(getattr(spec, "read_noise", 0.0))
    return o
