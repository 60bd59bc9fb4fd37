"""Oracle OPD canvas (paper Sec. III.A Eq. 1, Sec. III.B Eq. 2, Sec. III.C Eq. 7).

TEST INFRASTRUCTURE ONLY: tests, the smoke check and the benchmark's CPU baseline
use this module; the product path never does.

The arithmetic lives in ``raster_oracle.c`` (plain FP64 loops, one thread); this
module compiles it with gcc on first use and wraps it with ctypes.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "raster_oracle.c")
_LIB = os.path.join(_HERE, "_raster_oracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle rasteriser (gcc, -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        i64 = ctypes.c_int64
        p = ctypes.c_void_p
        lib.oracle_opd.argtypes = [ctypes.c_int, ctypes.c_int, p, i64, i64, p]
        lib.oracle_opd_f64.argtypes = [ctypes.c_int, ctypes.c_int, p, i64, i64, p]
        lib.oracle_opd_at.argtypes = [ctypes.c_int, ctypes.c_int, p, i64, i64, p, p, i64, p]
        lib.oracle_pixel_area.argtypes = [p, p, ctypes.c_int, ctypes.c_double, ctypes.c_double]
        lib.oracle_pixel_area.restype = ctypes.c_double
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def opd(soa: np.ndarray, H: int, W: int, habits=None, topo_seed: int = 0) -> np.ndarray:
    """OPD canvas [H][W] in micrometres, FP64.

    ``soa`` is the [8][ld] particle table (rows: cx, cy, angle, a, b, height, dn,
    shape; a ninth row, if present, is ignored).  An FP32 table is widened value
    by value to FP64; an FP64 table is used as is (finite differences step below
    FP32 resolution).
    """
    lib = _load()
    soa = np.ascontiguousarray(soa[:8])
    assert soa.ndim == 2 and soa.shape[0] == 8
    n = soa.shape[1]
    out = np.zeros((H, W), dtype=np.float64)
    if soa.dtype == np.float32:
        lib.oracle_opd(H, W, _ptr(soa), n, n, _ptr(out))
    elif soa.dtype == np.float64:
        lib.oracle_opd_f64(H, W, _ptr(soa), n, n, _ptr(out))
    else:
        raise TypeError("soa must be float32 or float64")
    if habits:
        from . import habits as _habits
        _habits.add_habits(out, soa, habits, topo_seed, row=6)
    return out


def absorbance(soa: np.ndarray, H: int, W: int, habits=None, topo_seed: int = 0) -> np.ndarray:
    """Absorbance canvas tau [H][W], FP64, of a [9][n] table whose row 8 is the
    attenuation contrast dmu = mu_particle - mu_solvent [1/um].

    Eq. 4's Beer-Lambert factor is exp(-h (mu_p - mu_s)) for a particle of
    thickness h; over overlapping particles the exponents add, so
    tau(x) = sum_p dmu_p t_p(x) with the same thickness t_p of Eq. 1 that the OPD
    weights by dn_p.  It is that same integral with dmu in the place of dn.
    """
    soa = np.asarray(soa)
    assert soa.ndim == 2 and soa.shape[0] == 9
    t = np.array(soa[:8], copy=True)
    t[6] = soa[8]
    out = opd(t, H, W)
    if habits:
        from . import habits as _habits
        _habits.add_habits(out, soa, habits, topo_seed, row=8)
    return out


def opd_at(soa: np.ndarray, H: int, W: int, rows, cols) -> np.ndarray:
    """OPD at the listed pixels only (full-size sampled checks)."""
    lib = _load()
    soa = np.ascontiguousarray(soa, dtype=np.float32)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    out = np.zeros(rows.shape[0], dtype=np.float64)
    n = soa.shape[1]
    lib.oracle_opd_at(H, W, _ptr(soa), n, n, _ptr(rows), _ptr(cols), rows.shape[0], _ptr(out))
    return out


def pixel_area(xs, ys, x0: float, y0: float) -> float:
    """Area of the unit pixel [x0,x0+1]x[y0,y0+1] intersected with a convex CCW polygon."""
    lib = _load()
    xs = np.ascontiguousarray(xs, dtype=np.float64)
    ys = np.ascontiguousarray(ys, dtype=np.float64)
    return lib.oracle_pixel_area(_ptr(xs), _ptr(ys), xs.shape[0], float(x0), float(y0))
