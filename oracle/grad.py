"""Oracle gradients by FP64 central finite differences -- TEST INFRASTRUCTURE ONLY.

The paper's forward model is differentiable end to end (Sec. III.C, after Eq. 7:
the gradient of the image with respect to the state tensor is kept).  The oracle
states that gradient by its definition: for a real loss L(I) = sum_ij g_ij I_ij,

    dL/dp ~ (L(p + d) - L(p - d)) / (2 d),   d = 1e-5 in natural units (px, rad, um, 1),

evaluated on an FP64 copy of the particle table and FP64 globals.  Each estimate
is repeated at d/2; components whose two estimates disagree by more than 1e-6
relative (and more than the rounding noise of the difference) are flagged (a prism vertex or edge crossing a pixel boundary inside the
stencil makes the thickness only piecewise smooth there).
"""
from __future__ import annotations

import numpy as np

from . import optics as _optics
from . import raster as _raster


def image64(soa64: np.ndarray, H: int, W: int, optics, g64, habits=None, topo_seed: int = 0) -> np.ndarray:
    """Noiseless image of an FP64 table; a [9][n] table is an absorbing one."""
    soa64 = np.asarray(soa64, dtype=np.float64)
    opd = _raster.opd(soa64, H, W, habits, topo_seed)
    tau = _raster.absorbance(soa64, H, W, habits, topo_seed) if soa64.shape[0] == 9 else None
    return _optics.intensity(opd, optics, float(g64[0]), float(g64[1]), float(g64[2]), tau=tau)


def loss(soa64, H, W, optics, g64, weights, habits=None, topo_seed: int = 0) -> float:
    """L = sum_ij weights_ij * I_ij (a linear probe of the noiseless image)."""
    return float(np.sum(weights * image64(soa64, H, W, optics, g64, habits, topo_seed)))


def _central(f, x0: float, d: float) -> float:
    return (f(x0 + d) - f(x0 - d)) / (2.0 * d)


def fd_gradients(soa, H, W, optics, globals4, weights, rows=(0, 1, 2, 3, 4, 5, 6),
                 delta: float = 1e-5, habits=None, topo_seed: int = 0):
    """FD gradients of sum(weights * I) w.r.t. SoA rows ``rows`` and globals 0..2.

    Returns (grad_soa [rows of the table][n] FP64 with untouched rows zero,
    grad_globals [3], flags_soa bool like grad_soa, flags_globals [3] bool).
    """
    soa64 = np.array(soa, dtype=np.float64)
    g64 = np.array(globals4, dtype=np.float64)
    D, n = soa64.shape
    # rounding noise of a central difference is ~ eps |L| / d; never flag below it
    floor = 1e-9 * max(abs(loss(soa64, H, W, optics, g64, weights, habits, topo_seed)), 1.0)
    gs = np.zeros((D, n))
    fs = np.zeros((D, n), dtype=bool)
    for r in rows:
        for p in range(n):
            def f(v, r=r, p=p):
                s = soa64.copy()
                s[r, p] = v
                return loss(s, H, W, optics, g64, weights, habits, topo_seed)
            x0 = soa64[r, p]
            e1 = _central(f, x0, delta)
            e2 = _central(f, x0, delta / 2)
            gs[r, p] = e2
            fs[r, p] = abs(e1 - e2) > max(1e-6 * max(abs(e1), abs(e2)), floor)
    gg = np.zeros(3)
    fg = np.zeros(3, dtype=bool)
    for k in range(3):
        def f(v, k=k):
            g = g64.copy()
            g[k] = v
            return loss(soa64, H, W, optics, g, weights, habits, topo_seed)
        e1 = _central(f, g64[k], delta)
        e2 = _central(f, g64[k], delta / 2)
        gg[k] = e2
        fg[k] = abs(e1 - e2) > max(1e-6 * max(abs(e1), abs(e2)), floor)
    return gs, gg, fs, fg


def mse(I: np.ndarray, target: np.ndarray) -> float:
    """Inverse-rendering loss: mean squared error against a pixel-aligned target."""
    d = np.asarray(I, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d))


def directional_fd(soa, H, W, optics, globals4, weights, v_soa, v_glob, delta: float = 1e-5):
    """Central differences of L = sum(weights * I) along one direction of the whole
    parameter vector (every table entry and the three globals at once):
    (L(p + d v) - L(p - d v)) / (2 d), at d and at d/2.  This is J v for the linear
    probe, the left side of the dot-product identity <J v, w> = <v, J^T w>."""
    soa64 = np.array(soa, dtype=np.float64)
    g64 = np.array(globals4, dtype=np.float64)
    v_soa = np.asarray(v_soa, dtype=np.float64)
    v_glob = np.asarray(v_glob, dtype=np.float64)

    def L(t):
        g = g64.copy()
        g[:3] += t * v_glob[:3]
        return loss(soa64 + t * v_soa, H, W, optics, g, weights)

    return (L(delta) - L(-delta)) / (2 * delta), (L(delta / 2) - L(-delta / 2)) / delta


def ellipsoid_rim_margin(soa, H: int, W: int) -> np.ndarray:
    """Per particle: min over canvas pixel centres of |1 - q|, q = (u/a)^2 + (v/b)^2
    the centre's normalised radius in the ellipsoid's frame (FP64); inf for other
    shapes.  The centre-sampled thickness h sqrt(1 - q) has unbounded slope at the
    rim, so a finite difference is well conditioned only where no pixel centre lies
    close to it."""
    s = np.asarray(soa, dtype=np.float64)
    out = np.full(s.shape[1], np.inf)
    for p in np.nonzero(s[7] == 1.0)[0]:
        cx, cy, ang, a, b = s[0, p], s[1, p], s[2, p], s[3, p], s[4, p]
        r = max(a, b) + 2.0
        x = np.arange(max(0, int(np.floor(cx - r))), min(W - 1, int(np.floor(cx + r))) + 1) + 0.5
        y = np.arange(max(0, int(np.floor(cy - r))), min(H - 1, int(np.floor(cy + r))) + 1) + 0.5
        if x.size == 0 or y.size == 0:
            continue
        dx, dy = np.meshgrid(x - cx, y - cy)
        c, sn = np.cos(ang), np.sin(ang)
        u, v = c * dx + sn * dy, -sn * dx + c * dy
        q = (u / a) ** 2 + (v / b) ** 2
        out[p] = float(np.min(np.abs(1.0 - q)))
    return out
