"""Oracle of polyhedral crystal habits with micro-topography -- TEST INFRASTRUCTURE ONLY.

Paper Sec. III.A, Eq. 1: a crystal habit is the intersection of M half-spaces
A x <= b.  Readings used here:
  * a habit is given in unit coordinates (U, V, W) by its faces
    (n_x, n_y, n_z, d): {n_x U + n_y V + n_z W <= d}; it must be a bounded,
    non-empty polytope, and `radius` bounds sqrt(U^2 + V^2) over it;
  * a particle of habit k (table row 7 = 2 + k) with centre (cx, cy), angle alpha,
    in-plane scales a, b [px] and height h [um] occupies
    {(x, y) = c + R(alpha) (a U, b V), z = h W};
  * its thickness at pixel (i, j) is the length of the vertical ray through the
    pixel centre inside the solid (Cyrus-Beck clipping of the ray by every face):
        t = h * max(0, W_hi - W_lo),
        W_hi = min over faces with n_z > 0 of (d - n_x U - n_y V) / n_z,
        W_lo = max over faces with n_z < 0 of the same,
    and t = 0 where a face with n_z = 0 has n_x U + n_y V > d;
  * micro-topography (the procedural high-frequency perturbation of the height
    map): where t > 0, t <- max(0, t + amplitude * r(x, y)), r value noise on a
    square lattice of `cell` px in canvas coordinates: lattice values uniform in
    [-1, 1) from the first word of the Philox4x32-10 block at counter
    (lattice x, lattice y, k, 3) under the topography seed, blended with the
    smoothstep weights s(f) = f^2 (3 - 2 f) of the pixel centre's position in
    its cell;
  * the OPD adds dn t (the absorbance dmu t for a nine-row table).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .noise import philox4x32_10


@dataclass
class Habit:
    faces: np.ndarray           # [M][4]: n_x, n_y, n_z, d
    radius: float               # bound on sqrt(U^2 + V^2) over the polytope
    topo_amplitude_um: float = 0.0
    topo_cell_px: float = 8.0


def chord(faces: np.ndarray, U: np.ndarray, V: np.ndarray) -> np.ndarray:
    """W_hi - W_lo clamped at 0 (unit thickness) at unit-coordinate points (U, V)."""
    hi = np.full(np.shape(U), np.inf)
    lo = np.full(np.shape(U), -np.inf)
    ok = np.ones(np.shape(U), dtype=bool)
    for nx, ny, nz, d in np.asarray(faces, dtype=np.float64):
        c = d - nx * U - ny * V
        if nz > 0:
            hi = np.minimum(hi, c / nz)
        elif nz < 0:
            lo = np.maximum(lo, c / nz)
        else:
            ok &= c >= 0
    w = np.where(ok, hi - lo, 0.0)
    return np.maximum(w, 0.0)


def _lattice_value(ix: int, iy: int, k: int, seed: int) -> float:
    w = philox4x32_10((ix & 0xFFFFFFFF, iy & 0xFFFFFFFF, k, 3), (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF))
    return ((w[0] >> 9) + 0.5) * 2.0 ** -22 - 1.0   # (2 u - 1) with u the 23-bit uniform of the noise stage


def value_noise(x: float, y: float, cell: float, k: int, seed: int) -> float:
    gx, gy = x / cell, y / cell
    ix, iy = math.floor(gx), math.floor(gy)
    fx, fy = gx - ix, gy - iy
    sx, sy = fx * fx * (3 - 2 * fx), fy * fy * (3 - 2 * fy)
    v00, v10 = _lattice_value(ix, iy, k, seed), _lattice_value(ix + 1, iy, k, seed)
    v01, v11 = _lattice_value(ix, iy + 1, k, seed), _lattice_value(ix + 1, iy + 1, k, seed)
    a = v00 + (v10 - v00) * sx
    b = v01 + (v11 - v01) * sx
    return a + (b - a) * sy


def add_habits(out: np.ndarray, soa: np.ndarray, habits, topo_seed: int, row: int = 6) -> None:
    """Add row[p] * t_p over the habit particles of `soa` to `out` ([H][W], FP64).
    row 6 gives the OPD (dn), row 8 the absorbance (dmu)."""
    H, W = out.shape
    s = np.asarray(soa, dtype=np.float64)
    for p in range(s.shape[1]):
        shape = s[7, p]
        if not (shape >= 1.5):
            continue
        k = int(math.floor(shape + 0.5)) - 2
        if k < 0 or k >= len(habits):
            continue
        hb = habits[k]
        cx, cy, ang, a, b, h, wgt = s[0, p], s[1, p], s[2, p], s[3, p], s[4, p], s[5, p], s[row, p]
        ext = max(a, b) * hb.radius + 1.0
        j0, j1 = max(0, int(math.floor(cx - ext))), min(W - 1, int(math.ceil(cx + ext)))
        i0, i1 = max(0, int(math.floor(cy - ext))), min(H - 1, int(math.ceil(cy + ext)))
        if j0 > j1 or i0 > i1:
            continue
        jj, ii = np.meshgrid(np.arange(j0, j1 + 1), np.arange(i0, i1 + 1))
        dx, dy = jj + 0.5 - cx, ii + 0.5 - cy
        c, sn = math.cos(ang), math.sin(ang)
        U = (c * dx + sn * dy) / a
        V = (-sn * dx + c * dy) / b
        t = h * chord(hb.faces, U, V)
        if hb.topo_amplitude_um > 0:
            for (r, q) in zip(*np.nonzero(t > 0)):
                x, y = float(jj[r, q]) + 0.5, float(ii[r, q]) + 0.5
                t[r, q] = max(0.0, t[r, q] + hb.topo_amplitude_um * value_noise(x, y, hb.topo_cell_px, k, topo_seed))
        out[i0:i1 + 1, j0:j1 + 1] += wgt * t


def vertices(faces: np.ndarray, tol: float = 1e-9) -> np.ndarray:
    """Vertices of the polytope (every feasible intersection of three face planes)."""
    F = np.asarray(faces, dtype=np.float64)
    pts = []
    M = F.shape[0]
    for a in range(M):
        for b in range(a + 1, M):
            for c in range(b + 1, M):
                A = F[[a, b, c], :3]
                if abs(np.linalg.det(A)) < 1e-12:
                    continue
                x = np.linalg.solve(A, F[[a, b, c], 3])
                if np.all(F[:, :3] @ x <= F[:, 3] + tol):
                    pts.append(x)
    return np.array(pts)


def octahedron() -> np.ndarray:
    """|U| + |V| + |W| <= 1: eight faces."""
    return np.array([[sx, sy, sz, 1.0] for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)], dtype=np.float64)


def box() -> np.ndarray:
    """|U| <= 1, |V| <= 1, 0 <= W <= 1: six faces (two of them vertical)."""
    return np.array([[1, 0, 0, 1], [-1, 0, 0, 1], [0, 1, 0, 1], [0, -1, 0, 1], [0, 0, 1, 1], [0, 0, -1, 0]],
                    dtype=np.float64)


def tetragonal_bipyramid(prism_half_height: float = 0.5) -> np.ndarray:
    """A square prism |U|, |V| <= 1 capped by four-sided pyramids (apex at W = +-(w + 1)),
    the tetragonal habit of lysozyme crystals: four vertical faces and eight caps."""
    w = prism_half_height
    f = [[1, 0, 0, 1], [-1, 0, 0, 1], [0, 1, 0, 1], [0, -1, 0, 1]]
    for sx, sy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        f.append([sx, sy, 1.0, 1.0 + w])
        f.append([sx, sy, -1.0, 1.0 + w])
    return np.array(f, dtype=np.float64)
