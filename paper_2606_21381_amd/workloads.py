"""Seeded synthetic workloads (particle tables, optics, globals).

This module draws inputs only; it holds none of the renderer's arithmetic, so
the GPU path and the CPU oracle can be fed the same tables.  Tables are drawn in
FP64 with numpy's PCG64 generator and rounded to FP32.

SoA table layout, [8][n] float32, one row per attribute:
  0 cx [px]  1 cy [px]  2 angle [rad]  3 a [px]  4 b [px]  5 height [um]  6 dn  7 shape
  (shape 0 = tetragonal prism with half-widths a, b; 1 = ellipsoid with semi-axes a, b)
Absorbing tables (optics.absorption = 1) carry a ninth row, 8 dmu [1/um], the
attenuation contrast mu_particle - mu_solvent of Beer-Lambert absorption.

Recipes (sizes and distributions of the paper's workloads as used here):
  prism      a = b ~ U[3, 12] px, height ~ U[0.5, 3] um, angle ~ U[0, pi)
  ellipsoid  a, b ~ U[2, 10] px, height ~ U[0.5, 2] um (full central thickness), angle ~ U[0, pi)
  centres    uniform over the canvas; dn ~ U[0.01, 0.05]; n_medium 1.33
  optics     lambda 0.55 um, pixel 0.1 um
  absorbing  dmu ~ U[0, 0.4] 1/um (the paper gives no values: up to ~70% amplitude
             loss through the thickest particles)
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

BRIGHTFIELD, DIC, OBLIQUE, DIC_INCOHERENT = 0, 1, 2, 3
SOA_ROWS = 8
SOA_ROWS_ABS = 9


@dataclass
class OpticsSpec:
    """Static optics of a frame; mirrors the C struct ``osog_optics``."""
    mode: int = BRIGHTFIELD
    wavelength_um: float = 0.55
    na: float = 0.4
    n_medium: float = 1.33
    pixel_um: float = 0.1
    shear_angle_rad: float = 0.0
    tilt_fx: float = 0.0
    tilt_fy: float = 0.0
    photons_mean: float = 0.0
    seed: int = 0
    absorption: int = 0
    read_noise: float = 0.0   # Gaussian read noise, photon counts (needs photons_mean > 0)


@dataclass
class Frame:
    H: int
    W: int
    soa: np.ndarray                 # [8][n] float32
    optics: OpticsSpec
    globals4: np.ndarray            # float32[4]: defocus_um, shear_px, bias_rad, 0
    name: str = ""
    extra: dict = field(default_factory=dict)


def prisms(rng: np.random.Generator, n: int, H: int, W: int) -> np.ndarray:
    s = np.zeros((SOA_ROWS, n), dtype=np.float64)
    s[0] = rng.uniform(0, W, n)
    s[1] = rng.uniform(0, H, n)
    s[2] = rng.uniform(0, math.pi, n)
    s[3] = rng.uniform(3, 12, n)
    s[4] = s[3]
    s[5] = rng.uniform(0.5, 3.0, n)
    s[6] = rng.uniform(0.01, 0.05, n)
    s[7] = 0.0
    return s


def ellipsoids(rng: np.random.Generator, n: int, H: int, W: int) -> np.ndarray:
    s = np.zeros((SOA_ROWS, n), dtype=np.float64)
    s[0] = rng.uniform(0, W, n)
    s[1] = rng.uniform(0, H, n)
    s[2] = rng.uniform(0, math.pi, n)
    s[3] = rng.uniform(2, 10, n)
    s[4] = rng.uniform(2, 10, n)
    s[5] = rng.uniform(0.5, 2.0, n)
    s[6] = rng.uniform(0.01, 0.05, n)
    s[7] = 1.0
    return s


def mixed(rng: np.random.Generator, n: int, H: int, W: int) -> np.ndarray:
    """Half prisms, half ellipsoids, randomly interleaved."""
    npr = n // 2
    s = np.concatenate([prisms(rng, npr, H, W), ellipsoids(rng, n - npr, H, W)], axis=1)
    return s[:, rng.permutation(n)] if n else s


def clustered(rng: np.random.Generator, n: int, H: int, W: int, clusters: int = 64, sigma_px: float = 25.0) -> np.ndarray:
    """The mixed table with its centres drawn in clusters (a suspension whose crystals
    aggregate): cluster centres uniform over the canvas, each particle's centre
    Gaussian (sigma_px) around a uniformly chosen cluster, wrapped onto the canvas."""
    s = mixed(rng, n, H, W)
    cc = np.stack([rng.uniform(0, W, clusters), rng.uniform(0, H, clusters)])
    k = rng.integers(0, clusters, n)
    s[0] = np.mod(cc[0, k] + rng.normal(0.0, sigma_px, n), W)
    s[1] = np.mod(cc[1, k] + rng.normal(0.0, sigma_px, n), H)
    return s


def config1_clustered(seed: int = 1, n: int = 40000, size: int = 2048, photons: float = 1000.0) -> Frame:
    """The 2048x2048 DIC frame of config1 with its 40,000 particles in 64 Gaussian
    clusters of sigma 25 px (tiles at the cluster cores hold hundreds of particles)."""
    rng = np.random.Generator(np.random.PCG64(seed + 7000))
    soa = f32(clustered(rng, n, size, size))
    dz = rng.uniform(-2.0, 2.0)
    g = np.array([dz, 1.0, math.pi / 2, 0.0], np.float32)
    return Frame(size, size, soa, dic_optics(photons, seed), g, "dic%d_n%d_clustered" % (size, n))


def with_absorption(rng: np.random.Generator, s: np.ndarray, lo: float = 0.0, hi: float = 0.4) -> np.ndarray:
    """The table with a ninth row, dmu ~ U[lo, hi] 1/um, appended."""
    dmu = rng.uniform(lo, hi, s.shape[1])
    return np.concatenate([s, dmu[None, :].astype(s.dtype)], axis=0)


@dataclass
class HabitSpec:
    """A polyhedral crystal habit in unit coordinates: faces [M][4] (n_x, n_y, n_z, d)
    of {n . (U, V, W) <= d}, a bound on sqrt(U^2 + V^2) over it, and its
    micro-topography (amplitude in um, lattice cell in px, a power of two)."""
    faces: np.ndarray
    radius: float
    topo_amplitude_um: float = 0.0
    topo_cell_px: float = 8.0


def habit_octahedron(**kw) -> HabitSpec:
    f = np.array([[sx, sy, sz, 1.0] for sx in (1, -1) for sy in (1, -1) for sz in (1, -1)], dtype=np.float32)
    return HabitSpec(f, 1.0, **kw)


def habit_tetragonal(cap: float = 0.5, **kw) -> HabitSpec:
    """Square prism |U|, |V| <= 1 between four-sided pyramidal caps reaching W = +-(1 + cap):
    the tetragonal habit of lysozyme crystals."""
    f = [[1, 0, 0, 1], [-1, 0, 0, 1], [0, 1, 0, 1], [0, -1, 0, 1]]
    for sx, sy in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        f += [[sx, sy, 1.0, 1.0 + cap], [sx, sy, -1.0, 1.0 + cap]]
    return HabitSpec(np.array(f, dtype=np.float32), math.sqrt(2.0), **kw)


def habits_table(rng: np.random.Generator, n: int, H: int, W: int, n_habits: int) -> np.ndarray:
    """n particles of habits 0..n_habits-1: in-plane scales a, b ~ U[4, 12] px, height
    ~ U[0.5, 2.5] um, angle ~ U[0, pi), dn ~ U[0.01, 0.05], centres uniform."""
    s = np.zeros((SOA_ROWS, n), dtype=np.float64)
    s[0] = rng.uniform(0, W, n)
    s[1] = rng.uniform(0, H, n)
    s[2] = rng.uniform(0, math.pi, n)
    s[3] = rng.uniform(4, 12, n)
    s[4] = rng.uniform(4, 12, n)
    s[5] = rng.uniform(0.5, 2.5, n)
    s[6] = rng.uniform(0.01, 0.05, n)
    s[7] = 2.0 + rng.integers(0, n_habits, n)
    return s


def artifacts(rng: np.random.Generator, H: int, W: int, organics: int = 0, debris: int = 0,
              fouling: int = 0) -> np.ndarray:
    """Artifact particles of the paper's physical-regularisation pipeline (Sec. III.C:
    out-of-focus organics, slide debris, objective fouling) as rows of an absorbing
    [9][m] table, to be appended to one.  The paper gives no models; readings:
      organics  large faint phase objects: ellipsoids a, b ~ U[20, 60] px, height ~ U[1, 3] um,
                dn ~ U[0.002, 0.006], dmu ~ U[0, 0.02] 1/um (smooth, low-frequency structure)
      debris    small dense absorbers: ellipsoids a, b ~ U[3, 12] px, height ~ U[0.3, 1] um,
                dn ~ U[0.05, 0.15], dmu ~ U[1, 4] 1/um
      fouling   broad faint absorbing smudges: ellipsoids a, b ~ U[80, 250] px, height ~ U[1, 2] um,
                dn = 0, dmu ~ U[0.01, 0.05] 1/um
    Centres are uniform over the canvas, angles U[0, pi)."""
    rows = []
    for count, ab, hh, dn, dmu in ((organics, (20, 60), (1, 3), (0.002, 0.006), (0.0, 0.02)),
                                  (debris, (3, 12), (0.3, 1), (0.05, 0.15), (1.0, 4.0)),
                                  (fouling, (80, 250), (1, 2), (0.0, 0.0), (0.01, 0.05))):
        if count <= 0:
            continue
        s = np.zeros((SOA_ROWS_ABS, count), dtype=np.float64)
        s[0] = rng.uniform(0, W, count)
        s[1] = rng.uniform(0, H, count)
        s[2] = rng.uniform(0, math.pi, count)
        s[3] = rng.uniform(*ab, count)
        s[4] = rng.uniform(*ab, count)
        s[5] = rng.uniform(*hh, count)
        s[6] = rng.uniform(*dn, count) if dn[1] > 0 else 0.0
        s[7] = 1.0
        s[8] = rng.uniform(*dmu, count)
        rows.append(s)
    return np.concatenate(rows, axis=1) if rows else np.zeros((SOA_ROWS_ABS, 0))


def f32(s: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(s.astype(np.float32))


def config0(seed: int = 0) -> Frame:
    """256x256 brightfield, 64 prisms, NA 0.4, defocus 1 um."""
    rng = np.random.Generator(np.random.PCG64(seed))
    soa = f32(prisms(rng, 64, 256, 256))
    opt = OpticsSpec(mode=BRIGHTFIELD, na=0.4)
    return Frame(256, 256, soa, opt, np.array([1.0, 0.0, 0.0, 0.0], np.float32), "bf256_n64")


def dic_optics(photons: float = 1000.0, seed: int = 1) -> OpticsSpec:
    return OpticsSpec(mode=DIC, na=0.5, shear_angle_rad=math.pi / 4, photons_mean=photons, seed=seed)


def config1(seed: int = 1, n: int = 40000, size: int = 2048, photons: float = 1000.0) -> Frame:
    """2048x2048 DIC, 40,000 particles (half prisms, half ellipsoids)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    soa = f32(mixed(rng, n, size, size))
    dz = rng.uniform(-2.0, 2.0)
    g = np.array([dz, 1.0, math.pi / 2, 0.0], np.float32)
    return Frame(size, size, soa, dic_optics(photons, seed), g, "dic%d_n%d" % (size, n))


def config2(seed: int = 2, n_frames: int = 64, sizes=(512, 1024, 2048), n_max: int = 40000):
    """64 frames: sizes uniform over {512,1024,2048}, n log-uniform 100..40000,
    frames [0, n/2) DIC, the rest oblique with tilt 0.3 NA/lambda along +x."""
    frames = []
    for f in range(n_frames):
        rng = np.random.Generator(np.random.PCG64(seed * 1000 + f))
        size = int(rng.choice(np.asarray(sizes)))
        n = int(round(math.exp(rng.uniform(math.log(100), math.log(n_max)))))
        soa = f32(mixed(rng, n, size, size))
        dz = rng.uniform(-2.0, 2.0)
        if f < n_frames // 2:
            opt = dic_optics(1000.0, seed * 1000 + f)
            g = np.array([dz, 1.0, math.pi / 2, 0.0], np.float32)
        else:
            na, lam = 0.5, 0.55
            opt = OpticsSpec(mode=OBLIQUE, na=na, tilt_fx=0.3 * na / lam, photons_mean=1000.0,
                             seed=seed * 1000 + f)
            g = np.array([dz, 0.0, 0.0, 0.0], np.float32)
        frames.append(Frame(size, size, soa, opt, g, "batch%d" % f))
    return frames


@dataclass
class InverseProblem:
    target: Frame                   # true parameters
    init: Frame                     # perturbed start
    dn_true: float
    w_true: np.ndarray


def config3(seed: int = 3, n: int = 500, size: int = 1024) -> InverseProblem:
    """1024x1024 noiseless DIC target from 500 prisms with one shared dn; the
    start perturbs globals by x(1 + U[-0.2, 0.2]) and each prism's x, y, half-width
    by +-U[0, 3] px and angle by +-U[0, 0.2] rad (half-width kept >= 1 px)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    s = prisms(rng, n, size, size)
    dn = rng.uniform(0.01, 0.05)
    s[6] = dn
    dz = rng.uniform(-2.0, 2.0)
    g = np.array([dz, 1.0, math.pi / 2, 0.0])
    opt = dic_optics(0.0, seed)
    target = Frame(size, size, f32(s), opt, g.astype(np.float32), "inverse_target")
    p = s.copy()
    sign = lambda k: rng.choice(np.array([-1.0, 1.0]), k)
    p[0] += sign(n) * rng.uniform(0, 3, n)
    p[1] += sign(n) * rng.uniform(0, 3, n)
    p[2] += sign(n) * rng.uniform(0, 0.2, n)
    w = np.maximum(p[3] + sign(n) * rng.uniform(0, 3, n), 1.0)
    p[3] = w
    p[4] = w
    fac = 1.0 + rng.uniform(-0.2, 0.2, 4)
    p[6] = dn * fac[0]
    g0 = np.array([dz * fac[1], 1.0 * fac[2], (math.pi / 2) * fac[3], 0.0])
    init = Frame(size, size, f32(p), replace(opt), g0.astype(np.float32), "inverse_init")
    return InverseProblem(target, init, float(dn), s[3].copy())


def crop_globals(rng: np.random.Generator):
    """Training distribution of the learned initializer's targets."""
    dn = rng.uniform(0.01, 0.05)
    dz = rng.uniform(-2.0, 2.0)
    s = rng.uniform(0.8, 1.2)
    th = (math.pi / 2) * rng.uniform(0.8, 1.2)
    return dn, dz, s, th


def crop(rng: np.random.Generator, size: int = 256, n_mean: float = 31.0):
    """One training crop: prisms at the 500-per-1024^2 density with one shared dn."""
    dn, dz, s, th = crop_globals(rng)
    n = max(1, int(rng.poisson(n_mean * (size / 256.0) ** 2)))
    t = prisms(rng, n, size, size)
    t[6] = dn
    return f32(t), np.array([dz, s, th, 0.0], np.float32), np.array([dn, dz, s, th])
