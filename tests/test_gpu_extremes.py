"""Edge cases of the forward and adjoint paths against the FP64 oracle.

* Non-square canvases: rows and columns of different lengths through binning,
  the raster and the three FFT passes, with a DIC shear direction and an
  oblique tilt off both axes, so that an index transposed anywhere shows.
* Particle extremes on one canvas: centres outside the canvas, sub-pixel
  particles, particles wider than the canvas, axis-aligned and diagonal angles
  with centres and half-widths on pixel edges.
* The adjoint on a non-square canvas against central differences, and a batch
  of non-square frames against its single renders (bitwise).

Tolerances as in the forward tests (OPD max abs <= 1e-5 um, noiseless image
relative L2 <= 1e-4) and the adjoint tests (per row: relative error <= 1e-3
on components above 1e-3 of the row's largest, cosine >= 0.99999)."""
import math
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
from paper_2606_21381_amd import render, workloads
from tests.gpu_util import dev_globals, dev_soa, need_gpu, oracle_optics, rel_l2, say

pytestmark = pytest.mark.gpu

OPD_TOL = 1e-5
I_TOL = 1e-4


def optics_for(mode):
    if mode == workloads.DIC:
        return replace(workloads.dic_optics(0.0), shear_angle_rad=0.4), [0.8, 1.3, 1.4, 0]
    if mode == workloads.OBLIQUE:
        return workloads.OpticsSpec(mode=mode, na=0.5, tilt_fx=0.2, tilt_fy=-0.35), [-0.9, 0, 0, 0]
    return workloads.OpticsSpec(mode=mode, na=0.4), [1.2, 0, 0, 0]


def compare(soa, H, W, opt, g, label):
    I, opd = render.render(dev_soa(soa), H, W, opt, dev_globals(g), want_opd=True)
    torch.cuda.synchronize()
    ropd = oracle.raster.opd(soa, H, W)
    rI = oracle.optics.intensity(ropd, oracle_optics(opt), float(g[0]), float(g[1]), float(g[2]))
    e_opd = float(np.max(np.abs(opd.cpu().numpy() - ropd)))
    e_I = rel_l2(I.cpu().numpy(), rI)
    say("%s: OPD max abs %.3e um (peak %.3f), I rel L2 %.3e" % (label, e_opd, ropd.max(), e_I))
    assert e_opd <= OPD_TOL and e_I <= I_TOL
    return ropd


@pytest.mark.parametrize("H,W,mode", [(256, 1024, workloads.DIC), (1024, 128, workloads.OBLIQUE),
                                      (64, 2048, workloads.BRIGHTFIELD), (2048, 64, workloads.DIC),
                                      (32, 512, workloads.OBLIQUE)])
def test_non_square_parity(H, W, mode):
    need_gpu()
    say("non-square %dx%d mode %d" % (H, W, mode))
    rng = np.random.Generator(np.random.PCG64(H * 7 + W))
    soa = workloads.f32(workloads.mixed(rng, H * W // 200, H, W))
    opt, g = optics_for(mode)
    compare(soa, H, W, opt, np.array(g, np.float32), "%dx%d mode %d, n=%d" % (H, W, mode, soa.shape[1]))


def extreme_table(seed, H, W):
    """Prisms and ellipsoids (shape 0 / 1 alternating within each group):
    40 centred up to 30 px outside the canvas, 120 sub-pixel (half-widths
    0.05-0.6 px), 6 spanning 80-200 px, 60 at angles k pi/4 with integer or
    half-integer centres and integer half-widths."""
    rng = np.random.Generator(np.random.PCG64(seed))
    groups = []

    def group(n, cx, cy, ang, a, b, h, dn):
        s = np.zeros((8, n))
        s[0], s[1], s[2], s[3], s[4], s[5], s[6] = cx, cy, ang, a, b, h, dn
        s[7] = np.arange(n) % 2
        groups.append(s)

    n = 40
    side = rng.integers(0, 4, n)
    cx = np.where(side == 0, rng.uniform(-30, 0, n), np.where(side == 1, rng.uniform(W, W + 30, n),
                                                             rng.uniform(0, W, n)))
    cy = np.where(side == 2, rng.uniform(-30, 0, n), np.where(side == 3, rng.uniform(H, H + 30, n),
                                                             rng.uniform(0, H, n)))
    group(n, cx, cy, rng.uniform(0, math.pi, n), rng.uniform(5, 40, n), rng.uniform(5, 40, n),
          rng.uniform(0.5, 3, n), rng.uniform(0.01, 0.05, n))
    n = 120
    group(n, rng.uniform(0, W, n), rng.uniform(0, H, n), rng.uniform(0, math.pi, n), rng.uniform(0.05, 0.6, n),
          rng.uniform(0.05, 0.6, n), rng.uniform(0.5, 3, n), rng.uniform(0.01, 0.05, n))
    n = 6
    group(n, rng.uniform(0, W, n), rng.uniform(0, H, n), rng.uniform(0, math.pi, n), rng.uniform(80, 200, n),
          rng.uniform(80, 200, n), rng.uniform(0.1, 0.4, n), rng.uniform(0.005, 0.01, n))
    n = 60
    half = rng.integers(0, 2, (2, n)) * 0.5
    group(n, rng.integers(0, W, n) + half[0], rng.integers(0, H, n) + half[1], rng.integers(0, 5, n) * (math.pi / 4),
          rng.integers(1, 12, n).astype(float), rng.integers(1, 12, n).astype(float), rng.uniform(0.5, 3, n),
          rng.uniform(0.01, 0.05, n))
    s = np.concatenate(groups, axis=1)
    return workloads.f32(s[:, rng.permutation(s.shape[1])])


@pytest.mark.parametrize("mode", [workloads.DIC, workloads.OBLIQUE])
def test_extreme_particles_parity(mode):
    need_gpu()
    H, W = 256, 512
    soa = extreme_table(900 + mode, H, W)
    opt, g = optics_for(mode)
    ropd = compare(soa, H, W, opt, np.array(g, np.float32), "extremes %dx%d mode %d" % (H, W, mode))
    # every group reaches the canvas: the outside centres, the sub-pixel and the spanning particles
    for sel, what in ((soa[3] < 0.7, "sub-pixel"), (soa[3] > 70, "spanning"),
                      ((soa[0] < 0) | (soa[0] >= W) | (soa[1] < 0) | (soa[1] >= H), "outside")):
        only = soa.copy()
        only[6, ~sel] = 0.0
        peak = float(oracle.raster.opd(only, H, W).max())
        say("  %s particles alone: OPD peak %.4f um" % (what, peak))
        assert peak > 0.0


def test_single_particle_and_single_tile_row():
    """One particle; then a 32-row strip (two tile rows) holding particles that
    straddle the boundary between its tile rows and its top and bottom edges."""
    need_gpu()
    opt, g = optics_for(workloads.DIC)
    g = np.array(g, np.float32)
    one = workloads.f32(np.array([[40.3], [23.7], [0.3], [6.0], [6.0], [1.5], [0.04], [0.0]]))
    compare(one, 64, 128, opt, g, "one prism on 64x128")
    rng = np.random.Generator(np.random.PCG64(17))
    s = workloads.mixed(rng, 60, 16, 1024)
    s[1] = rng.uniform(-6, 22, 60)
    compare(workloads.f32(s), 32, 1024, opt, g, "60 particles across a 32x1024 strip")


ROWS = ["cx", "cy", "angle", "a", "b", "height", "dn"]


@pytest.mark.parametrize("H,W", [(64, 128), (128, 32)])
def test_non_square_gradients_vs_fd(H, W):
    need_gpu()
    rng = np.random.Generator(np.random.PCG64(H + 3 * W))
    n = 8
    s = workloads.mixed(rng, n, H, W)
    s[0] = rng.uniform(8, W - 8, n)
    s[1] = rng.uniform(8, H - 8, n)
    s[7] = 0.0        # prisms: exact-area coverage, tight FD agreement
    s[3] = rng.uniform(3, 10, n)
    s[4] = rng.uniform(3, 10, n)
    soa = workloads.f32(s)
    opt, g = optics_for(workloads.DIC)
    g = np.array(g, np.float32)
    w = rng.normal(size=(H, W))
    gs, gg = render.render_backward(dev_soa(soa), H, W, opt, dev_globals(g),
                                    torch.from_numpy(w.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    gs, gg = gs.cpu().double().numpy(), gg.cpu().double().numpy()
    rs, rg, fs, fg = oracle.grad.fd_gradients(soa, H, W, oracle_optics(opt), g, w)
    say("8 prisms on %dx%d, DIC" % (H, W))
    for r, name in enumerate(ROWS):
        keep = ~fs[r]
        got, ref = gs[r][keep], rs[r][keep]
        big = np.abs(ref) > 1e-3 * np.max(np.abs(ref))
        err = float(np.max(np.abs(got[big] - ref[big]) / np.abs(ref[big])))
        cos = float(np.dot(got, ref) / (np.linalg.norm(got) * np.linalg.norm(ref)))
        say("  %-6s max rel err %.2e  cosine %.8f  (%d flagged)" % (name, err, cos, fs[r].sum()))
        assert err <= 1e-3 and cos >= 0.99999, name
    scale = np.max(np.abs(rg[:3]))
    for k in range(3):
        e = abs(gg[k] - rg[k]) / max(abs(rg[k]), 1e-2 * scale)
        say("  global %d: gpu %.6e fd %.6e rel %.2e" % (k, gg[k], rg[k], e))
        assert e <= 1e-3


def test_non_square_batch_is_bitwise_single():
    need_gpu()
    frames = []
    for f, (H, W) in enumerate([(256, 1024), (1024, 256), (128, 2048), (512, 64)]):
        rng = np.random.Generator(np.random.PCG64(60 + f))
        soa = workloads.f32(workloads.mixed(rng, H * W // 300, H, W))
        opt, g = optics_for((workloads.DIC, workloads.OBLIQUE)[f % 2])
        frames.append((dev_soa(soa), H, W, replace(opt, photons_mean=500.0, seed=f + 3), dev_globals(g)))
    singles = [render.render(s, H, W, o, g) for (s, H, W, o, g) in frames]
    torch.cuda.synchronize()
    outs = render.Batch(frames).run()
    torch.cuda.synchronize()
    for f, (a, b) in enumerate(zip(singles, outs)):
        assert a.shape == b.shape == (frames[f][1], frames[f][2])
        assert torch.equal(a, b), f
