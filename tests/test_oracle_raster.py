"""Pins of the oracle's OPD canvas against closed forms, brute force and invariants."""
import math

import numpy as np
import pytest

from oracle import raster


def table(rows):
    """rows: list of (cx, cy, angle, a, b, h, dn, shape) -> [8][n] float32."""
    return np.ascontiguousarray(np.array(rows, dtype=np.float64).T.astype(np.float32))


def test_prism_patch_integral_equals_dn_times_volume():
    # Sum of OPD over a fully contained prism = dn * h * (2a)(2b) exactly (FP64 rounding only).
    rng = np.random.default_rng(10)
    for _ in range(20):
        a, b = rng.uniform(1.5, 12, 2)
        ang = rng.uniform(0, math.pi)
        cx, cy = rng.uniform(30, 98, 2)
        h, dn = rng.uniform(0.5, 3), rng.uniform(0.01, 0.05)
        s = table([(cx, cy, ang, a, b, h, dn, 0)])
        a32, b32, h32, dn32 = (float(v) for v in s[[3, 4, 5, 6], 0])
        opd = raster.opd(s, 128, 128)
        assert abs(opd.sum() - dn32 * h32 * 4 * a32 * b32) <= 1e-12 * dn32 * h32 * 4 * a32 * b32


def test_worked_example_patch_integral():
    # dn 0.03, h 2 um, a = b = 5 px: 0.03 * 2 * 100 = 6.0 px^2 um.
    s = table([(64.3, 61.7, 0.7, 5, 5, 2, 0.03, 0)])
    dn, h = float(s[6, 0]), float(s[5, 0])
    assert abs(raster.opd(s, 128, 128).sum() - dn * h * 100.0) < 1e-12


def test_axis_aligned_box_is_exact():
    # angle 0 and integer-aligned edges: every pixel fully in or fully out.
    s = table([(20, 30, 0, 5, 3, 2.0, 0.25, 0)])
    opd = raster.opd(s, 64, 64)
    expect = np.zeros((64, 64))
    expect[27:33, 15:25] = 0.5
    assert np.array_equal(opd, expect)


def test_diamond_corner_triangles():
    # A square of half-width 1/sqrt2 turned by 45 deg, centred on a pixel corner, is the
    # diamond |x|+|y|<=1: each of the four pixels around the corner holds a 0.5 triangle.
    s = np.zeros((8, 1), dtype=np.float64)
    s[:, 0] = (10.0, 12.0, math.pi / 4, 1 / math.sqrt(2), 1 / math.sqrt(2), 1.0, 1.0, 0.0)
    opd = raster.opd(s, 32, 32)
    for (i, j) in [(11, 9), (11, 10), (12, 9), (12, 10)]:
        assert abs(opd[i, j] - 0.5) < 1e-14
    assert abs(opd.sum() - 2.0) < 1e-13


def test_pixel_area_against_supersampling():
    # Brute force: count 400x400 sub-pixel centres inside the footprint.
    rng = np.random.default_rng(3)
    for _ in range(12):
        ang = rng.uniform(0, math.pi)
        a, b = rng.uniform(0.3, 2.0, 2)
        cx, cy = rng.uniform(-0.5, 1.5, 2)
        c, s_ = math.cos(ang), math.sin(ang)
        us = np.array([-a, a, a, -a])
        vs = np.array([-b, -b, b, b])
        xs, ys = cx + c * us - s_ * vs, cy + s_ * us + c * vs
        area = raster.pixel_area(xs, ys, 0.0, 0.0)
        g = (np.arange(400) + 0.5) / 400
        X, Y = np.meshgrid(g, g)
        u = c * (X - cx) + s_ * (Y - cy)
        v = -s_ * (X - cx) + c * (Y - cy)
        inside = ((np.abs(u) <= a) & (np.abs(v) <= b)).mean()
        assert abs(area - inside) < 0.01


def test_quarter_turn_and_translation_invariance():
    s1 = np.zeros((8, 1))
    s1[:, 0] = (40.3, 33.9, 0.4, 7.0, 4.0, 1.5, 0.02, 0)
    s2 = s1.copy()
    s2[2, 0] += math.pi / 2
    s2[3, 0], s2[4, 0] = 4.0, 7.0     # a quarter turn swaps the half-widths
    o1, o2 = raster.opd(s1, 96, 96), raster.opd(s2, 96, 96)
    assert np.max(np.abs(o1 - o2)) < 1e-13
    s3 = s1.copy()
    s3[0, 0] += 5
    s3[1, 0] += 9
    o3 = raster.opd(s3, 96, 96)
    assert np.max(np.abs(o3[9:, 5:] - o1[:-9, :-5])) < 1e-13


def test_canvas_edge_clips_without_wrap():
    # An axis-aligned box straddling the left edge keeps only its on-canvas part.
    s = table([(1.0, 20.0, 0, 4, 2, 1.0, 1.0, 0)])
    opd = raster.opd(s, 64, 64)
    assert abs(opd.sum() - 5 * 4) < 1e-12     # x in [0, 5) of [-3, 5)
    assert np.all(opd[:, 60:] == 0)


def test_ellipsoid_centre_and_profile():
    # Pixel centre on the particle centre -> full thickness; at u = a/2 -> h sqrt(3/4).
    s = table([(10.5, 10.5, 0, 4, 2, 2.0, 0.5, 1)])
    opd = raster.opd(s, 24, 24)
    assert abs(opd[10, 10] - 1.0) < 1e-12
    assert abs(opd[10, 12] - math.sqrt(0.75)) < 1e-7
    assert opd[10, 15] == 0.0 and opd[13, 10] == 0.0


def test_ellipsoid_volume_convergence():
    # Midpoint rule: sum -> dn * (2/3) pi a b h as the ellipsoid grows.
    rng = np.random.default_rng(7)
    for a, tol in [(10.0, 1e-2), (30.0, 1.5e-3)]:
        errs = []
        for _ in range(10):
            cx, cy = rng.uniform(40, 41, 2)
            s = np.zeros((8, 1))
            s[:, 0] = (cx, cy, rng.uniform(0, math.pi), a, a * 0.8, 1.5, 0.03, 1)
            tot = raster.opd(s, 96, 96).sum()
            ref = 0.03 * 2 / 3 * math.pi * a * a * 0.8 * 1.5
            errs.append(abs(tot - ref) / ref)
        assert max(errs) < tol


def test_overlaps_add_linearly():
    rows = [(30.2, 30.1, 0.3, 6, 6, 1.0, 0.02, 0), (33.0, 31.0, 1.1, 5, 3, 1.2, 0.03, 1)]
    both = raster.opd(table(rows), 64, 64)
    one = raster.opd(table(rows[:1]), 64, 64) + raster.opd(table(rows[1:]), 64, 64)
    assert np.max(np.abs(both - one)) < 1e-15


def test_sampled_pixels_match_full_canvas():
    from paper_2606_21381_amd import workloads
    fr = workloads.config0()
    full = raster.opd(fr.soa, fr.H, fr.W)
    rng = np.random.default_rng(1)
    r, c = rng.integers(0, 256, 500), rng.integers(0, 256, 500)
    assert np.max(np.abs(raster.opd_at(fr.soa, 256, 256, r, c) - full[r, c])) < 1e-13
