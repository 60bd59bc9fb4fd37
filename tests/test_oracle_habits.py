"""Pins of the oracle's polyhedral habits (Eq. 1) and micro-topography:
  * closed-form chords: octahedron 2 max(0, 1 - |U| - |V|), box 1 on |U|, |V| <= 1,
    tetragonal bipyramid 2 (1 + w - max(|U|, |V|));
  * a rotated, scaled habit placed by add_habits reproduces the closed form at
    every pixel centre, and its summed thickness converges to the volume (4/3) a b h;
  * vertex enumeration finds the octahedron's six vertices;
  * the value noise equals its lattice values at lattice points, is continuous
    across cell edges, stays in [-1, 1] and averages to ~0.
"""
import math

import numpy as np

from oracle import habits as Hb


def test_chord_closed_forms():
    U, V = np.meshgrid(np.linspace(-1.3, 1.3, 41), np.linspace(-1.2, 1.2, 37))
    assert np.max(np.abs(Hb.chord(Hb.octahedron(), U, V) - 2 * np.maximum(0, 1 - np.abs(U) - np.abs(V)))) < 1e-12
    inside = (np.abs(U) <= 1) & (np.abs(V) <= 1)
    assert np.array_equal(Hb.chord(Hb.box(), U, V), np.where(inside, 1.0, 0.0))
    w = 0.5
    tb = np.where(inside, 2 * (1 + w - np.maximum(np.abs(U), np.abs(V))), 0.0)
    assert np.max(np.abs(Hb.chord(Hb.tetragonal_bipyramid(w), U, V) - tb)) < 1e-12


def particle(cx, cy, ang, a, b, h, dn, k):
    return np.array([[cx], [cy], [ang], [a], [b], [h], [dn], [2.0 + k]], dtype=np.float64)


def test_placed_habit_closed_form_and_volume():
    H = W = 128
    cx, cy, ang, a, b, h, dn = 63.3, 60.7, 0.37, 40.0, 30.0, 1.5, 0.03
    hab = [Hb.Habit(Hb.octahedron(), 1.0)]
    out = np.zeros((H, W))
    Hb.add_habits(out, particle(cx, cy, ang, a, b, h, dn, 0), hab, 0)
    jj, ii = np.meshgrid(np.arange(W) + 0.5, np.arange(H) + 0.5)
    c, s = math.cos(ang), math.sin(ang)
    U = (c * (jj - cx) + s * (ii - cy)) / a
    V = (-s * (jj - cx) + c * (ii - cy)) / b
    want = dn * h * 2 * np.maximum(0, 1 - np.abs(U) - np.abs(V))
    assert np.max(np.abs(out - want)) < 1e-12
    vol = out.sum() / dn
    assert abs(vol - 4.0 / 3.0 * a * b * h) < 5e-3 * vol


def test_vertices():
    v = Hb.vertices(Hb.octahedron())
    v = np.unique(np.round(v, 12), axis=0)
    want = np.array([[s * (i == k) for k in range(3)] for i in range(3) for s in (-1, 1)], dtype=np.float64)
    assert v.shape == (6, 3)
    assert np.array_equal(np.sort(v, axis=0), np.sort(want, axis=0))


def test_value_noise():
    seed, cell, k = 1234, 8.0, 1
    for ix, iy in ((0, 0), (3, 5), (17, 2)):
        assert Hb.value_noise(ix * cell, iy * cell, cell, k, seed) == Hb._lattice_value(ix, iy, k, seed)
    # continuity across a cell edge and range
    a = Hb.value_noise(16.0 - 1e-9, 20.3, cell, k, seed)
    b = Hb.value_noise(16.0, 20.3, cell, k, seed)
    assert abs(a - b) < 1e-8
    vals = np.array([Hb.value_noise(x + 0.5, y + 0.5, cell, k, seed) for x in range(0, 512, 3) for y in range(0, 512, 7)])
    assert vals.min() >= -1 and vals.max() <= 1
    assert abs(vals.mean()) < 0.1 and vals.std() > 0.2
