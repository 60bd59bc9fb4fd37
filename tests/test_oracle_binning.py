"""Pins of the oracle's tile binning: brute force, invariants, conservativeness."""
import math

import numpy as np

from oracle import binning, raster
from paper_2606_21381_amd import workloads


def test_pairs_equal_brute_force_per_tile():
    fr = workloads.config0()
    for th, tw in [(16, 16), (8, 32), (32, 8)]:
        b = binning.bin_pairs(fr.soa, fr.H, fr.W, th, tw)
        x0, x1, y0, y1, valid = binning.pixel_boxes(fr.soa, fr.H, fr.W)
        ntx = fr.W // tw
        keys, pids = [], []
        for t in range(b["n_tiles"]):          # tile-major brute force, another loop order
            ty, tx = divmod(t, ntx)
            for p in range(fr.soa.shape[1]):
                if valid[p] and x0[p] < (tx + 1) * tw and x1[p] >= tx * tw \
                        and y0[p] < (ty + 1) * th and y1[p] >= ty * th:
                    keys.append(t)
                    pids.append(p)
        assert np.array_equal(b["keys"], np.array(keys)) and np.array_equal(b["pids"], np.array(pids))
        ts = b["tile_start"]
        assert ts[0] == 0 and ts[-1] == len(keys) and np.all(np.diff(ts) >= 0)
        assert b["counts"].sum() == len(keys)


def test_box_bounds_every_touched_pixel():
    # Every pixel the oracle raster touches lies inside the particle's FP32 box.
    fr = workloads.config1(n=400, size=256)
    x0, x1, y0, y1, valid = binning.pixel_boxes(fr.soa, 256, 256)
    for p in range(0, 400, 7):
        o = raster.opd(fr.soa[:, p:p + 1], 256, 256)
        ii, jj = np.nonzero(o)
        if ii.size:
            assert valid[p]
            assert ii.min() >= y0[p] and ii.max() <= y1[p] and jj.min() >= x0[p] and jj.max() <= x1[p]


def test_invalid_and_off_canvas_particles_emit_nothing():
    s = np.zeros((8, 5), np.float32)
    s[:, 0] = (10, 10, 0, 0, 3, 1, 0.1, 0)           # a = 0
    s[:, 1] = (np.nan, 10, 0, 3, 3, 1, 0.1, 0)       # NaN centre
    s[:, 2] = (-20, 10, 0, 3, 3, 1, 0.1, 1)          # left of the canvas
    s[:, 3] = (10, 100, 0, 3, 3, 1, 0.1, 0)          # below the canvas
    s[:, 4] = (-4.5, 10, 0, 3, 3, 1, 0.1, 0)         # reaches x = 0 through the margin
    b = binning.bin_pairs(s, 64, 64, 16, 16)
    assert list(b["counts"]) == [0, 0, 0, 0, 1]


def test_fp32_recipe_values():
    # Prism a = 5: ext = 5 * 1.41421366f + 1 rounded in FP32; cx 100.25.
    s = np.zeros((8, 1), np.float32)
    s[:, 0] = (100.25, 50.0, 0, 5, 5, 1, 0.1, 0)
    x0, x1, y0, y1, _ = binning.pixel_boxes(s, 256, 256)
    ext = np.float32(np.float32(5) * np.float32(1.41421366)) + np.float32(1)
    assert x0[0] == math.floor(np.float32(100.25) - ext) == 92 and x1[0] == 108
    assert y0[0] == 41 and y1[0] == 58
