"""Oracle tile binning -- TEST INFRASTRUCTURE ONLY.

The scatter-add composition of paper Sec. III.C (Eq. 7) isolates each particle's
on-canvas pixels by a boolean mask over its patch.  The GPU path replaces the
atomic scatter by a sorted list of (tile, particle) pairs; this module states
that list by its plain definition so the GPU list can be compared bit for bit.

The per-particle pixel box uses only IEEE FP32 operations that are exactly
rounded everywhere (multiply, add, max, floor) and no fused multiply-add, so
that any correct implementation reproduces it exactly:

    ext = max(a, b) * 1.41421366f + 1   for a prism (1.41421366f is the float just above sqrt 2:
                                          it bounds the footprint's circumradius sqrt(a^2+b^2))
    ext = max(a, b) + 1                 for an ellipsoid (0.5 <= shape < 1.5)
    ext = max(a, b) * R_k + 1           for a polyhedral habit k = floor(shape + 0.5) - 2 with
                                          the habit's bounding radius R_k (FP32); no pairs for a
                                          habit index the frame does not define
    x0 = floor(cx - ext), x1 = floor(cx + ext)   (same for y), clamped to the canvas
    no pairs if a <= 0, b <= 0, any bound is NaN, or the box misses the canvas.

Tiles are tile_h x tile_w pixel blocks, key = ty * (W / tile_w) + tx.  The
result is the list of (key, pid) sorted ascending by (key, pid), which is
unique, plus tile_start[k] = index of the first pair with key >= k.
"""
from __future__ import annotations

import numpy as np

SQRT2_UP = np.float32(1.41421366)


def pixel_boxes(soa: np.ndarray, H: int, W: int, habit_radius=None):
    """Per-particle clamped pixel box (x0, x1, y0, y1) and a validity mask (FP32 recipe).
    habit_radius: FP32 bounding radii of the frame's polyhedral habits (or None)."""
    soa = np.asarray(soa, dtype=np.float32)
    cx, cy, a, b, shape = soa[0], soa[1], soa[3], soa[4], soa[7]
    one = np.float32(1.0)
    R = np.asarray(habit_radius if habit_radius is not None else [], dtype=np.float32)
    with np.errstate(invalid="ignore", over="ignore"):
        valid = (a > 0) & (b > 0)
        m = np.where(valid, np.maximum(a, b), np.float32(0.0)).astype(np.float32)
        hab = shape >= np.float32(1.5)
        k = np.where(hab, np.floor(shape + np.float32(0.5)) - np.float32(2.0), np.float32(0.0))
        known = hab & (k >= 0) & (k < R.size)
        valid &= ~hab | known
        Rk = np.where(known, R[np.clip(k, 0, max(R.size - 1, 0)).astype(np.int64)] if R.size else np.float32(0),
                      np.float32(0.0)).astype(np.float32)
        ext = np.where(shape < np.float32(0.5), m * SQRT2_UP + one,
                       np.where(hab, (m * Rk).astype(np.float32) + one, m + one)).astype(np.float32)
        fx0 = np.floor(cx - ext)
        fx1 = np.floor(cx + ext)
        fy0 = np.floor(cy - ext)
        fy1 = np.floor(cy + ext)
        valid &= (fx0 <= fx1) & (fy0 <= fy1)
        valid &= (fx1 >= 0) & (fy1 >= 0) & (fx0 <= np.float32(W - 1)) & (fy0 <= np.float32(H - 1))
    x0 = np.where(valid, np.maximum(fx0, 0), 0).astype(np.int64)
    x1 = np.where(valid, np.minimum(fx1, W - 1), -1).astype(np.int64)
    y0 = np.where(valid, np.maximum(fy0, 0), 0).astype(np.int64)
    y1 = np.where(valid, np.minimum(fy1, H - 1), -1).astype(np.int64)
    return x0, x1, y0, y1, valid


def bin_pairs(soa: np.ndarray, H: int, W: int, tile_h: int, tile_w: int, habit_radius=None):
    """Sorted (tile key, particle id) pairs of the particle table.

    Returns a dict with int32 arrays ``keys``, ``pids``, ``tile_start``
    (n_tiles + 1 entries), ``counts`` (pairs per particle) and ``emit_start``
    (exclusive prefix sum of counts: where a particle's pairs begin in
    particle-major emission order).
    """
    assert H % tile_h == 0 and W % tile_w == 0
    ntx, nty = W // tile_w, H // tile_h
    x0, x1, y0, y1, valid = pixel_boxes(soa, H, W, habit_radius)
    n = x0.shape[0]
    keys, pids, counts = [], [], np.zeros(n, dtype=np.int64)
    for p in range(n):
        if not valid[p]:
            continue
        tx0, tx1 = x0[p] // tile_w, x1[p] // tile_w
        ty0, ty1 = y0[p] // tile_h, y1[p] // tile_h
        for ty in range(ty0, ty1 + 1):
            for tx in range(tx0, tx1 + 1):
                keys.append(ty * ntx + tx)
                pids.append(p)
        counts[p] = (tx1 - tx0 + 1) * (ty1 - ty0 + 1)
    keys = np.asarray(keys, dtype=np.int64)
    pids = np.asarray(pids, dtype=np.int64)
    order = np.lexsort((pids, keys))  # primary key: tile, secondary: particle id
    keys, pids = keys[order], pids[order]
    n_tiles = ntx * nty
    tile_start = np.searchsorted(keys, np.arange(n_tiles + 1), side="left")
    emit_start = np.concatenate([[0], np.cumsum(counts)])
    return {
        "keys": keys.astype(np.int32),
        "pids": pids.astype(np.int32),
        "tile_start": tile_start.astype(np.int32),
        "counts": counts.astype(np.int32),
        "emit_start": emit_start.astype(np.int64),
        "n_tiles": n_tiles,
    }
