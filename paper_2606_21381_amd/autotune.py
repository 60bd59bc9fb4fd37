"""Autotuner front end: picks the tile shape and FFT radix plan per canvas size.

The timing loop is native (``osog_autotune`` times every candidate plan with HIP
events and records the fastest in the context); this module feeds it a
representative frame per canvas size and keeps the choices in a JSON cache so a
later process can reuse them without timing again.
"""
from __future__ import annotations

import ctypes
import json
import os
from typing import Dict, Optional

import torch

from . import _lib
from .render import _check_globals, _check_soa, _ptr, _stream, context, soa_rows, workspace_size


def tune_frame(soa: torch.Tensor, H: int, W: int, optics, globals4: torch.Tensor, reps: int = 5,
               device=None) -> dict:
    """Time every plan on this frame; the context adopts the fastest for H x W."""
    device = soa.device if device is None else torch.device(device)
    n, ld = _check_soa(soa, soa_rows(optics))
    _check_globals(globals4, device)
    out = torch.empty((H, W), dtype=torch.float32, device=device)
    ws = torch.empty(workspace_size(H, W, n, int(optics.mode) == 3, device=device), dtype=torch.uint8,
                     device=device)
    th, tw, rad = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    ms = ctypes.c_float()
    o = _lib.make_optics(optics)
    _lib.check(_lib.load().osog_autotune(context(device), _stream(device), H, W, _ptr(soa) if n else None, n, ld,
                                          ctypes.byref(o), _ptr(globals4), _ptr(out), _ptr(ws), ws.numel(), reps,
                                          ctypes.byref(th), ctypes.byref(tw), ctypes.byref(rad), ctypes.byref(ms)),
               "osog_autotune")
    return {"tile_h": th.value, "tile_w": tw.value, "fft_radix": rad.value, "ms": ms.value}


def apply(choices: Dict[str, dict], device=None):
    """Install cached choices ({"HxW": {"tile_h", "tile_w", "fft_radix"}}) in the context."""
    lib = _lib.load()
    ctx = context(device)
    for key, c in choices.items():
        H, W = (int(v) for v in key.split("x"))
        _lib.check(lib.osog_set_size_tiling(ctx, H, W, int(c["tile_h"]), int(c["tile_w"])), "osog_set_size_tiling")
        _lib.check(lib.osog_set_size_radix(ctx, H, W, int(c["fft_radix"])), "osog_set_size_radix")


def tune_sizes(frames_by_size: dict, cache: Optional[str] = None, reps: int = 5, device=None) -> Dict[str, dict]:
    """frames_by_size: {(H, W): (soa, optics, globals4)}.  Uses and updates a JSON cache."""
    choices: Dict[str, dict] = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            choices = json.load(f)
    todo = {k: v for k, v in frames_by_size.items() if "%dx%d" % k not in choices}
    for (H, W), (soa, optics, g) in todo.items():
        choices["%dx%d" % (H, W)] = tune_frame(soa, H, W, optics, g, reps, device)
    apply(choices, device)
    if cache and todo:
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(choices, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return choices
