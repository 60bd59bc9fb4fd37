"""FP64 CPU oracle of the OSOG forward model -- TEST INFRASTRUCTURE ONLY.

A plain, slow, single-threaded statement of what the renderer computes, written
from the paper (arXiv 2606.21381, Sec. III) and sharing no code with the GPU
library.  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import it; the product path never does.

  binning.py  sorted (tile, particle) pairs (FP32-exact box recipe)
  raster.py   OPD canvas: exact-area prisms, centre-sampled ellipsoids (C, FP64)
  optics.py   exit wave (with absorption), DFT, pupil/defocus, BF / DIC / oblique, |E|^2,
              Eq. 5's literal (incoherent) DIC, direct DFT
  noise.py    Philox4x32-10 and Poisson shot noise
  grad.py     central finite-difference gradients, solver loss
  spectral.py the spectral (log-amplitude) loss of Eq. 8 and its gradient
  cnn.py      the learned initializer's network in float64 PyTorch (autograd gradients)
"""
from __future__ import annotations

import numpy as np

from . import binning, grad, noise, optics, raster, spectral
from .optics import BRIGHTFIELD, DIC, DIC_INCOHERENT, OBLIQUE, Optics


def render(soa, H: int, W: int, opt: Optics, globals4, with_noise: bool = False, frame: int = 0):
    """OPD (um) and intensity of one frame, FP64 throughout.

    ``globals4`` = (defocus_um, shear_px, bias_rad, unused); FP32 values are widened.
    """
    g = np.asarray(globals4, dtype=np.float32).astype(np.float64)
    opd = raster.opd(np.asarray(soa, dtype=np.float32), H, W)
    I = optics.intensity(opd, opt, g[0], g[1], g[2])
    if with_noise and opt.photons_mean > 0:
        I = noise.add_noise(I, opt.photons_mean, opt.seed, frame)
    return opd, I


__all__ = ["binning", "grad", "noise", "optics", "raster", "spectral", "render", "Optics",
           "BRIGHTFIELD", "DIC", "DIC_INCOHERENT", "OBLIQUE"]
