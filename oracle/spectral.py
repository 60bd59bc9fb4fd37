"""Oracle of the spectral loss of Eq. 8 -- TEST INFRASTRUCTURE ONLY.

Eq. 8 compares the log amplitude spectra of a rendered image I and a target T,
the squared norm of log|F(I)| - log|F(T)|, F the 2-D DFT.  Readings used here:
the norm is taken as the mean over the H x W DFT bins (so the loss does not
grow with the canvas), F is numpy's unnormalised fft2, and eps > 0 is added
inside both logarithms (the logarithm of an empty bin is undefined):

    A(k) = log(|F(I)(k)| + eps) - log(|F(T)(k)| + eps),   L = (1/HW) sum_k A(k)^2.

Only amplitudes enter, so L ignores where in the frame the particles sit (a
circular shift of I leaves |F(I)| unchanged): the loss of targets that cannot
be aligned pixel by pixel.

Gradient (I real): d|F| = Re(conj(F) dF) / |F| and dF = DFT(dI), so
    dL/dI = Re(DFT(g)),   g(k) = (2/HW) A(k) conj(F(k)) / (|F(k)| (|F(k)| + eps)),
with g = 0 on bins where F = 0.
"""
from __future__ import annotations

import numpy as np


def log_amplitude(x: np.ndarray, eps: float, dft=None) -> np.ndarray:
    """log(|F(x)| + eps) on every DFT bin, FP64."""
    dft = dft or np.fft.fft2
    return np.log(np.abs(dft(np.asarray(x, dtype=np.float64))) + eps)


def loss(I: np.ndarray, T: np.ndarray, eps: float, dft=None) -> float:
    A = log_amplitude(I, eps, dft) - log_amplitude(T, eps, dft)
    return float(np.mean(A * A))


def grad(I: np.ndarray, T: np.ndarray, eps: float) -> np.ndarray:
    """dL/dI, FP64, [H][W]."""
    I = np.asarray(I, dtype=np.float64)
    F = np.fft.fft2(I)
    m = np.abs(F)
    A = np.log(m + eps) - log_amplitude(T, eps)
    g = np.zeros_like(F)
    nz = m > 0
    g[nz] = (2.0 / I.size) * A[nz] * np.conj(F[nz]) / (m[nz] * (m[nz] + eps))
    return np.fft.fft2(g).real
