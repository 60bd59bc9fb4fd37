"""Pins of the oracle's spectral loss (Eq. 8):
  * L(I, I) = 0, and with eps = 0 a contrast scale c gives exactly (log c)^2;
  * a circular shift of the image leaves the loss unchanged (amplitudes only);
  * the DFT step agrees with the direct DFT sum on a small image;
  * the gradient agrees with central differences of the loss (every pixel of a
    small image), and a wrong sign, a missing conjugate or a dropped factor 2
    would not.
"""
import numpy as np

from oracle import optics as O
from oracle import spectral as S


def img(seed, H=16, W=16):
    return np.random.default_rng(seed).uniform(0.5, 1.5, (H, W))


def test_zero_at_the_target_and_log_scale_law():
    I = img(0)
    assert S.loss(I, I, 1e-3) == 0.0
    for c in (0.5, 2.0, 3.7):
        assert abs(S.loss(c * I, I, 0.0) - np.log(c) ** 2) < 1e-12


def test_circular_shift_invariance():
    I, T = img(1, 32, 32), img(2, 32, 32)
    base = S.loss(I, T, 1e-2)
    for sy, sx in ((3, 0), (0, 5), (7, 11)):
        assert abs(S.loss(np.roll(I, (sy, sx), axis=(0, 1)), T, 1e-2) - base) < 1e-12 * max(base, 1.0)


def test_direct_dft_sum():
    I, T = img(3, 8, 8), img(4, 8, 8)
    a = S.loss(I, T, 1e-3)
    b = S.loss(I, T, 1e-3, dft=O.dft2_direct)
    assert abs(a - b) < 1e-12 * a


def test_gradient_against_central_differences():
    I, T = img(5, 8, 8), img(6, 8, 8)
    eps = 1e-2
    g = S.grad(I, T, eps)
    d = 1e-6
    fd = np.zeros_like(I)
    for i in range(8):
        for j in range(8):
            P, M = I.copy(), I.copy()
            P[i, j] += d
            M[i, j] -= d
            fd[i, j] = (S.loss(P, T, eps) - S.loss(M, T, eps)) / (2 * d)
    assert np.max(np.abs(g - fd)) < 1e-6 * np.max(np.abs(fd))
    # plausible mistakes fail the same comparison
    F = np.fft.fft2(I)
    m = np.abs(F)
    A = np.log(m + eps) - np.log(np.abs(np.fft.fft2(T)) + eps)
    no_conj = np.fft.fft2((2.0 / I.size) * A * F / (m * (m + eps))).real
    half = 0.5 * g
    for wrong in (no_conj, half, -g):
        assert np.max(np.abs(wrong - fd)) > 1e-3 * np.max(np.abs(fd))
