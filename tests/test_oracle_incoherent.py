"""Pins of the oracle's literal Eq. 5 DIC (sheared interference, then the
incoherent blur by |h_obj|^2):
  * with a pupil covering the whole DFT grid and no defocus the blur is the
    identity, and a shear of one pixel each way is a circular shift: the image is
    |U(x+1) e^{i th} - U(x-1) e^{-i th}|^2, pixel by pixel, along x and along y;
  * an empty field images to 4 sin^2(th) (the unit-sum PSF keeps a uniform |D|^2);
  * the OTF is the pupil's normalised autocorrelation (Wiener-Khinchin), checked
    by brute force on a small grid, with and without defocus;
  * the blur keeps the mean: mean(I) = mean(|D|^2).
"""
import math

import numpy as np

from oracle import optics as O
from oracle import raster as R


def wide_open(psi):
    return O.Optics(mode=O.DIC_INCOHERENT, wavelength_um=0.55, na=4.5, n_medium=5.0, pixel_um=0.1,
                    shear_angle_rad=psi)


def test_full_pupil_unit_shear_is_a_circular_difference():
    rng = np.random.default_rng(0)
    H = W = 32
    opd = rng.uniform(0, 0.4, (H, W))
    tau = rng.uniform(0, 0.5, (H, W))
    U = np.exp(-tau) * np.exp(1j * 2 * np.pi / 0.55 * opd)
    th = 0.9
    for psi, axis in ((0.0, 1), (math.pi / 2, 0)):
        I = O.intensity(opd, wide_open(psi), 0.0, 2.0, th, tau=tau)   # total shear 2 px: ds = 1 px
        D = np.roll(U, -1, axis=axis) * np.exp(1j * th) - np.roll(U, 1, axis=axis) * np.exp(-1j * th)
        assert np.max(np.abs(I - np.abs(D) ** 2)) < 1e-11


def test_empty_field_images_to_four_sin_squared():
    H = W = 64
    th = 1.2
    opt = O.Optics(mode=O.DIC_INCOHERENT, na=0.5, shear_angle_rad=math.pi / 4)
    for dz in (0.0, 1.7):
        I = O.intensity(np.zeros((H, W)), opt, dz, 1.0, th)
        assert np.max(np.abs(I - 4 * math.sin(th) ** 2)) < 1e-12


def autocorrelation(P):
    """A(k) = sum_f P(f) conj(P(f - k)), indices mod the grid, by brute force."""
    H, W = P.shape
    A = np.zeros((H, W), dtype=np.complex128)
    for ky in range(H):
        for kx in range(W):
            A[ky, kx] = np.sum(P * np.conj(np.roll(np.roll(P, ky, axis=0), kx, axis=1)))
    return A


def test_otf_is_the_normalised_pupil_autocorrelation():
    H = W = 16
    opt = O.Optics(mode=O.DIC_INCOHERENT, na=1.0, n_medium=1.33, wavelength_um=0.55, pixel_um=0.1)
    for dz in (0.0, 0.8):
        P = O.pupil(H, W, opt, dz, tilt=False)
        A = autocorrelation(P)
        otf = O.incoherent_otf(H, W, opt, dz)
        assert abs(otf[0, 0] - 1.0) < 1e-14
        assert np.max(np.abs(otf - A / A[0, 0])) < 1e-13


def test_blur_keeps_the_mean():
    rng = np.random.default_rng(2)
    H = W = 64
    soa = np.array([[20.0, 40.0], [30.0, 25.0], [0.3, 1.1], [6.0, 5.0], [6.0, 3.0], [1.5, 1.0],
                    [0.03, 0.04], [0.0, 1.0]])
    opd = R.opd(soa, H, W)
    opt = O.Optics(mode=O.DIC_INCOHERENT, na=0.5, shear_angle_rad=0.6)
    I = O.intensity(opd, opt, 0.9, 1.0, 1.4)
    U = O.exit_wave(opd, opt)
    D = np.fft.ifft2(np.fft.fft2(U) * O.shear_factor(H, W, opt, 1.0, 1.4))
    assert abs(I.mean() - np.mean(np.abs(D) ** 2)) < 1e-12
    # and the blur is not the identity at this NA (the check is not vacuous)
    assert np.max(np.abs(I - np.abs(D) ** 2)) > 1e-2
