"""Pins of the oracle's imaging chain: direct DFT, closed forms, identities."""
import math

import numpy as np

from oracle import optics as O


def rand_opd(rng, H, W, scale=0.3):
    return rng.uniform(0, scale, (H, W))


def test_fft_matches_direct_dft_32x32():
    rng = np.random.default_rng(0)
    x = rng.normal(size=(32, 32)) + 1j * rng.normal(size=(32, 32))
    d = O.dft2_direct(x)
    assert np.max(np.abs(np.fft.fft2(x) - d)) <= 1e-12 * np.max(np.abs(d))
    xi = O.dft2_direct(d, inverse=True)
    assert np.max(np.abs(xi - x)) < 1e-12


def test_image_chain_with_direct_dft_32x32():
    rng = np.random.default_rng(1)
    opd = rand_opd(rng, 32, 32)
    for mode, g in [(O.BRIGHTFIELD, (0.7, 0, 0)), (O.DIC, (-0.4, 1.0, math.pi / 2)),
                    (O.OBLIQUE, (0.3, 0, 0))]:
        opt = O.Optics(mode=mode, na=0.5, shear_angle_rad=math.pi / 4, tilt_fx=0.27)
        a = O.intensity(opd, opt, *g)
        b = O.intensity(opd, opt, *g, dft=O.dft2_direct, idft=lambda z: O.dft2_direct(z, True))
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)


def test_in_focus_full_pupil_gives_unit_intensity():
    # dx = 1 um, lambda 0.55, NA 0.4: NA/lambda = 0.727 >= sqrt(2)/2 -> every bin passes.
    rng = np.random.default_rng(2)
    opt = O.Optics(mode=O.BRIGHTFIELD, na=0.4, pixel_um=1.0)
    assert O.pupil_mask(64, 64, opt).all()
    I = O.intensity(rand_opd(rng, 64, 64, 2.0), opt, 0.0)
    assert np.max(np.abs(I - 1)) < 1e-12


def test_empty_canvas_closed_forms():
    z = np.zeros((64, 64))
    bf = O.Optics(mode=O.BRIGHTFIELD, na=0.5)
    assert np.max(np.abs(O.intensity(z, bf, 1.3) - 1)) < 1e-12
    for th in (math.pi / 2, 0.3, 1.1):
        dic = O.Optics(mode=O.DIC, na=0.5, shear_angle_rad=math.pi / 4)
        assert np.max(np.abs(O.intensity(z, dic, -0.8, 1.0, th) - 4 * math.sin(th) ** 2)) < 1e-12
    ob_in = O.Optics(mode=O.OBLIQUE, na=0.5, tilt_fx=0.3 * 0.5 / 0.55)
    assert np.max(np.abs(O.intensity(z, ob_in, 0.5) - 1)) < 1e-12
    ob_out = O.Optics(mode=O.OBLIQUE, na=0.5, tilt_fx=1.2 * 0.5 / 0.55)
    assert np.max(np.abs(O.intensity(z, ob_out, 0.5))) < 1e-24


def test_dic_full_pupil_integer_shear_closed_form():
    # In focus, full pupil, total shear 2 px along x (ds = 1 px):
    # I = 2 - 2 cos(phi(r + ds) - phi(r - ds) + 2 theta), periodic indexing.
    rng = np.random.default_rng(3)
    opd = rand_opd(rng, 32, 64, 1.0)
    theta = 0.3
    opt = O.Optics(mode=O.DIC, na=0.4, pixel_um=1.0, shear_angle_rad=0.0)
    I = O.intensity(opd, opt, 0.0, 2.0, theta)
    phi = 2 * math.pi / opt.wavelength_um * opd
    d = np.roll(phi, -1, axis=1) - np.roll(phi, 1, axis=1)
    assert np.max(np.abs(I - (2 - 2 * np.cos(d + 2 * theta)))) < 1e-12


def test_dic_shear_is_a_fourier_shift():
    # The DIC transfer divided by the pupil has the two shift kernels e^{+-2 pi i f.ds};
    # with an integer ds along y the '+' kernel shifts the field by -ds (np.roll).
    rng = np.random.default_rng(4)
    E = rng.normal(size=(64, 32)) + 1j * rng.normal(size=(64, 32))
    opt = O.Optics(mode=O.DIC, na=0.4, pixel_um=1.0, shear_angle_rad=math.pi / 2)
    Ht = O.transfer(64, 32, opt, 0.0, 6.0, math.pi / 2)     # ds = 3 px along +y
    P = O.pupil(64, 32, opt, 0.0)
    # bias pi/2: H/P = i e^{+r} + i e^{-r}; with bias 0 it is e^{+r} - e^{-r}
    H0 = O.transfer(64, 32, opt, 0.0, 6.0, 0.0)
    plus = 0.5 * (Ht / (1j * P) + H0 / P)
    shifted = np.fft.ifft2(np.fft.fft2(E) * plus)
    assert np.max(np.abs(shifted - np.roll(E, -3, axis=0))) < 1e-12


def test_oblique_integer_tilt_is_pupil_roll():
    opt_bf = O.Optics(mode=O.BRIGHTFIELD, na=0.5)
    t = 7
    opt_ob = O.Optics(mode=O.OBLIQUE, na=0.5, tilt_fx=t / (128 * 0.1))
    P = O.pupil(128, 128, opt_bf, 0.9)
    Ht = O.transfer(128, 128, opt_ob, 0.9, 0, 0)
    assert np.max(np.abs(Ht - np.roll(P, -t, axis=1))) < 1e-12


def test_weak_phase_defocus_transfer():
    # U ~ 1 + i phi:  I ~ 1 - 2 IDFT[ DFT(phi) circ sin(dz (kz - k0)) ] + O(phi^2).
    # Fixes the defocus sign and k0 = 2 pi n_m / lambda.
    rng = np.random.default_rng(5)
    H = W = 64
    opt = O.Optics(mode=O.BRIGHTFIELD, na=0.4, pixel_um=0.1)
    phi = rng.normal(scale=1e-3, size=(H, W))
    opd = phi * opt.wavelength_um / (2 * math.pi)
    dz = 1.0
    I = O.intensity(opd, opt, dz)
    fy, fx = O.freqs(H, W, opt.pixel_um)
    f2 = fx[None, :] ** 2 + fy[:, None] ** 2
    circ = f2 <= (opt.na / opt.wavelength_um) ** 2
    kn = opt.n_medium / opt.wavelength_um
    kz = 2 * math.pi * np.sqrt(np.maximum(kn * kn - f2, 0))
    k0 = 2 * math.pi * kn
    lin = 1 - 2 * np.real(np.fft.ifft2(np.fft.fft2(phi) * circ * np.sin(dz * (kz - k0))))
    contrast = np.max(np.abs(lin - 1))
    assert contrast > 1e-4
    assert np.max(np.abs(I - lin)) < 0.02 * contrast
    # the opposite sign convention would flip the contrast
    assert np.max(np.abs(O.intensity(opd, opt, -dz) - lin)) > 0.5 * contrast


def test_parseval():
    rng = np.random.default_rng(6)
    opd = rand_opd(rng, 64, 128, 0.5)
    opt = O.Optics(mode=O.DIC, na=0.5, shear_angle_rad=math.pi / 4)
    g = (0.8, 1.0, math.pi / 2)
    I = O.intensity(opd, opt, *g)
    G = np.fft.fft2(O.exit_wave(opd, opt)) * O.transfer(64, 128, opt, *g)
    assert abs(I.sum() - np.sum(np.abs(G) ** 2) / (64 * 128)) < 1e-12 * I.sum()


def test_pupil_support_is_closed_disc():
    opt = O.Optics(mode=O.BRIGHTFIELD, na=0.5, pixel_um=0.1)
    m = O.pupil_mask(2048, 2048, opt)
    # radius NA/lambda * W * dx = 186.18 bins: 373 in-band kx columns
    cols = np.nonzero(m.any(axis=0))[0]
    assert cols.size == 373
    assert m[0, 186] and not m[0, 187]
