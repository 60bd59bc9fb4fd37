"""Pins of the oracle's Beer-Lambert absorption (Eq. 4's exponential factor).

Each pin is a fact the paper and the mathematics fix, not a retyping of the
oracle's formula:
  * a canvas-filling absorber transmits exp(-2 dmu h) of the light at every
    pixel, in every modality's closed form (the DC bin passes every pupil);
  * overlapping absorbers compose multiplicatively (exponents add);
  * with a pupil covering the whole DFT grid and no defocus the imaging chain is
    the identity, so I = |U|^2 = exp(-2 tau) pixel by pixel, for any canvas;
  * defocus is unitary on that grid: sum I = sum exp(-2 tau) (Parseval);
  * dmu = 0 reduces to the phase-only chain exactly;
  * a pixel deep inside a prism has absorbance dmu h, one outside has 0.
"""
import math

import numpy as np

from oracle import optics as O
from oracle import raster as R


def table(rows):
    """[9][n] FP64 table from per-particle tuples (cx, cy, ang, a, b, h, dn, shape, dmu)."""
    return np.array(rows, dtype=np.float64).T.copy()


def test_canvas_filling_absorber_closed_forms():
    H = W = 64
    h, dmu = 1.5, 0.3
    soa = table([(32.0, 32.0, 0.0, 1000.0, 1000.0, h, 0.0, 0.0, dmu)])
    tau = R.absorbance(soa, H, W)
    assert np.array_equal(tau, np.full((H, W), dmu * h))
    opd = R.opd(soa, H, W)
    assert np.array_equal(opd, np.zeros((H, W)))
    t = math.exp(-2.0 * dmu * h)
    # brightfield, any defocus: |P(0)| = 1
    for dz in (0.0, 1.3):
        I = O.intensity(opd, O.Optics(mode=O.BRIGHTFIELD, na=0.4), dz, tau=tau)
        assert np.max(np.abs(I - t)) < 1e-13
    # DIC: H(0) = P(0) (e^{i th} - e^{-i th}) = 2 i sin(th) P(0)
    th = 1.1
    I = O.intensity(opd, O.Optics(mode=O.DIC, na=0.5, shear_angle_rad=0.7), -0.5, 1.0, th, tau=tau)
    assert np.max(np.abs(I - 4.0 * math.sin(th) ** 2 * t)) < 1e-13


def test_overlapping_absorbers_multiply():
    H = W = 32
    soa = table([(16.0, 16.0, 0.0, 500.0, 500.0, 1.0, 0.0, 0.0, 0.2),
                 (16.0, 16.0, 0.3, 500.0, 500.0, 2.0, 0.0, 0.0, 0.15)])
    tau = R.absorbance(soa, H, W)
    I = O.intensity(np.zeros((H, W)), O.Optics(mode=O.BRIGHTFIELD, na=0.4), 0.0, tau=tau)
    assert np.max(np.abs(I - math.exp(-2 * 0.2 * 1.0) * math.exp(-2 * 0.15 * 2.0))) < 1e-13


def wide_open():
    # NA / lambda = 8.2 cycles/um exceeds the grid's corner frequency sqrt(2) * 5 at dx = 0.1 um
    return O.Optics(mode=O.BRIGHTFIELD, wavelength_um=0.55, na=4.5, n_medium=5.0, pixel_um=0.1)


def random_absorbing_table(rng, n, H, W):
    rows = []
    for k in range(n):
        shape = float(k % 2)
        a = rng.uniform(3, 9)
        b = a if shape == 0.0 else rng.uniform(2, 8)
        rows.append((rng.uniform(0, W), rng.uniform(0, H), rng.uniform(0, math.pi), a, b,
                     rng.uniform(0.5, 2.5), rng.uniform(0.01, 0.05), shape, rng.uniform(0.0, 0.4)))
    return table(rows)


def test_full_pupil_in_focus_is_pointwise_beer_lambert():
    H = W = 64
    soa = random_absorbing_table(np.random.default_rng(3), 12, H, W)
    tau = R.absorbance(soa, H, W)
    assert tau.max() > 0.2
    I = O.intensity(R.opd(soa, H, W), wide_open(), 0.0, tau=tau)
    assert np.max(np.abs(I - np.exp(-2.0 * tau))) < 1e-12


def test_defocus_conserves_transmitted_power():
    H = W = 64
    soa = random_absorbing_table(np.random.default_rng(4), 12, H, W)
    tau = R.absorbance(soa, H, W)
    I = O.intensity(R.opd(soa, H, W), wide_open(), 2.0, tau=tau)
    assert abs(I.sum() - np.exp(-2.0 * tau).sum()) < 1e-9 * I.sum()
    # and the pointwise image does change under defocus (the check is not vacuous)
    assert np.max(np.abs(I - np.exp(-2.0 * tau))) > 1e-3


def test_zero_attenuation_is_the_phase_only_chain():
    H = W = 48
    soa = random_absorbing_table(np.random.default_rng(5), 10, H, W)
    soa[8] = 0.0
    opd = R.opd(soa, H, W)
    tau = R.absorbance(soa, H, W)
    assert np.array_equal(tau, np.zeros((H, W)))
    opt = O.Optics(mode=O.DIC, na=0.5, shear_angle_rad=math.pi / 4)
    assert np.array_equal(O.intensity(opd, opt, 0.4, 1.0, 1.2, tau=tau), O.intensity(opd, opt, 0.4, 1.0, 1.2))


def test_absorbance_inside_and_outside_a_prism():
    H = W = 64
    h, dmu, dn = 2.0, 0.25, 0.03
    soa = table([(32.3, 31.7, 0.4, 10.0, 7.0, h, dn, 0.0, dmu)])
    tau = R.absorbance(soa, H, W)
    opd = R.opd(soa, H, W)
    assert tau[32, 32] == dmu * h          # centre pixel: fully covered
    assert tau[0, 0] == 0.0 and tau[63, 63] == 0.0
    # the absorbance is the OPD's thickness integral reweighted: tau / dmu == opd / dn
    assert np.max(np.abs(tau / dmu - opd / dn)) < 1e-12
