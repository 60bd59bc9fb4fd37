"""Oracle imaging chain -- TEST INFRASTRUCTURE ONLY.

Plain FP64 statement of what the renderer computes from an OPD canvas:

  exit wave      U = A exp(i 2 pi / lambda * OPD)                 (Sec. III.B, Eq. 2)
                 A = 1 for a phase object; with absorption A = exp(-tau), tau the
                 absorbance canvas (Eq. 4's Beer-Lambert factor, with its Fresnel
                 transmittance taken as 1 and no caustic term: see the readings)
  spectrum       Ut[ky,kx] = sum_ij U[i,j] exp(-2 pi i (ky i/H + kx j/W))
  pupil          P(f) = circ(|f| <= NA/lambda) exp(i dz sqrt(k0^2 - (2 pi |f|)^2)),
                 k0 = 2 pi n_m / lambda                              (Eq. 3)
  brightfield    E = IDFT(Ut P), I = |E|^2                           (Eq. 4 text: I = |U * h_obj|^2)
  DIC            E = IDFT(Ut P (e^{i th} e^{+2 pi i f.ds} - e^{-i th} e^{-2 pi i f.ds})),
                 i.e. the pupil-filtered field sheared by +-ds and interfered at bias th
                 (Eq. 5 without its trailing incoherent blur, see the readings)
  oblique        E = IDFT(Ut P(f + f_t)): a tilted plane-wave illumination shifts the
                 spectrum against the pupil (the directional frequency-domain phase shift
                 of Sec. III.B, oblique modality)
  DIC, Eq. 5     the literal form: D = U(r + ds) e^{i th} - U(r - ds) e^{-i th} at full
  literal        resolution (D~ = Ut S, S the shear factor above without the pupil), then
                 I = |D|^2 * |h_obj|^2 with h_obj = IDFT(P) and the intensity PSF scaled to
                 unit sum (a uniform |D|^2 is reproduced): I = IDFT(DFT(|D|^2) OTF)
  noise          see ``noise.py`` (Sec. III.C, last paragraph)

Frequencies follow numpy's fftfreq order, f = k / (N dx) cycles per micrometre.
numpy's FFT serves as the DFT step; ``dft2_direct`` is the literal sum it stands for.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

BRIGHTFIELD, DIC, OBLIQUE, DIC_INCOHERENT = 0, 1, 2, 3


@dataclass
class Optics:
    """Static optics of a frame (all lengths in micrometres)."""
    mode: int = BRIGHTFIELD
    wavelength_um: float = 0.55
    na: float = 0.4
    n_medium: float = 1.33
    pixel_um: float = 0.1
    shear_angle_rad: float = 0.0
    tilt_fx: float = 0.0
    tilt_fy: float = 0.0
    photons_mean: float = 0.0
    seed: int = 0


def freqs(H: int, W: int, dx: float):
    """Signed spatial frequencies (cycles/um) of the DFT bins, fftfreq order."""
    return np.fft.fftfreq(H, d=dx), np.fft.fftfreq(W, d=dx)


def pupil_mask(H: int, W: int, optics: Optics, shifted: bool = True) -> np.ndarray:
    """Closed disc |f + f_t| <= NA/lambda on the DFT grid (a tie counts as inside)."""
    fy, fx = freqs(H, W, optics.pixel_um)
    tx = optics.tilt_fx if (shifted and optics.mode == OBLIQUE) else 0.0
    ty = optics.tilt_fy if (shifted and optics.mode == OBLIQUE) else 0.0
    gx = fx[None, :] + tx
    gy = fy[:, None] + ty
    r = optics.na / optics.wavelength_um
    return (gx * gx + gy * gy) <= r * r


def pupil(H: int, W: int, optics: Optics, defocus_um: float, tilt: bool = True) -> np.ndarray:
    """P(f [+ f_t]) of Eq. 3 on the DFT grid, with k0 = 2 pi n_m / lambda.

    The phase exp(i dz kz) is evaluated only inside the disc; kz is the axial
    angular wavenumber 2 pi sqrt((n_m/lambda)^2 - |f|^2).
    """
    fy, fx = freqs(H, W, optics.pixel_um)
    tx = optics.tilt_fx if (tilt and optics.mode == OBLIQUE) else 0.0
    ty = optics.tilt_fy if (tilt and optics.mode == OBLIQUE) else 0.0
    gx = fx[None, :] + tx
    gy = fy[:, None] + ty
    f2 = gx * gx + gy * gy
    r = optics.na / optics.wavelength_um
    inside = f2 <= r * r
    kn = optics.n_medium / optics.wavelength_um
    kz = np.zeros_like(f2)
    kz[inside] = 2.0 * np.pi * np.sqrt(kn * kn - f2[inside])
    P = np.zeros(f2.shape, dtype=np.complex128)
    P[inside] = np.exp(1j * defocus_um * kz[inside])
    return P


def transfer(H: int, W: int, optics: Optics, defocus_um: float, shear_px: float,
             bias_rad: float) -> np.ndarray:
    """Coherent transfer function H(f) of the modality (BF, DIC or oblique)."""
    P = pupil(H, W, optics, defocus_um)
    if optics.mode == BRIGHTFIELD or optics.mode == OBLIQUE:
        return P
    if optics.mode == DIC:
        return P * shear_factor(H, W, optics, shear_px, bias_rad)
    raise ValueError("unknown mode %r" % optics.mode)


def shear_factor(H: int, W: int, optics: Optics, shear_px: float, bias_rad: float) -> np.ndarray:
    """S(f) = e^{i th} e^{+2 pi i f.ds} - e^{-i th} e^{-2 pi i f.ds} on the whole DFT grid:
    the spectrum of U(r + ds) e^{i th} - U(r - ds) e^{-i th} is DFT(U) S (shift theorem),
    ds = (shear_px / 2) dx (cos psi, sin psi), total shear 2 |ds| (Eq. 5)."""
    fy, fx = freqs(H, W, optics.pixel_um)
    half = 0.5 * shear_px * optics.pixel_um          # |ds| in micrometres, total shear 2|ds|
    dsx = half * np.cos(optics.shear_angle_rad)
    dsy = half * np.sin(optics.shear_angle_rad)
    ramp = 2.0 * np.pi * (fx[None, :] * dsx + fy[:, None] * dsy)
    return np.exp(1j * bias_rad) * np.exp(1j * ramp) - np.exp(-1j * bias_rad) * np.exp(-1j * ramp)


def incoherent_otf(H: int, W: int, optics: Optics, defocus_um: float) -> np.ndarray:
    """DFT of the intensity PSF |h_obj|^2, h_obj = IDFT(P) (Eq. 3's pupil, no tilt),
    with the PSF scaled to unit sum, so the OTF is 1 at f = 0."""
    h = np.fft.ifft2(pupil(H, W, optics, defocus_um, tilt=False))
    psf = h.real * h.real + h.imag * h.imag
    return np.fft.fft2(psf / psf.sum())


def intensity_dic_incoherent(opd: np.ndarray, optics: Optics, defocus_um: float, shear_px: float,
                             bias_rad: float, tau=None) -> np.ndarray:
    """Eq. 5 as written: I = |U(r + ds) e^{i th} - U(r - ds) e^{-i th}|^2 * |h_obj|^2."""
    H, W = opd.shape
    U = exit_wave(opd, optics, tau)
    D = np.fft.ifft2(np.fft.fft2(U) * shear_factor(H, W, optics, shear_px, bias_rad))
    D2 = D.real * D.real + D.imag * D.imag
    return np.fft.ifft2(np.fft.fft2(D2) * incoherent_otf(H, W, optics, defocus_um)).real


def exit_wave(opd: np.ndarray, optics: Optics, tau=None) -> np.ndarray:
    """U = A exp(i 2 pi / lambda * OPD) (Eq. 2, OPD in micrometres), A = 1 or,
    given the absorbance canvas tau, A = exp(-tau) (Eq. 4)."""
    U = np.exp(1j * (2.0 * np.pi / optics.wavelength_um) * np.asarray(opd, dtype=np.float64))
    if tau is not None:
        U = U * np.exp(-np.asarray(tau, dtype=np.float64))
    return U


def field(opd: np.ndarray, optics: Optics, defocus_um: float, shear_px: float = 0.0,
          bias_rad: float = 0.0, dft=None, idft=None, tau=None) -> np.ndarray:
    """Image-plane field E = IDFT(DFT(U) * H); ``dft``/``idft`` default to numpy's FFT."""
    dft = dft or np.fft.fft2
    idft = idft or np.fft.ifft2
    H, W = opd.shape
    U = exit_wave(opd, optics, tau)
    return idft(dft(U) * transfer(H, W, optics, defocus_um, shear_px, bias_rad))


def intensity(opd: np.ndarray, optics: Optics, defocus_um: float, shear_px: float = 0.0,
              bias_rad: float = 0.0, dft=None, idft=None, tau=None) -> np.ndarray:
    """Noiseless image: I = |E|^2 (coherent modes) or Eq. 5's literal DIC."""
    if optics.mode == DIC_INCOHERENT:
        return intensity_dic_incoherent(np.asarray(opd, dtype=np.float64), optics, defocus_um, shear_px,
                                        bias_rad, tau)
    E = field(opd, optics, defocus_um, shear_px, bias_rad, dft, idft, tau)
    return E.real * E.real + E.imag * E.imag


def dft2_direct(x: np.ndarray, inverse: bool = False) -> np.ndarray:
    """The 2-D DFT by its defining double sum, every output from every input.

    Forward: X[ky,kx] = sum_{i,j} x[i,j] exp(-2 pi i (ky i / H + kx j / W));
    inverse: the conjugate kernel and a 1/(H W) factor.  O((HW)^2): small canvases only.
    """
    H, W = x.shape
    i = np.arange(H)
    j = np.arange(W)
    sgn = 1.0 if inverse else -1.0
    # kernel[(ky,kx),(i,j)] = exp(sgn 2 pi i (ky i/H + kx j/W)); phases reduced mod the length first
    ph_y = np.outer(i, i) % H / H
    ph_x = np.outer(j, j) % W / W
    phase = ph_y[:, None, :, None] + ph_x[None, :, None, :]
    kern = np.exp(sgn * 2j * np.pi * phase).reshape(H * W, H * W)
    out = (kern @ x.reshape(H * W)).reshape(H, W)
    return out / (H * W) if inverse else out
