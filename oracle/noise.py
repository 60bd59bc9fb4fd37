"""Oracle sensor shot noise -- TEST INFRASTRUCTURE ONLY.

Paper Sec. III.C (last paragraph) adds Poisson photon shot noise to the
composited image.  Reading used: the clean image is scaled to photon counts by
s = photons_mean / mean(I) (mean over the frame), counts ~ Poisson(s I) per
pixel, and the output is counts / s.

Random numbers come from a counter-based generator implemented here from its
published definition, Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), so the
GPU implementation and this one draw the same stream.  Key = (seed low 32, seed
high 32).  Pixels 2m and 2m+1 share the block at counter (m, frame, 0, 0):
words 0,1 belong to the even pixel, words 2,3 to the odd one; any further words
of pixel p come from its own blocks at counter (p, frame, round, 1), round =
1, 2, ...  uniform = ((x >> 9) + 0.5) * 2^-23 in FP32 (every value exact, never
0 or 1).
Gaussian read noise (optional): read_noise * z counts added to each count, z
from Box-Muller on the first two words of the block at counter (m, frame, 0, 2)
of pixels 2m and 2m+1 (read_normals).
Poisson variates: mean < 10 by inversion with sequential search on the pixel's
first word (at most 40 steps); mean >= 10 by Hoermann's transformed rejection
with squeeze "PTRS" (Insurance: Math. and Econ. 12, 1993), two uniforms per
attempt: the first attempt from the shared block, then two per own block, at
most 15 own blocks.  Its acceptance test compares
log(V inv_alpha / (a/us^2 + b)) with -mu + k log(mu) - log(k!), where log(k!)
is tabulated below k = 10 and taken from Stirling's series above.  The
decisions are taken in FP32, the precision of the GPU sampler.
"""
from __future__ import annotations

import math

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """One Philox4x32 block with 10 rounds on plain Python integers."""
    c0, c1, c2, c3 = (int(x) & MASK for x in ctr)
    k0, k1 = (int(x) & MASK for x in key)
    for r in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = (p0 >> 32) & MASK, p0 & MASK
        hi1, lo1 = (p1 >> 32) & MASK, p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return c0, c1, c2, c3


def philox4x32_10_np(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10 over uint32 arrays (the same rounds as above)."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    k0 = np.uint64(k0 & MASK)
    k1 = np.uint64(k1 & MASK)
    m = np.uint64(MASK)
    for r in range(10):
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if r < 9:
            k0 = (k0 + np.uint64(W0)) & m
            k1 = (k1 + np.uint64(W1)) & m
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def uniform_f32(x: int) -> np.float32:
    return np.float32(((int(x) >> 9) + 0.5) * 2.0 ** -23)


def _f(x) -> np.float32:
    return np.float32(x)


def log_factorial_f32(k: float) -> np.float32:
    """log(k!) in FP32: correctly rounded table below 10, Stirling's series
    (x - 1/2) ln x - x + ln(2 pi)/2 + 1/(12 x) - 1/(360 x^3), x = k + 1, above."""
    if k < 10:
        return _f(math.lgamma(int(k) + 1.0))
    x = _f(_f(k) + _f(1.0))
    t = _f(_f(_f(x - _f(0.5)) * _f(np.log(x))) - x)
    t = _f(t + _f(0.918938533))
    t = _f(t + _f(_f(1.0) / _f(_f(12.0) * x)))
    return _f(t - _f(_f(1.0) / _f(_f(_f(_f(360.0) * x) * x) * x)))


def _ptrs_attempt(wu, wv, mu, log_mu, a, b, inv_alpha, vr):
    """One PTRS attempt from two words: k >= 0 if accepted, -1 if rejected."""
    U = _f(uniform_f32(wu) - _f(0.5))
    V = uniform_f32(wv)
    us = _f(_f(0.5) - _f(abs(U)))
    kf = _f(np.floor(_f(_f(_f(_f(_f(_f(2.0) * a) / us) + b) * U) + _f(mu + _f(0.43)))))
    if us >= _f(0.07) and V <= vr:
        return int(kf)
    if kf < 0 or (us < _f(0.013) and V > us):
        return -1
    lhs = _f(np.log(_f(_f(V * inv_alpha) / _f(_f(a / _f(us * us)) + b))))
    rhs = _f(_f(-mu + _f(kf * log_mu)) - log_factorial_f32(float(kf)))
    return int(kf) if lhs <= rhs else -1


def poisson_one(mu: float, pixel: int, frame: int, seed: int) -> int:
    """One Poisson(mu) variate for one pixel (FP32 decisions, as on the GPU)."""
    mu = _f(mu)
    if not (mu > 0):
        return 0
    key = (seed & MASK, (seed >> 32) & MASK)
    shared = philox4x32_10((pixel >> 1, frame, 0, 0), key)
    w0, w1 = shared[2 * (pixel & 1)], shared[2 * (pixel & 1) + 1]
    if mu < _f(10.0):
        u = uniform_f32(w0)
        p = _f(np.exp(-mu))
        F = p
        k = 0
        while u > F and k < 40:
            k += 1
            p = _f(p * _f(mu / _f(k)))
            F = _f(F + p)
        return k
    smu = _f(np.sqrt(mu))
    log_mu = _f(np.log(mu))
    b = _f(_f(0.931) + _f(_f(2.53) * smu))
    a = _f(_f(-0.059) + _f(_f(0.02483) * b))
    inv_alpha = _f(_f(1.1239) + _f(_f(1.1328) / _f(b - _f(3.4))))
    vr = _f(_f(0.9277) - _f(_f(3.6224) / _f(b - _f(2.0))))
    k = _ptrs_attempt(w0, w1, mu, log_mu, a, b, inv_alpha, vr)
    if k >= 0:
        return k
    for rnd in range(1, 16):
        r = philox4x32_10((pixel, frame, rnd, 1), key)
        for t in range(2):
            k = _ptrs_attempt(r[2 * t], r[2 * t + 1], mu, log_mu, a, b, inv_alpha, vr)
            if k >= 0:
                return k
    return int(math.floor(float(mu)))


def read_normals(pair: int, frame: int, seed: int):
    """Two standard normal variates for pixels 2 pair and 2 pair + 1 (Box and Muller,
    Ann. Math. Statist. 29, 1958) from the first two words u1, u2 of the Philox block
    at counter (pair, frame, 0, 2): r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2).
    FP64 on the FP32 uniforms."""
    key = (seed & MASK, (seed >> 32) & MASK)
    w = philox4x32_10((pair, frame, 0, 2), key)
    u1, u2 = float(uniform_f32(w[0])), float(uniform_f32(w[1]))
    r = math.sqrt(-2.0 * math.log(u1))
    return r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2)


def add_noise(I: np.ndarray, photons_mean: float, seed: int, frame: int = 0,
              mean_I: float | None = None, read_noise: float = 0.0) -> np.ndarray:
    """(counts + read_noise z) / s with counts ~ Poisson(s I), s = photons_mean / mean(I),
    z standard normal (read_normals): the heteroscedastic sensor model of Sec. III.C,
    Poisson shot noise plus Gaussian read noise of read_noise counts.  Slow: small frames."""
    I = np.asarray(I, dtype=np.float64)
    m = float(I.mean()) if mean_I is None else float(mean_I)
    if not (photons_mean > 0) or not (m > 0):
        return I.copy()
    s = photons_mean / m
    flat = I.reshape(-1)
    out = np.empty_like(flat)
    for p in range(flat.shape[0]):
        k = float(poisson_one(s * flat[p], p, frame, seed))
        if read_noise > 0:
            k += read_noise * read_normals(p >> 1, frame, seed)[p & 1]
        out[p] = k / s
    return out.reshape(I.shape)
