"""Oracle sensor shot noise -- TEST INFRASTRUCTURE ONLY.

Paper Sec. III.C (last paragraph) adds Poisson photon shot noise to the
composited image.  Reading used: the clean image is scaled to photon counts by
s = photons_mean / mean(I) (mean over the frame), counts ~ Poisson(s I) per
pixel, and the output is counts / s.

Random numbers come from a counter-based generator implemented here from its
published definition, Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), keyed
on (seed low 32, seed high 32).  Which words a pixel consumes is a reading (the
paper names no generator): pixels 2m and 2m+1 share the block at counter
(m, frame, 0, 0), words 0,1 for the even pixel and 2,3 for the odd one; any
further words of pixel p come from its own blocks at counter (p, frame, round, 1),
round = 1, 2, ...  A word x maps to the uniform ((x >> 9) + 1/2) 2^-23, a value
on a 23-bit grid that is never 0 or 1.

Gaussian read noise (optional): read_noise * z counts added to each count, z
from Box-Muller on the first two words of the block at counter (m, frame, 0, 2)
of pixels 2m and 2m+1 (read_normals).

Poisson variates, both methods exact samplers stated in FP64:
  * mean < 10: inversion -- the smallest k whose cumulative probability reaches
    the pixel's first uniform (sequential search, at most 40 steps);
  * mean >= 10: Hoermann's transformed rejection with squeeze, "PTRS"
    (W. Hoermann, Insurance: Mathematics and Economics 12, 39-45, 1993), as that
    paper states it: constants b, a, 1/alpha, v_r from sqrt(mu); per attempt
    U ~ U(-1/2, 1/2), V ~ U(0, 1), u_s = 1/2 - |U|,
    k = floor((2a/u_s + b) U + mu + 0.43); accept at once when u_s >= 0.07 and
    V <= v_r; reject when k < 0 or (u_s < 0.013 and V > u_s); otherwise accept
    when log(V / alpha / (a/u_s^2 + b)) <= -mu + k log mu - log k!, log k! from
    the log-gamma function.  The first attempt takes the pixel's two shared
    words, later attempts two words each from its own blocks (at most 15 blocks).
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
    """The uniform of one word; exact in FP32 (and hence in FP64)."""
    return np.float32(((int(x) >> 9) + 0.5) * 2.0 ** -23)


def uniform(x) -> np.ndarray:
    """The uniforms of an array of words, FP64 (the same values as uniform_f32)."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def ptrs_constants(mu):
    """Hoermann's PTRS constants for means mu >= 10: (b, a, 1/alpha, v_r)."""
    smu = np.sqrt(mu)
    b = 0.931 + 2.53 * smu
    a = -0.059 + 0.02483 * b
    inv_alpha = 1.1239 + 1.1328 / (b - 3.4)
    vr = 0.9277 - 3.6224 / (b - 2.0)
    return b, a, inv_alpha, vr


def _log_factorial(k):
    return np.array([math.lgamma(float(v) + 1.0) for v in np.ravel(k)], dtype=np.float64).reshape(np.shape(k))


def ptrs_attempt(U01, V, mu):
    """One PTRS attempt per element: k >= 0 where accepted, -1 where rejected.

    U01, V: uniforms in (0, 1); mu >= 10 (arrays of one shape).  FP64."""
    mu = np.asarray(mu, dtype=np.float64)
    b, a, inv_alpha, vr = ptrs_constants(mu)
    U = np.asarray(U01, dtype=np.float64) - 0.5
    V = np.asarray(V, dtype=np.float64)
    us = 0.5 - np.abs(U)
    k = np.floor((2.0 * a / us + b) * U + mu + 0.43)
    quick = (us >= 0.07) & (V <= vr)
    reject = (k < 0) | ((us < 0.013) & (V > us))
    out = np.where(quick, k, -1.0)
    t = ~quick & ~reject
    if np.any(t):
        lhs = np.log(V[t] * inv_alpha[t] / (a[t] / (us[t] * us[t]) + b[t]))
        rhs = -mu[t] + k[t] * np.log(mu[t]) - _log_factorial(k[t])
        out[t] = np.where(lhs <= rhs, k[t], -1.0)
    return out.astype(np.int64)


def poisson_inversion(mu, u):
    """Inversion for mu < 10: the smallest k with P(X <= k) >= u (at most 40)."""
    mu = np.asarray(mu, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    p = np.exp(-mu)
    F = p.copy()
    k = np.zeros(mu.shape, dtype=np.int64)
    live = u > F
    for step in range(1, 41):
        if not np.any(live):
            break
        p = np.where(live, p * (mu / step), p)
        F = np.where(live, F + p, F)
        k = np.where(live, step, k)
        live = live & (u > F)
    return k


def poisson_many(mu, pixels, frame: int, seed: int) -> np.ndarray:
    """Poisson(mu[i]) for pixel indices pixels[i] of one frame (vectorised)."""
    mu = np.asarray(mu, dtype=np.float64).reshape(-1)
    pixels = np.asarray(pixels, dtype=np.int64).reshape(-1)
    k0, k1 = seed & MASK, (seed >> 32) & MASK
    out = np.zeros(mu.shape, dtype=np.int64)
    pos = mu > 0
    m = (pixels >> 1).astype(np.uint32)
    z = np.zeros_like(m)
    w = philox4x32_10_np(m, np.full_like(m, frame), z, z, k0, k1)
    odd = (pixels & 1).astype(bool)
    wa = np.where(odd, w[2], w[0])
    wb = np.where(odd, w[3], w[1])
    small = pos & (mu < 10.0)
    if np.any(small):
        out[small] = poisson_inversion(mu[small], uniform(wa[small]))
    large = np.nonzero(pos & (mu >= 10.0))[0]
    if large.size:
        k = ptrs_attempt(uniform(wa[large]), uniform(wb[large]), mu[large])
        done = k >= 0
        out[large[done]] = k[done]
        todo = large[~done]
        for rnd in range(1, 16):
            if todo.size == 0:
                break
            pt = pixels[todo].astype(np.uint32)
            r = philox4x32_10_np(pt, np.full_like(pt, frame), np.full_like(pt, rnd), np.ones_like(pt), k0, k1)
            for t in range(2):
                if todo.size == 0:
                    break
                k = ptrs_attempt(uniform(r[2 * t]), uniform(r[2 * t + 1]), mu[todo])
                done = k >= 0
                out[todo[done]] = k[done]
                keep = ~done
                todo = todo[keep]
                r = tuple(x[keep] for x in r)
        out[todo] = np.floor(mu[todo]).astype(np.int64)  # 31 rejections in a row: never seen
    return out


def poisson_one(mu: float, pixel: int, frame: int, seed: int) -> int:
    """One Poisson(mu) variate for one pixel."""
    return int(poisson_many(np.array([mu]), np.array([pixel]), frame, seed)[0])


def read_normals(pair: int, frame: int, seed: int):
    """Two standard normal variates for pixels 2 pair and 2 pair + 1 (Box and Muller,
    Ann. Math. Statist. 29, 1958) from the first two words u1, u2 of the Philox block
    at counter (pair, frame, 0, 2): r = sqrt(-2 ln u1), (r cos 2 pi u2, r sin 2 pi u2).
    FP64 on the uniforms."""
    key = (seed & MASK, (seed >> 32) & MASK)
    w = philox4x32_10((pair, frame, 0, 2), key)
    u1, u2 = float(uniform_f32(w[0])), float(uniform_f32(w[1]))
    r = math.sqrt(-2.0 * math.log(u1))
    return r * math.cos(2.0 * math.pi * u2), r * math.sin(2.0 * math.pi * u2)


def add_noise(I: np.ndarray, photons_mean: float, seed: int, frame: int = 0,
              mean_I: float | None = None, read_noise: float = 0.0) -> np.ndarray:
    """(counts + read_noise z) / s with counts ~ Poisson(s I), s = photons_mean / mean(I),
    z standard normal (read_normals): the heteroscedastic sensor model of Sec. III.C,
    Poisson shot noise plus Gaussian read noise of read_noise counts."""
    I = np.asarray(I, dtype=np.float64)
    m = float(I.mean()) if mean_I is None else float(mean_I)
    if not (photons_mean > 0) or not (m > 0):
        return I.copy()
    s = photons_mean / m
    flat = I.reshape(-1)
    k = poisson_many(s * flat, np.arange(flat.size), frame, seed).astype(np.float64)
    if read_noise > 0:
        z = np.array([read_normals(p >> 1, frame, seed)[p & 1] for p in range(flat.size)])
        k = k + read_noise * z
    return (k / s).reshape(I.shape)
