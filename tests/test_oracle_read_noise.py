"""Pins of the oracle's Gaussian read noise (Box-Muller on Philox words):
  * the pair identity z0^2 + z1^2 = -2 ln u1 of the block's first word;
  * 40,000 variates pass a Kolmogorov-Smirnov test against the standard normal
    CDF and have mean ~ 0 and variance ~ 1 within 5 standard errors;
  * in add_noise the read noise adds read_noise * z counts to the shot-noise
    counts of the same pixels (counts recovered exactly when subtracted back).
"""
import math

import numpy as np
from scipy import stats

from oracle import noise as N


def test_pair_identity():
    for pair in (0, 1, 77, 123456):
        z0, z1 = N.read_normals(pair, 3, 0x1234567890ABCDEF)
        w = N.philox4x32_10((pair, 3, 0, 2), (0x90ABCDEF, 0x12345678))
        u1 = float(N.uniform_f32(w[0]))
        assert abs(z0 * z0 + z1 * z1 + 2.0 * math.log(u1)) < 1e-12


def test_standard_normal():
    z = np.array([v for p in range(20000) for v in N.read_normals(p, 0, 99)])
    n = z.size
    assert abs(z.mean()) < 5 / math.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_read_noise_adds_to_the_counts():
    rng = np.random.default_rng(0)
    I = rng.uniform(1.0, 3.0, (8, 8))
    shot = N.add_noise(I, 500.0, 11)
    both = N.add_noise(I, 500.0, 11, read_noise=4.0)
    s = 500.0 / I.mean()
    z = np.array([N.read_normals(p >> 1, 0, 11)[p & 1] for p in range(64)]).reshape(8, 8)
    assert np.max(np.abs((both - shot) * s - 4.0 * z)) < 1e-9
    assert np.array_equal(np.round(shot * s), shot * s)  # shot-noise counts are integers
