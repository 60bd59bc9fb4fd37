"""Pins of the oracle's shot noise: Philox known answers and Poisson moments."""
import os

import numpy as np
import pytest

from oracle import noise

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    rows = [l.split() for l in open(GOLD) if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        assert noise.philox4x32_10(v[0:4], v[4:6]) == tuple(v[6:10])
        vec = noise.philox4x32_10_np(*[np.array([x], np.uint32) for x in v[0:4]], v[4], v[5])
        assert tuple(int(x[0]) for x in vec) == tuple(v[6:10])


def test_uniform_range_exact():
    assert noise.uniform_f32(0) == np.float32(2.0 ** -24)
    assert noise.uniform_f32(0xFFFFFFFF) == np.float32(1 - 2.0 ** -24)


@pytest.mark.parametrize("mu", [0.7, 4.0, 9.9, 10.0, 37.5, 1000.0, 4000.0])
def test_poisson_moments(mu):
    n = 6000
    x = np.array([noise.poisson_one(mu, p, 3, 12345) for p in range(n)], dtype=np.float64)
    assert abs(x.mean() - mu) < 4.5 * np.sqrt(mu / n)
    # variance of the sample variance ~ 2 mu^2 / n (+ mu / n)
    assert abs(x.var() - mu) < 4.5 * np.sqrt((2 * mu * mu + mu) / n)
    assert np.all(x >= 0) and np.all(x == np.round(x))


def test_poisson_small_mean_pmf():
    from scipy.stats import poisson
    mu, n = 2.5, 8000
    x = np.array([noise.poisson_one(mu, p, 0, 7) for p in range(n)])
    for k in range(7):
        f = np.mean(x == k)
        pk = poisson.pmf(k, mu)
        assert abs(f - pk) < 4.5 * np.sqrt(pk * (1 - pk) / n)


def test_add_noise_scaling_and_seed():
    I = np.full((20, 20), 4.0)
    a = noise.add_noise(I, 1000.0, seed=9)
    b = noise.add_noise(I, 1000.0, seed=9)
    c = noise.add_noise(I, 1000.0, seed=10)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    z = (a * 250.0 - 1000.0) / np.sqrt(1000.0)       # s = 1000 / 4
    assert abs(z.mean()) < 4.5 / 20 and abs(z.var() - 1) < 0.35


def test_log_factorial_matches_lgamma():
    import math
    for k in list(range(0, 40)) + [57, 99, 512, 1000, 1003, 4096, 20000]:
        ref = math.lgamma(k + 1.0)
        got = float(noise.log_factorial_f32(float(k)))
        assert abs(got - ref) <= 2e-7 * max(1.0, abs(ref)) + 1e-6, k
