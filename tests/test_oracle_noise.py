"""Pins of the oracle's shot noise.

  * Philox4x32-10 against the generator's published known-answer vectors;
  * the word-to-uniform map's end points;
  * sample mean and variance of Poisson(mu) over the inversion and the PTRS ranges;
  * the empirical PMF against scipy's Poisson PMF by a chi-square test, for the
    inversion (mu = 2.5) and for PTRS (mu = 37.5, 1000), which is an exact sampler;
  * the chi-square test has the power to see a plausible slip: with log k! off by
    one factorial (log (k-1)!) the same test fails (the slip is planted here, in the
    oracle, on the CPU);
  * add_noise's scale s = photons / mean(I) and its seed dependence.
"""
import math
import os

import numpy as np
import pytest
from scipy import stats

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
    w = np.array([0, 1 << 9, 0xFFFFFFFF], np.uint32)
    assert np.array_equal(noise.uniform(w), [float(noise.uniform_f32(int(x))) for x in w])


@pytest.mark.parametrize("mu", [0.7, 4.0, 9.9, 10.0, 37.5, 1000.0, 4000.0])
def test_poisson_moments(mu):
    n = 20000
    x = noise.poisson_many(np.full(n, mu), np.arange(n), 3, 12345).astype(np.float64)
    assert abs(x.mean() - mu) < 4.5 * np.sqrt(mu / n)
    # variance of the sample variance ~ 2 mu^2 / n (+ mu / n)
    assert abs(x.var() - mu) < 4.5 * np.sqrt((2 * mu * mu + mu) / n)
    assert np.all(x >= 0)


def chi2_pvalue(x, mu):
    """Chi-square goodness of fit of integer samples x to Poisson(mu), bins with
    expected count >= 20 (tails pooled)."""
    n = x.size
    lo, hi = int(stats.poisson.ppf(1e-4, mu)), int(stats.poisson.ppf(1 - 1e-4, mu))
    edges = list(range(lo, hi + 1))
    # pool neighbouring values until every bin expects >= 20 samples
    bins, cur = [], [edges[0]]
    for k in edges[1:]:
        if n * stats.poisson.pmf(cur, mu).sum() >= 20:
            bins.append(cur)
            cur = [k]
        else:
            cur.append(k)
    bins.append(cur)
    obs, exp = [], []
    obs.append(np.sum(x < bins[0][0]))
    exp.append(n * stats.poisson.cdf(bins[0][0] - 1, mu))
    for b in bins:
        obs.append(np.sum((x >= b[0]) & (x <= b[-1])))
        exp.append(n * (stats.poisson.cdf(b[-1], mu) - stats.poisson.cdf(b[0] - 1, mu)))
    obs.append(np.sum(x > bins[-1][-1]))
    exp.append(n * stats.poisson.sf(bins[-1][-1], mu))
    obs, exp = np.array(obs, float), np.array(exp, float)
    keep = exp > 0
    chi2 = np.sum((obs[keep] - exp[keep]) ** 2 / exp[keep])
    return stats.chi2.sf(chi2, keep.sum() - 1)


@pytest.mark.parametrize("mu", [2.5, 37.5, 1000.0])
def test_pmf_chi_square(mu):
    n = 200000
    x = noise.poisson_many(np.full(n, mu), np.arange(n), 1, 2024)
    assert chi2_pvalue(x, mu) > 1e-4


def test_chi_square_sees_a_wrong_log_factorial(monkeypatch):
    monkeypatch.setattr(noise, "_log_factorial",
                        lambda k: np.array([math.lgamma(float(v)) if v > 0 else 0.0 for v in np.ravel(k)]))
    n = 200000
    x = noise.poisson_many(np.full(n, 37.5), np.arange(n), 1, 2024)
    assert chi2_pvalue(x, 37.5) < 1e-6


def test_scalar_and_vector_paths_agree():
    mus = np.array([0.3, 5.0, 9.99, 10.0, 80.0, 2500.0])
    v = noise.poisson_many(mus, np.arange(6) + 100, 2, 99)
    s = [noise.poisson_one(m, p + 100, 2, 99) for p, m in enumerate(mus)]
    assert list(v) == s


def test_add_noise_scaling_and_seed():
    I = np.full((40, 40), 4.0)
    a = noise.add_noise(I, 1000.0, seed=9)
    b = noise.add_noise(I, 1000.0, seed=9)
    c = noise.add_noise(I, 1000.0, seed=10)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    z = (a * 250.0 - 1000.0) / np.sqrt(1000.0)       # s = 1000 / 4
    assert abs(z.mean()) < 4.5 / 40 and abs(z.var() - 1) < 0.2
    assert np.max(np.abs(np.round(a * 250.0) - a * 250.0)) < 1e-9
