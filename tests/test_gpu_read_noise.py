"""Gaussian read noise of the sensor model (Sec. III.C, Poisson plus Gaussian)
on the GPU against the oracle: removing the oracle's read-noise term from the
GPU image leaves integer counts equal to the oracle's shot-noise counts, the
variance of a uniform field is photons + sigma^2, and read noise without a
photon scale is refused."""
import math

import numpy as np
import pytest
import torch
from dataclasses import replace

import oracle
from paper_2606_21381_amd import _lib, render, workloads
from tests.gpu_util import dev_globals, dev_soa, need_gpu, say

pytestmark = pytest.mark.gpu


def test_read_noise_matches_the_oracle_generator():
    need_gpu()
    rng = np.random.Generator(np.random.PCG64(10))
    soa = workloads.f32(workloads.mixed(rng, 30, 64, 64))
    g = np.array([0.3, 1.0, math.pi / 2, 0], np.float32)
    sigma = 6.0
    opt = replace(workloads.dic_optics(1000.0, 5), read_noise=sigma)
    Ig = render.render(dev_soa(soa), 64, 64, opt, dev_globals(g)).cpu().double().numpy()
    clean = oracle.render(soa, 64, 64, oracle.Optics(mode=1, na=0.5, shear_angle_rad=math.pi / 4), g)[1]
    s = 1000.0 / clean.mean()
    z = np.array([oracle.noise.read_normals(p >> 1, 0, 5)[p & 1] for p in range(64 * 64)]).reshape(64, 64)
    counts = Ig * s - sigma * z
    shot = oracle.noise.add_noise(clean, 1000.0, 5) * s
    frac = float(np.max(np.abs(counts - np.round(counts))))
    same = float(np.mean(np.round(counts) == np.round(shot)))
    say("read noise: |counts - integer| <= %.2e, counts equal to the oracle's on %.4f of pixels" % (frac, same))
    assert frac < 2e-3 and same > 0.98


def test_read_noise_variance_on_a_uniform_field():
    need_gpu()
    soa = torch.zeros((8, 0), dtype=torch.float32, device="cuda")
    sigma = 20.0
    opt = workloads.OpticsSpec(mode=1, na=0.5, shear_angle_rad=math.pi / 4, photons_mean=1000.0, seed=77,
                               read_noise=sigma)
    I = render.render(soa, 512, 512, opt, dev_globals([0.3, 1.0, math.pi / 2, 0])).cpu().double().numpy()
    c = I * 250.0  # s = 1000 / 4
    n = c.size
    var_expect = 1000.0 + sigma * sigma
    z = (c.var() - var_expect) / (var_expect * math.sqrt(2.0 / n))
    say("uniform field: mean %.3f (1000), variance %.1f (%.1f), z %.2f" % (c.mean(), c.var(), var_expect, z))
    assert abs(c.mean() - 1000.0) < 5 * math.sqrt(var_expect / n) and abs(z) < 5


def test_read_noise_needs_photons():
    need_gpu()
    soa = torch.zeros((8, 0), dtype=torch.float32, device="cuda")
    opt = workloads.OpticsSpec(mode=1, na=0.5, read_noise=3.0)
    with pytest.raises(_lib.OsogError) as e:
        render.render(soa, 64, 64, opt, dev_globals([0, 1, 1, 0]))
    assert e.value.status == 1
