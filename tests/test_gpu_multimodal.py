"""Several modalities from one binning, raster and row FFT: each output equal bit
for bit to its own single-modality render, and to the FP64 oracle's image of the
same OPD within the stated tolerances."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2606_21381_amd import workloads
from tests.gpu_util import dev_globals, dev_soa, need_gpu, oracle_optics, rel_l2, say

pytestmark = pytest.mark.gpu


def modes():
    return [
        (workloads.OpticsSpec(mode=workloads.BRIGHTFIELD, na=0.4), [1.0, 0.0, 0.0, 0.0]),
        (workloads.dic_optics(0.0), [-0.7, 1.0, math.pi / 2, 0.0]),
        (workloads.OpticsSpec(mode=workloads.OBLIQUE, na=0.5, tilt_fx=0.3 * 0.5 / 0.55), [0.4, 0.0, 0.0, 0.0]),
        (workloads.dic_optics(1000.0, seed=7), [0.3, 1.1, 0.45 * math.pi, 0.0]),
        (workloads.OpticsSpec(mode=workloads.DIC, na=0.3, shear_angle_rad=0.0), [0.0, 2.0, 1.2, 0.0]),
    ]


@pytest.mark.parametrize("size,n", [(256, 300), (512, 2000)])
def test_multimodal_equals_single_renders_and_oracle(size, n):
    need_gpu()
    from paper_2606_21381_amd import render
    rng = np.random.Generator(np.random.PCG64(size + n))
    soa = workloads.f32(workloads.mixed(rng, n, size, size))
    ms = modes()
    g = torch.tensor([m[1] for m in ms], dtype=torch.float32, device="cuda")
    s = dev_soa(soa)
    say("multimodal %d^2, %d particles, %d modes" % (size, n, len(ms)))
    outs, opd = render.render_multi(s, size, size, [m[0] for m in ms], g, want_opd=True)
    torch.cuda.synchronize()
    ref_opd = oracle.raster.opd(soa, size, size)
    e_opd = float(np.abs(opd.cpu().numpy() - ref_opd).max())
    assert e_opd <= 1e-5
    for k, (opt, gl) in enumerate(ms):
        single = render.render(s, size, size, opt, dev_globals(gl))
        torch.cuda.synchronize()
        assert torch.equal(single, outs[k]), k
        if opt.photons_mean == 0.0:
            ref = oracle.optics.intensity(ref_opd, oracle_optics(opt), gl[0], gl[1], gl[2])
            e = rel_l2(outs[k].cpu().numpy(), ref)
            say("  mode %d (kind %d, NA %.2f): I rel L2 %.2e, bitwise equal to its single render" % (k, opt.mode, opt.na, e))
            assert e <= 1e-4
        else:
            say("  mode %d (kind %d, noise): bitwise equal to its single render" % (k, opt.mode))


def test_multimodal_rejects_mixed_wavelengths():
    need_gpu()
    from paper_2606_21381_amd import render
    from dataclasses import replace
    soa = dev_soa(workloads.f32(workloads.mixed(np.random.default_rng(1), 10, 64, 64)))
    a = workloads.OpticsSpec(mode=workloads.BRIGHTFIELD, na=0.4)
    b = replace(a, wavelength_um=0.6)
    g = torch.zeros((2, 4), dtype=torch.float32, device="cuda")
    with pytest.raises(RuntimeError, match="wavelength"):
        render.render_multi(soa, 64, 64, [a, b], g)
