"""Calibration against a target that cannot be aligned pixel by pixel (paper
Sec. IV.B, DiffOSOG): the target is another random placement of prisms with the
same statistics, rendered with the true optics; the model's own placement stays
frozen (a curriculum stage that moves only defocus and bias) and Adam descends
the spectral loss of Eq. 8 through the renderer's adjoint.  The pixel-wise MSE
has no meaning against such a target and lands far from the true defocus.
(The amplitude spectrum of a phase object's image does not see the sign of the
defocus, so the start is taken on the true side.)"""
import numpy as np
import pytest
import torch

from paper_2606_21381_amd import inverse, render, workloads
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def prism_table(seed, n, size):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = workloads.prisms(rng, n, size, size)
    s[6] = 0.03
    return torch.from_numpy(workloads.f32(s)).cuda()


def test_spectral_loss_recovers_defocus_from_an_unaligned_target():
    need_gpu()
    size, n = 512, 800
    opt = workloads.dic_optics(0.0)
    dz_t, bias_t = 0.7, 1.2
    T = render.render(prism_table(1, n, size), size, size, opt,
                      torch.tensor([dz_t, 1.0, bias_t, 0], device="cuda"))
    s0 = prism_table(2, n, size)
    out = {}
    for loss in ("spectral", "mse"):
        glob0 = torch.tensor([0.03, 1.8, 1.0, 0.9], dtype=torch.float32, device="cuda")
        p = inverse.Params(s0[0], s0[1], s0[2], s0[3], s0[5], glob0).cuda()
        cfg = inverse.SolverConfig(steps=300, loss=loss, curriculum=((300, ("dz", "bias")),),
                                   lr_dz=0.05, lr_bias=0.02)
        r = inverse.solve(T, p, None, size, size, opt, cfg)
        out[loss] = r.final
        say("%s: dz %.4f (true %.1f), bias %.4f (true %.1f), loss %.4g -> %.4g" % (
            loss, r.final["dz"], dz_t, r.final["bias"], bias_t, r.loss[0], r.loss[-1]))
    assert abs(out["spectral"]["dz"] - dz_t) < 0.1
    assert abs(out["spectral"]["bias"] - bias_t) < 0.15
    assert abs(out["mse"]["dz"] - dz_t) > 0.4
