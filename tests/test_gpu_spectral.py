"""The spectral loss of Eq. 8 on the GPU against the FP64 oracle: loss (relative
1e-4) and gradient (relative L2 1e-3) on rendered images, shift invariance,
zero at the target, and its gradient composed with the renderer's adjoint
against central differences of the oracle in the optical globals.

eps sits inside the logarithms.  A noiseless image is band-limited: beyond the
optics' cut-off its bins hold only the rounding of the transforms (FP32 on the
GPU, ~1e-7 of the DC term), which the logarithm would amplify, so eps is taken
well above that floor -- 1e-4 of the target's DC term -- wherever the tests
compare with the FP64 oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2606_21381_amd import render, workloads
from tests.gpu_util import dev_globals, dev_soa, need_gpu, oracle_optics, rel_l2, say

pytestmark = pytest.mark.gpu

EPS = 1.0


def frame_image(seed, size, n, photons):
    rng = np.random.Generator(np.random.PCG64(seed))
    soa = workloads.f32(workloads.mixed(rng, n, size, size))
    g = np.array([rng.uniform(-1, 1), 1.0, math.pi / 2, 0], np.float32)
    opt = workloads.dic_optics(photons, seed)
    I = render.render(dev_soa(soa), size, size, opt, dev_globals(g))
    torch.cuda.synchronize()
    return soa, opt, g, I


@pytest.mark.parametrize("size,photons", [(256, 1000.0), (512, 0.0), (1024, 1000.0)])
def test_spectral_loss_and_gradient_parity(size, photons):
    need_gpu()
    say("spectral loss parity %d^2 photons %.0f" % (size, photons))
    _, _, _, I = frame_image(400 + size, size, size * size // 200, photons)
    _, _, _, T = frame_image(500 + size, size, size * size // 200, photons)
    eps = 1e-4 * float(T.double().sum())
    tl = render.spectral_target(T, eps)
    loss, grad = render.spectral_loss(I, tl, eps)
    torch.cuda.synchronize()
    In, Tn = I.cpu().double().numpy(), T.cpu().double().numpy()
    rl = oracle.spectral.loss(In, Tn, eps)
    rg = oracle.spectral.grad(In, Tn, eps)
    el = abs(float(loss) - rl) / rl
    eg = rel_l2(grad.cpu().numpy(), rg)
    say("  loss %.6e (oracle %.6e, rel %.2e), gradient rel L2 %.2e" % (float(loss), rl, el, eg))
    assert el <= 1e-4 and eg <= 1e-3


def test_spectral_loss_shift_invariance_and_zero_at_target():
    need_gpu()
    _, _, _, I = frame_image(7, 512, 1500, 1000.0)
    _, _, _, T = frame_image(8, 512, 1500, 1000.0)
    tl = render.spectral_target(T, EPS)
    base = float(render.spectral_loss(I, tl, EPS, want_grad=False)[0])
    for sh in ((5, 0), (0, 17), (100, 33)):
        v = float(render.spectral_loss(torch.roll(I, sh, dims=(0, 1)), tl, EPS, want_grad=False)[0])
        say("shift %s: loss %.7e vs %.7e" % (sh, v, base))
        assert abs(v - base) <= 1e-5 * base
    assert float(render.spectral_loss(T, tl, EPS, want_grad=False)[0]) == 0.0


def test_spectral_gradient_through_the_renderer_vs_fd():
    """d L_spectral(render(globals)) / d globals: the spectral gradient image fed to
    the renderer's adjoint, against FP64 central differences of the oracle."""
    need_gpu()
    size = 128
    rng = np.random.Generator(np.random.PCG64(31))
    soa = workloads.f32(workloads.mixed(rng, 60, size, size))
    opt = workloads.dic_optics(0.0)
    g = np.array([0.6, 1.0, 1.3, 0], np.float32)
    gt = np.array([-0.4, 1.2, 1.5, 0], np.float32)
    # target: a different placement of particles (not pixel-aligned), other globals
    soa_t = workloads.f32(workloads.mixed(np.random.Generator(np.random.PCG64(32)), 60, size, size))
    T = render.render(dev_soa(soa_t), size, size, opt, dev_globals(gt))
    eps = 1e-4 * float(T.double().sum())
    tl = render.spectral_target(T, eps)
    I = render.render(dev_soa(soa), size, size, opt, dev_globals(g))
    _, gI = render.spectral_loss(I, tl, eps)
    _, gg = render.render_backward(dev_soa(soa), size, size, opt, dev_globals(g), gI, need_soa=False)
    torch.cuda.synchronize()
    gg = gg.cpu().double().numpy()
    Tn = T.cpu().double().numpy()
    o = oracle_optics(opt)
    opd = oracle.raster.opd(soa, size, size)

    def L(gv):
        return oracle.spectral.loss(oracle.optics.intensity(opd, o, gv[0], gv[1], gv[2]), Tn, eps)

    g64 = g.astype(np.float64)
    for k in range(3):
        d = 1e-5
        p, m = g64.copy(), g64.copy()
        p[k] += d
        m[k] -= d
        fd = (L(p) - L(m)) / (2 * d)
        e = abs(gg[k] - fd) / abs(fd)
        say("global %d: gpu %.6e fd %.6e rel %.2e" % (k, gg[k], fd, e))
        assert e <= 2e-3
