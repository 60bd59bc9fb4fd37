"""DIC as Eq. 5 writes it (mode OSOG_DIC_INCOHERENT) on the GPU, against the
FP64 oracle: image relative L2 <= 1e-4 (phase and absorbing tables), the empty
field's 4 sin^2(theta), shot noise, the batch path (bitwise its single renders)
and the entry points that do not take this mode."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2606_21381_amd import _lib, render, workloads
from tests.gpu_util import dev_globals, dev_soa, need_gpu, oracle_optics, rel_l2, say

pytestmark = pytest.mark.gpu

I_TOL = 1e-4


def inc_optics(na=0.5, photons=0.0, seed=0, absorption=0):
    return workloads.OpticsSpec(mode=workloads.DIC_INCOHERENT, na=na, shear_angle_rad=math.pi / 4,
                                photons_mean=photons, seed=seed, absorption=absorption)


def frame(seed, size, n, absorption=0):
    rng = np.random.Generator(np.random.PCG64(seed))
    s = workloads.mixed(rng, n, size, size)
    if absorption:
        s = workloads.with_absorption(rng, s)
    g = np.array([rng.uniform(-1.5, 1.5), rng.uniform(0.8, 1.6), (math.pi / 2) * rng.uniform(0.7, 1.1), 0], np.float32)
    return workloads.f32(s), g


def oracle_image(soa, size, opt, g):
    opd = oracle.raster.opd(soa, size, size)
    tau = oracle.raster.absorbance(soa, size, size) if soa.shape[0] == 9 else None
    return oracle.optics.intensity(opd, oracle_optics(opt), float(g[0]), float(g[1]), float(g[2]), tau=tau)


@pytest.mark.parametrize("size,n,na,absorption", [(256, 300, 0.5, 0), (512, 2000, 0.5, 1), (512, 2000, 0.9, 0),
                                                  (1024, 10000, 0.5, 0)])
def test_incoherent_dic_parity(size, n, na, absorption):
    need_gpu()
    say("incoherent DIC parity: %d^2 n=%d NA %.1f absorption %d" % (size, n, na, absorption))
    soa, g = frame(70 + size + absorption, size, n, absorption)
    opt = inc_optics(na=na, absorption=absorption)
    I = render.render(dev_soa(soa), size, size, opt, dev_globals(g)).cpu().numpy()
    rI = oracle_image(soa, size, opt, g)
    e = rel_l2(I, rI)
    # the coherent DIC of the same frame differs (the check is not vacuous)
    coh = oracle.optics.intensity(oracle.raster.opd(soa, size, size),
                                  oracle_optics(workloads.OpticsSpec(mode=workloads.DIC, na=na,
                                                                     shear_angle_rad=math.pi / 4)),
                                  float(g[0]), float(g[1]), float(g[2]),
                                  tau=oracle.raster.absorbance(soa, size, size) if absorption else None)
    say("  I rel L2 %.3e (coherent DIC differs by %.3e)" % (e, rel_l2(coh, rI)))
    assert e <= I_TOL
    assert rel_l2(coh, rI) > 1e-2


def test_incoherent_dic_empty_field():
    need_gpu()
    soa = torch.zeros((8, 0), dtype=torch.float32, device="cuda")
    for dz, th in ((0.0, 1.2), (1.7, math.pi / 2)):
        I = render.render(soa, 256, 256, inc_optics(), dev_globals([dz, 1.0, th, 0])).cpu().double().numpy()
        want = 4 * math.sin(th) ** 2
        say("empty field dz %.1f: I in [%.7f, %.7f], closed form %.7f" % (dz, I.min(), I.max(), want))
        assert np.max(np.abs(I - want)) <= 1e-5 * want


def test_incoherent_dic_noise_matches_oracle_sampler():
    need_gpu()
    soa, g = frame(91, 64, 30)
    opt = inc_optics(photons=1000.0, seed=5)
    Ig = render.render(dev_soa(soa), 64, 64, opt, dev_globals(g)).cpu().double().numpy()
    clean = oracle_image(soa, 64, opt, g)
    ref = oracle.noise.add_noise(clean, 1000.0, 5)
    s = 1000.0 / clean.mean()
    same = float(np.mean(np.round(Ig * s) == np.round(ref * s)))
    say("incoherent DIC with noise: counts identical to the oracle's on %.4f of pixels" % same)
    assert same > 0.98


def test_incoherent_dic_in_a_batch_is_bitwise_single():
    need_gpu()
    frames = []
    for f in range(4):
        size = (256, 512)[f % 2]
        soa, g = frame(300 + f, size, 500 + 200 * f)
        opt = inc_optics() if f % 2 == 0 else workloads.dic_optics(0.0)
        frames.append((dev_soa(soa), size, size, opt, dev_globals(g)))
    singles = [render.render(s, H, W, o, g) for (s, H, W, o, g) in frames]
    torch.cuda.synchronize()
    outs = render.Batch(frames).run()
    torch.cuda.synchronize()
    for f, (a, b) in enumerate(zip(singles, outs)):
        assert torch.equal(a, b), f
    say("batch with 2 incoherent DIC frames: bitwise equal to single renders")


def test_incoherent_dic_is_forward_only():
    need_gpu()
    soa, g = frame(5, 64, 10)
    s, gl = dev_soa(soa), dev_globals(g)
    with pytest.raises(_lib.OsogError) as e:
        render.render_backward(s, 64, 64, inc_optics(), gl, torch.ones((64, 64), device="cuda"))
    assert e.value.status == 2  # OSOG_ERR_UNSUPPORTED
    with pytest.raises(_lib.OsogError) as e:
        render.render_multi(s, 64, 64, [inc_optics()], gl.view(1, 4))
    assert e.value.status == 2
    # the small (forward) workspace is refused with a clear error (at 512^2 the
    # incoherent mode's full-width spectra need megabytes more than the forward
    # carve holds, whatever pair capacity it is given)
    soa5, g5 = frame(5, 512, 10)
    s5, gl5 = dev_soa(soa5), dev_globals(g5)
    small = torch.empty(render.workspace_size(512, 512, 10, False), dtype=torch.uint8, device="cuda")
    with pytest.raises(_lib.OsogError) as e:
        render.render(s5, 512, 512, inc_optics(), gl5, workspace=small)
    assert e.value.status == 3  # OSOG_ERR_WORKSPACE
