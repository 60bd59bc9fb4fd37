"""osog_render_noalloc (the render in the library's fixed device scratch) against
osog_render with a caller workspace: bitwise the same images, on two calls in a
row (the second on a smaller frame, so it reuses the scratch the first one left),
and a clear error for a frame whose buffers exceed the scratch."""
import ctypes
from dataclasses import replace

import numpy as np
import pytest
import torch

from gpu_util import dev_globals, dev_soa, need_gpu, say

pytestmark = pytest.mark.gpu


def _frame(seed, n, size, photons):
    from paper_2606_21381_amd import workloads
    rng = np.random.Generator(np.random.PCG64(seed))
    soa = workloads.f32(workloads.mixed(rng, n, size, size))
    opt = workloads.dic_optics(photons=photons, seed=seed)
    return soa, opt


def _both(soa_np, size, opt, g):
    from paper_2606_21381_amd import render
    soa = dev_soa(soa_np)
    gd = dev_globals(g)
    ref, ref_opd = render.render(soa, size, size, opt, gd, want_opd=True)
    out = torch.full((size, size), float("nan"), device="cuda")
    opd = torch.full((size, size), float("nan"), device="cuda")
    render.render_noalloc(soa, size, size, opt, gd, out=out, opd_out=opd)
    out2 = torch.full((size, size), float("nan"), device="cuda")
    render.render_noalloc(soa, size, size, opt, gd, out=out2)  # OPD kept in the scratch
    torch.cuda.synchronize()
    return ref, ref_opd, out, opd, out2


def test_noalloc_matches_render_on_two_calls_in_a_row():
    need_gpu()
    cases = [(41, 40000, 2048, 1000.0, [1.3, 1.0, np.pi / 2, 0.0]),   # the 2048^2 x 40k DIC frame
             (42, 300, 256, 0.0, [-0.7, 1.2, 1.4, 0.0])]              # then a smaller, noiseless one
    for seed, n, size, photons, g in cases:
        say("noalloc case: seed %d, n %d, %d^2, photons %g" % (seed, n, size, photons))
        soa, opt = _frame(seed, n, size, photons)
        ref, ref_opd, out, opd, out2 = _both(soa, size, opt, g)
        assert torch.equal(out, ref), "image differs from osog_render"
        assert torch.equal(opd, ref_opd), "OPD differs from osog_render"
        assert torch.equal(out2, ref), "image without opd_out differs from osog_render"


def test_noalloc_oblique_and_absorbing_frames():
    need_gpu()
    from paper_2606_21381_amd import render, workloads
    rng = np.random.Generator(np.random.PCG64(43))
    soa = workloads.f32(workloads.with_absorption(rng, workloads.mixed(rng, 2000, 1024, 1024)))
    opt = replace(workloads.dic_optics(photons=500.0, seed=9), absorption=1)
    say("noalloc case: absorbing DIC 1024^2, 2000 particles")
    ref, ref_opd = render.render(dev_soa(soa), 1024, 1024, opt, dev_globals([0.4, 1.0, 1.5, 0.0]), want_opd=True)
    out = torch.empty((1024, 1024), device="cuda")
    opd = torch.empty((2, 1024, 1024), device="cuda")
    render.render_noalloc(dev_soa(soa), 1024, 1024, opt, dev_globals([0.4, 1.0, 1.5, 0.0]), out=out, opd_out=opd)
    torch.cuda.synchronize()
    assert torch.equal(out, ref) and torch.equal(opd, ref_opd)
    say("noalloc case: oblique 512^2, 800 particles")
    soa2 = workloads.f32(workloads.mixed(rng, 800, 512, 512))
    opt2 = workloads.OpticsSpec(mode=workloads.OBLIQUE, na=0.5, tilt_fx=0.3 * 0.5 / 0.55)
    g2 = dev_globals([1.0, 0.0, 0.0, 0.0])
    ref2 = render.render(dev_soa(soa2), 512, 512, opt2, g2)
    out2 = torch.empty((512, 512), device="cuda")
    render.render_noalloc(dev_soa(soa2), 512, 512, opt2, g2, out=out2)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref2)


def test_noalloc_rejects_frames_beyond_the_scratch():
    need_gpu()
    from paper_2606_21381_amd import _lib, render, workloads
    lib = _lib.load()
    say("noalloc case: 4096^2 without opd_out (beyond the scratch)")
    soa = dev_soa(workloads.f32(workloads.mixed(np.random.Generator(np.random.PCG64(44)), 100, 4096, 4096)))
    g = dev_globals([0.0, 1.0, np.pi / 2, 0.0])
    out = torch.zeros((4096, 4096), device="cuda")
    o = _lib.make_optics(workloads.dic_optics(photons=0.0))
    st = lib.osog_render_noalloc(render.context(), None, 4096, 4096, ctypes.c_void_p(soa.data_ptr()), 100,
                                 soa.stride(0), ctypes.byref(o), ctypes.c_void_p(g.data_ptr()), None,
                                 ctypes.c_void_p(out.data_ptr()))
    assert st == _lib.ERR_WORKSPACE
    assert b"bytes of scratch" in lib.osog_last_error()
    torch.cuda.synchronize()
    assert float(out.abs().max()) == 0.0  # nothing was launched
