"""Batched rendering (one HIP graph launch): every frame bitwise equal to its single-frame render."""
import math

import numpy as np
import pytest
import torch

from paper_2606_21381_amd import workloads
from tests.gpu_util import dev_globals, dev_soa, need_gpu, say

pytestmark = pytest.mark.gpu


def frames_small(seed=7, count=10):
    out = []
    rng = np.random.Generator(np.random.PCG64(seed))
    for f in range(count):
        size = int(rng.choice([128, 256, 512]))
        n = int(rng.integers(0, 1500)) if f != 3 else 0
        soa = workloads.f32(workloads.mixed(rng, n, size, size))
        if f % 2 == 0:
            opt = workloads.dic_optics(1000.0 if f % 4 == 0 else 0.0, seed=100 + f)
            g = [rng.uniform(-2, 2), 1.0, math.pi / 2, 0]
        else:
            opt = workloads.OpticsSpec(mode=workloads.OBLIQUE, na=0.5, tilt_fx=0.3 * 0.5 / 0.55,
                                       photons_mean=1000.0 if f % 3 == 0 else 0.0, seed=200 + f)
            g = [rng.uniform(-2, 2), 0, 0, 0]
        out.append((dev_soa(soa), size, size, opt, dev_globals(g)))
    return out


def test_batch_equals_single_frames_bitwise():
    need_gpu()
    from paper_2606_21381_amd import render
    fr = frames_small()
    singles = []
    for f, (soa, H, W, opt, g) in enumerate(fr):
        say("single frame %d: %dx%d, n=%d, mode %d, photons %g" % (f, H, W, soa.shape[1], opt.mode, opt.photons_mean))
        I, opd = render.render(soa, H, W, opt, g, want_opd=True)
        torch.cuda.synchronize()
        singles.append((I, opd))
    for group in (0, 3):
        render.set_batch_group(group)
        b = render.Batch(fr, want_opd=True)
        for rep in range(2):  # second call replays the captured graph
            say("batch of %d small frames, group %d, call %d" % (len(fr), group, rep))
            b.run()
            torch.cuda.synchronize()
            assert b.error_flag() == 0
            for f, (I, opd) in enumerate(singles):
                assert torch.equal(opd, b.opd[f]), (group, rep, f)
                assert torch.equal(I, b.out[f]), (group, rep, f)
        lat = b.latencies_ms()
        say("group %d: frame latencies ms p50 %.3f max %.3f" % (group, np.median(lat), lat.max()))
        assert np.all(lat > 0)
    render.set_batch_group(4)


def test_batch_headline_mix_runs_and_matches_spot_frames():
    need_gpu()
    from paper_2606_21381_amd import render
    frs = workloads.config2()
    fr = [(dev_soa(x.soa), x.H, x.W, x.optics, dev_globals(x.globals4)) for x in frs]
    b = render.Batch(fr)
    say("batch of %d headline-mix frames" % len(fr))
    b.run()
    torch.cuda.synchronize()
    assert b.error_flag() == 0
    for f in (0, 17, 40, 63):
        soa, H, W, opt, g = fr[f]
        I = render.render(soa, H, W, opt, g)
        torch.cuda.synchronize()
        assert torch.equal(I, b.out[f]), f
