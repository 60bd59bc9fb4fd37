"""The 2048^2 DIC frame with its 40,000 particles in 64 Gaussian clusters (sigma
25 px; a 16 x 16 tile at a core holds up to 323 particles): binning bit-exact
against the oracle, OPD and image against the FP64 oracle, and the canvas bitwise
the same under another tiling."""
import numpy as np
import pytest
import torch

import oracle
from gpu_util import dev_globals, dev_soa, need_gpu, oracle_optics, rel_l2, say

pytestmark = pytest.mark.gpu


def test_clustered_frame_bins_and_renders_like_the_oracle():
    need_gpu()
    from dataclasses import replace
    from paper_2606_21381_amd import render, workloads
    fr = workloads.config1_clustered(photons=0.0)
    soa, g = dev_soa(fr.soa), dev_globals(fr.globals4)
    th, tw = render.get_tiling()
    keys, pids, ts, counts, P = render.bin_pairs(soa, fr.H, fr.W)
    ref = oracle.binning.bin_pairs(fr.soa, fr.H, fr.W, th, tw)
    per_tile = np.diff(ref["tile_start"])
    say("clustered: %d pairs, max %d per tile, %d tiles over 64" % (P, per_tile.max(), (per_tile > 64).sum()))
    assert (per_tile > 64).sum() > 100
    assert np.array_equal(keys.cpu().numpy(), ref["keys"]) and np.array_equal(pids.cpu().numpy(), ref["pids"])
    assert np.array_equal(ts.cpu().numpy(), ref["tile_start"])
    I, opd = render.render(soa, fr.H, fr.W, fr.optics, g, want_opd=True)
    torch.cuda.synchronize()
    ropd = oracle.raster.opd(fr.soa, fr.H, fr.W)
    rI = oracle.optics.intensity(ropd, oracle_optics(fr.optics), *[float(v) for v in fr.globals4[:3]])
    e_opd = float(np.abs(opd.cpu().numpy() - ropd).max())
    e_i = rel_l2(I.cpu().numpy(), rI)
    say("clustered 2048^2 x 40000 DIC: OPD max abs %.3e um, I rel L2 %.3e" % (e_opd, e_i))
    assert e_opd <= 1e-5 and e_i <= 1e-4
    render.set_tiling(*((16, 16) if (th, tw) != (16, 16) else (32, 16)))
    try:
        I2, opd2 = render.render(soa, fr.H, fr.W, fr.optics, g, want_opd=True)
        torch.cuda.synchronize()
    finally:
        render.set_tiling(th, tw)
    assert torch.equal(opd, opd2) and torch.equal(I, I2)
