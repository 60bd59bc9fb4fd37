"""GPU parity of the forward path against the FP64 oracle (calls through the C ABI).

Tolerances: OPD max abs <= 1e-5 um; noiseless intensity relative L2 <= 1e-4;
binning bit-exact.
"""
import math
from dataclasses import replace

import numpy as np
import pytest
import torch

import oracle
from paper_2606_21381_amd import workloads
from tests.gpu_util import dev_globals, dev_soa, need_gpu, oracle_optics, rel_l2, say

pytestmark = pytest.mark.gpu

OPD_TOL = 1e-5
I_TOL = 1e-4


def R():
    need_gpu()
    from paper_2606_21381_amd import render
    return render


def gpu_frame(fr, want_opd=True, optics=None):
    r = R()
    opt = optics or fr.optics
    I, opd = r.render(dev_soa(fr.soa), fr.H, fr.W, opt, dev_globals(fr.globals4), want_opd=True)
    torch.cuda.synchronize()
    return opd.cpu().numpy(), I.cpu().numpy()


def oracle_frame(fr, optics=None):
    opt = optics or fr.optics
    opd = oracle.raster.opd(fr.soa, fr.H, fr.W)
    g = fr.globals4.astype(np.float64)
    I = oracle.optics.intensity(opd, oracle_optics(opt), g[0], g[1], g[2])
    return opd, I


def mid_frame(seed, size, n, mode):
    rng = np.random.Generator(np.random.PCG64(seed))
    soa = workloads.f32(workloads.mixed(rng, n, size, size))
    if mode == workloads.OBLIQUE:
        opt = workloads.OpticsSpec(mode=mode, na=0.5, tilt_fx=0.3 * 0.5 / 0.55)
        g = [rng.uniform(-2, 2), 0, 0, 0]
    elif mode == workloads.DIC:
        opt = workloads.dic_optics(0.0)
        g = [rng.uniform(-2, 2), 1.0, math.pi / 2, 0]
    else:
        opt = workloads.OpticsSpec(mode=mode, na=0.4)
        g = [1.0, 0, 0, 0]
    return workloads.Frame(size, size, soa, opt, np.array(g, np.float32), "mid")


@pytest.mark.parametrize("tiling", [(16, 16), (8, 32), (32, 8), (32, 32), (16, 64)])
def test_binning_bit_exact(tiling):
    r = R()
    fr = workloads.config1(n=5000, size=1024)
    th0, tw0 = r.get_tiling()
    r.set_tiling(*tiling)
    try:
        keys, pids, ts, counts, P = r.bin_pairs(dev_soa(fr.soa), fr.H, fr.W)
        ref = oracle.binning.bin_pairs(fr.soa, fr.H, fr.W, *tiling)
        say("binning", tiling, "pairs", P)
        assert P == len(ref["keys"])
        assert np.array_equal(keys.cpu().numpy(), ref["keys"])
        assert np.array_equal(pids.cpu().numpy(), ref["pids"])
        assert np.array_equal(ts.cpu().numpy(), ref["tile_start"])
        assert np.array_equal(counts.cpu().numpy(), ref["counts"])
    finally:
        r.set_tiling(th0, tw0)


def test_binning_bit_exact_full_size():
    r = R()
    fr = workloads.config1()
    keys, pids, ts, counts, P = r.bin_pairs(dev_soa(fr.soa), fr.H, fr.W)
    ref = oracle.binning.bin_pairs(fr.soa, fr.H, fr.W, *r.get_tiling())
    say("binning 2048^2 x 40000 pairs (tiles %s)" % (r.get_tiling(),), P)
    assert np.array_equal(keys.cpu().numpy(), ref["keys"])
    assert np.array_equal(pids.cpu().numpy(), ref["pids"])
    assert np.array_equal(ts.cpu().numpy(), ref["tile_start"])


def test_config0_brightfield_parity():
    fr = workloads.config0()
    opd, I = gpu_frame(fr)
    ropd, rI = oracle_frame(fr)
    e_opd = float(np.max(np.abs(opd - ropd)))
    e_I = rel_l2(I, rI)
    say("config0 256^2 BF: OPD max abs %.3e um, I rel L2 %.3e" % (e_opd, e_I))
    assert e_opd <= OPD_TOL and e_I <= I_TOL


@pytest.mark.parametrize("mode,size,n", [(workloads.DIC, 512, 2000), (workloads.OBLIQUE, 512, 2000),
                                         (workloads.BRIGHTFIELD, 1024, 3000), (workloads.DIC, 256, 700),
                                         (workloads.OBLIQUE, 2048, 5000)])
def test_mid_parity(mode, size, n):
    fr = mid_frame(11 + mode, size, n, mode)
    opd, I = gpu_frame(fr)
    ropd, rI = oracle_frame(fr)
    e_opd = float(np.max(np.abs(opd - ropd)))
    e_I = rel_l2(I, rI)
    say("mode %d %d^2 n=%d: OPD max abs %.3e, I rel L2 %.3e" % (mode, size, n, e_opd, e_I))
    assert e_opd <= OPD_TOL and e_I <= I_TOL


def test_config1_full_size_parity_noiseless():
    fr = workloads.config1(photons=0.0)
    opd, I = gpu_frame(fr)
    ropd, rI = oracle_frame(fr)
    e_opd = float(np.max(np.abs(opd - ropd)))
    e_I = rel_l2(I, rI)
    say("config1 2048^2 x 40000 DIC: OPD max abs %.3e um, I rel L2 %.3e" % (e_opd, e_I))
    assert e_opd <= OPD_TOL and e_I <= I_TOL


def test_deterministic_and_tiling_invariant():
    r = R()
    fr = mid_frame(5, 512, 3000, workloads.DIC)
    a_opd, a_I = gpu_frame(fr)
    b_opd, b_I = gpu_frame(fr)
    assert np.array_equal(a_opd, b_opd) and np.array_equal(a_I, b_I)
    th0, tw0 = r.get_tiling()
    for tl in [(16, 16), (8, 32), (32, 8), (64, 4), (32, 32), (32, 16), (4, 256)]:
        r.set_tiling(*tl)
        try:
            c_opd, c_I = gpu_frame(fr)
        finally:
            r.set_tiling(th0, tw0)
        assert np.array_equal(a_opd, c_opd), tl
        assert np.array_equal(a_I, c_I), tl


def test_pair_overflow_fallback_is_bitwise_identical():
    r = R()
    fr = mid_frame(6, 256, 600, workloads.BRIGHTFIELD)
    soa, g = dev_soa(fr.soa), dev_globals(fr.globals4)
    I1, o1 = r.render(soa, 256, 256, fr.optics, g, want_opd=True)
    small = torch.empty(r.workspace_size(256, 256, 600, pairs_per_particle=1), dtype=torch.uint8, device="cuda")
    I2, o2 = r.render(soa, 256, 256, fr.optics, g, want_opd=True, workspace=small)
    torch.cuda.synchronize()
    assert torch.equal(o1, o2) and torch.equal(I1, I2)


def crowded_frame(seed=11):
    """256^2 brightfield frame whose particles crowd into a few tiles: 700 small
    prisms and ellipsoids in a 48x48 px patch (16x16 tiles of 65-512 particles:
    the LDS sort, rows split into parts) and 700 more centred in one 16x16 tile
    (a segment of more than 512 ids: the id-ordered scan, also in parts)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    a = workloads.mixed(rng, 700, 256, 256)
    a[0] = rng.uniform(100, 148, 700)
    a[1] = rng.uniform(60, 108, 700)
    a[3] = rng.uniform(1.5, 4, 700)
    a[4] = np.where(a[7] > 0.5, rng.uniform(1.5, 4, 700), a[3])
    b = workloads.mixed(rng, 700, 256, 256)
    b[0] = rng.uniform(200, 208, 700)
    b[1] = rng.uniform(200, 208, 700)
    b[3] = rng.uniform(1, 3, 700)
    b[4] = np.where(b[7] > 0.5, rng.uniform(1, 3, 700), b[3])
    soa = workloads.f32(np.concatenate([a, b], axis=1))
    opt = workloads.OpticsSpec(mode=workloads.BRIGHTFIELD, na=0.4)
    return workloads.Frame(256, 256, soa, opt, np.array([1.0, 0, 0, 0], np.float32), "crowded")


def test_crowded_tiles_sorted_and_scanned_paths():
    r = R()
    fr = crowded_frame()
    soa, g = dev_soa(fr.soa), dev_globals(fr.globals4)
    th0, tw0 = r.get_tiling()
    r.set_tiling(16, 16)  # the frame's crowding is laid out for 16 x 16 tiles
    try:
        keys, pids, ts, counts, P = r.bin_pairs(soa, fr.H, fr.W)
    finally:
        r.set_tiling(th0, tw0)
    ref = oracle.binning.bin_pairs(fr.soa, fr.H, fr.W, 16, 16)
    per_tile = np.diff(ref["tile_start"])
    say("crowded: pairs %d, max per tile %d, tiles over 64: %d, over 512: %d" % (
        P, per_tile.max(), (per_tile > 64).sum(), (per_tile > 512).sum()))
    assert ((per_tile > 64) & (per_tile <= 512)).sum() > 0 and (per_tile > 512).sum() > 0
    assert P == len(ref["keys"])
    assert np.array_equal(keys.cpu().numpy(), ref["keys"])
    assert np.array_equal(pids.cpu().numpy(), ref["pids"])
    assert np.array_equal(ts.cpu().numpy(), ref["tile_start"])
    r.set_tiling(16, 16)
    try:
        I, opd = r.render(soa, fr.H, fr.W, fr.optics, g, want_opd=True)
        torch.cuda.synchronize()
    finally:
        r.set_tiling(th0, tw0)
    ref_opd = oracle.raster.opd(fr.soa, fr.H, fr.W)
    e = float(np.abs(opd.cpu().numpy() - ref_opd).max())
    ref_I = oracle.optics.intensity(ref_opd, oracle_optics(fr.optics), 1.0, 0.0, 0.0)
    e_i = rel_l2(I.cpu().numpy(), ref_I)
    say("crowded: OPD max abs %.3e um, I rel L2 %.3e" % (e, e_i))
    assert e <= 1e-5 and e_i <= 1e-4
    # tilings whose tiles hold everything differently (other sorted, scanned and
    # row-split tiles) must give the same canvas
    for tl in [(8, 32), (32, 16), (32, 32)]:
        r.set_tiling(*tl)
        try:
            I2, opd2 = r.render(soa, fr.H, fr.W, fr.optics, g, want_opd=True)
            torch.cuda.synchronize()
        finally:
            r.set_tiling(th0, tw0)
        assert torch.equal(opd, opd2) and torch.equal(I, I2), tl


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_empty_canvas(mode):
    r = R()
    th = 1.1
    opt = workloads.OpticsSpec(mode=mode, na=0.5, shear_angle_rad=math.pi / 4, tilt_fx=0.27)
    soa = torch.zeros((8, 0), dtype=torch.float32, device="cuda")
    I, opd = r.render(soa, 128, 64, opt, dev_globals([0.7, 1.0, th, 0]), want_opd=True)
    torch.cuda.synchronize()
    expect = {0: 1.0, 1: 4 * math.sin(th) ** 2, 2: 1.0}[mode]
    assert float(opd.abs().max()) == 0.0
    assert float((I - expect).abs().max()) < 1e-5


def test_full_pupil_in_focus_is_unity():
    r = R()
    fr = mid_frame(7, 256, 400, workloads.BRIGHTFIELD)
    opt = workloads.OpticsSpec(mode=0, na=0.4, pixel_um=1.0)
    I = r.render(dev_soa(fr.soa), 256, 256, opt, dev_globals([0, 0, 0, 0]))
    torch.cuda.synchronize()
    assert float((I - 1).abs().max()) < 2e-5


def test_dic_integer_shear_closed_form():
    # full pupil, in focus, total shear 2 px along x: I = 2 - 2 cos(phi(x+1) - phi(x-1) + 2 theta)
    r = R()
    fr = mid_frame(8, 128, 150, workloads.BRIGHTFIELD)
    opt = workloads.OpticsSpec(mode=1, na=0.4, pixel_um=1.0, shear_angle_rad=0.0)
    th = 0.3
    I, opd = r.render(dev_soa(fr.soa), 128, 128, opt, dev_globals([0, 2.0, th, 0]), want_opd=True)
    torch.cuda.synchronize()
    phi = 2 * math.pi / 0.55 * opd.cpu().double().numpy()
    ref = 2 - 2 * np.cos(np.roll(phi, -1, 1) - np.roll(phi, 1, 1) + 2 * th)
    assert np.max(np.abs(I.cpu().numpy() - ref)) < 1e-4


def test_fft_chain_matches_rocfft():
    # The same OPD through torch.fft (rocFFT) in FP32 vs the library's fused chain.
    r = R()
    fr = mid_frame(9, 1024, 4000, workloads.DIC)
    soa, g = dev_soa(fr.soa), dev_globals(fr.globals4)
    I, opd = r.render(soa, 1024, 1024, fr.optics, g, want_opd=True)
    Hf = torch.from_numpy(oracle.optics.transfer(1024, 1024, oracle_optics(fr.optics),
                                                 *fr.globals4[:3].astype(np.float64))).to(torch.complex64).cuda()
    U = torch.polar(torch.ones_like(opd), (2 * math.pi / 0.55) * opd)
    E = torch.fft.ifft2(torch.fft.fft2(U) * Hf)
    ref = (E.real ** 2 + E.imag ** 2)
    torch.cuda.synchronize()
    e = rel_l2(I.cpu().numpy(), ref.cpu().numpy())
    say("vs rocFFT chain: rel L2 %.3e" % e)
    assert e < 2e-5


def test_philox_bit_exact():
    r = R()
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, size=(4096, 4), dtype=np.uint64).astype(np.uint32)
    k0, k1 = 0x12345678, 0x9ABCDEF0
    out = r.philox(torch.from_numpy(ctr.view(np.int32)).cuda(), k0, k1).cpu().numpy().view(np.uint32)
    ref = np.stack(oracle.noise.philox4x32_10_np(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], k0, k1), 1)
    assert np.array_equal(out, ref)


def test_noise_statistics_and_oracle_counts():
    r = R()
    # uniform DIC background (I = 4 at theta = pi/2): s = 1000/4
    opt = workloads.OpticsSpec(mode=1, na=0.5, shear_angle_rad=math.pi / 4, photons_mean=1000.0, seed=77)
    soa = torch.zeros((8, 0), dtype=torch.float32, device="cuda")
    I = r.render(soa, 512, 512, opt, dev_globals([0.3, 1.0, math.pi / 2, 0])).cpu().double().numpy()
    z = (I * 250.0 - 1000.0) / math.sqrt(1000.0)
    n = z.size
    assert abs(z.mean()) < 4 / math.sqrt(n) and abs(z.var() - 1) < 0.02
    assert np.all(np.abs(I * 250.0 - np.round(I * 250.0)) < 1e-3)
    # counts against the oracle's sampler on a structured frame
    fr = mid_frame(10, 64, 30, workloads.DIC)
    fr.optics = replace(fr.optics, photons_mean=1000.0, seed=5)
    Ig = r.render(dev_soa(fr.soa), 64, 64, fr.optics, dev_globals(fr.globals4)).cpu().double().numpy()
    _, clean = oracle_frame(fr)
    ref = oracle.noise.add_noise(clean, 1000.0, 5)
    s = 1000.0 / clean.mean()
    same = np.mean(np.round(Ig * s) == np.round(ref * s))
    say("noise: counts identical to the oracle's on %.4f of pixels" % same)
    assert same > 0.98


def test_radix4_plan_and_autotuner():
    r = R()
    from paper_2606_21381_amd import autotune, render
    fr = mid_frame(12, 512, 2000, workloads.DIC)
    soa, g = dev_soa(fr.soa), dev_globals(fr.globals4)
    ropd, rI = oracle_frame(fr)
    lib = render._lib.load()
    render._lib.check(lib.osog_set_size_radix(render.context(), 512, 512, 4), "radix")
    I4 = render.render(soa, 512, 512, fr.optics, g)
    torch.cuda.synchronize()
    e4 = rel_l2(I4.cpu().numpy(), rI)
    choice = autotune.tune_frame(soa, 512, 512, fr.optics, g, reps=2)
    I = render.render(soa, 512, 512, fr.optics, g)
    torch.cuda.synchronize()
    e = rel_l2(I.cpu().numpy(), rI)
    say("radix-4 plan rel L2 %.2e; autotuner chose %s, rel L2 %.2e" % (e4, choice, e))
    assert e4 <= I_TOL and e <= I_TOL
    assert (choice["tile_h"], choice["tile_w"]) in [(16, 16), (32, 32), (32, 16), (16, 32), (64, 16)]
    assert choice["fft_radix"] in (4, 8)
    # back to the defaults for the other tests
    render._lib.check(lib.osog_set_size_tiling(render.context(), 512, 512, *render.get_tiling()), "tiling")
    render._lib.check(lib.osog_set_size_radix(render.context(), 512, 512, 8), "radix")
