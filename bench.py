"""Benchmark: frames/s of the full forward path on 2048x2048 DIC frames with
40,000 particles (half prisms, half ellipsoids), Poisson noise at 1000 photons/px.

One step = one complete frame through every stage (binning, rasterisation,
row FFT, column FFT with the transfer function, row IFFT with |E|^2 and noise),
with the particle table already resident in HBM.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3   # MI355X FP32 vector peak (packed); scalar-issue FP32 FMA peaks at half
# Algorithmic FP32 operations of the raster per unit of work (an FMA counts 2): a candidate
# pixel test -- a pixel of a particle's conservative binning box, which any exact per-pixel
# method must classify -- 20 (centre offsets, rotation, edge distances, classification, the
# thickness, the add); an exact clip of a prism boundary pixel (the box-filtered area where an
# edge crosses the pixel) 80.  The 2048^2 x 40k frame has 19.2 M tests and 1.5 M clips: 0.50 GFLOP.
RASTER_FLOP_PER_TEST = 20.0
RASTER_FLOP_PER_CLIP = 80.0
HBM_TARGET_FRAC = 0.6      # the frame's target share of the HBM roofline
METRIC = "frames/s at 2048²×40k-particle DIC"


def algorithmic_bytes(H, W, n, P, kx_n):
    """Bytes each stage must move at minimum (one read of its inputs, one write
    of its outputs), per frame."""
    hw4 = 4.0 * H * W
    band = 8.0 * H * kx_n
    return {
        # SoA table read, per-particle pair counts, the pair list (one 4-byte id per
        # pair, written once), per-tile count / first / end
        "binning": 32.0 * n + 4.0 * n + 4.0 * P + 12.0 * (H * W / 256),
        # pair list + the 8 attributes of each listed particle, OPD written once
        "raster": 4.0 * P + 32.0 * P + hw4,
        "pass1": hw4 + band,
        "pass2": 2.0 * band,
        "pass3": band + hw4,
    }


COUNTERS = os.path.join(ROOT, "profiles", "counters_dic2048_n40000.txt")


def raster_work(soa, H, W):
    """Units of the raster's algorithmic work: (candidate pixel tests, prism boundary
    clips).  Tests: the canvas pixels of each particle's conservative binning box
    (ext = max(a, b) sqrt 2 + 1 for a prism, max(a, b) + 1 for an ellipsoid).  Clips:
    the pixels a prism's four edges cross, 4 (a + b) (|cos| + |sin|) on average for a
    rectangle of half-widths a, b (perimeter 4 (a + b)) at a uniform sub-pixel offset."""
    cx, cy, ang, a, b = (soa[k].astype(np.float64) for k in range(5))
    prism = soa[7] < 0.5
    ext = np.where(prism, np.maximum(a, b) * math.sqrt(2.0) + 1.0, np.maximum(a, b) + 1.0)
    nx = np.clip(np.floor(cx + ext), 0, W - 1) - np.clip(np.floor(cx - ext), 0, W - 1) + 1
    ny = np.clip(np.floor(cy + ext), 0, H - 1) - np.clip(np.floor(cy - ext), 0, H - 1) + 1
    tests = float((nx * ny).sum())
    clips = float((4.0 * (a + b) * (np.abs(np.cos(ang)) + np.abs(np.sin(ang))))[prism].sum())
    return tests, clips


def host_cpu():
    """(model name, logical cores) of the host running the oracle."""
    name = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                name = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return name, os.cpu_count()


def kernel_hash():
    """sha1 of the built library, whose device code is what a counter summary measured
    (comment-only source edits leave it unchanged)."""
    import hashlib
    with open(os.path.join(ROOT, "paper_2606_21381_amd", "lib", "libosog.so"), "rb") as fh:
        return hashlib.sha1(fh.read()).hexdigest()


def measured_counters(kernel):
    """HBM bytes (scaled FETCH_SIZE + WRITE_SIZE) and VALU busy share of `kernel`
    from the committed rocprofv3 counter summary, or None when that summary was
    taken on another build of the library than the one loaded now."""
    try:
        lines = open(COUNTERS).read().splitlines()
    except OSError:
        return None
    stamp = [l for l in lines if l.startswith("# kernel library: sha1 ")]
    if not stamp or stamp[0].split()[4] != kernel_hash():
        return None
    head = [l.split() for l in lines if l.startswith("kernel ")]
    if not head:
        return None
    cols = head[0][1:]
    for l in lines:
        f = l.split()
        if not f or l.startswith("#") or l.startswith("kernel ") or len(f) <= len(cols):
            continue
        # the kernel name may contain spaces ("k_pass1<11, 8>"): the numbers are the last fields
        name = " ".join(f[:-len(cols)])
        # a whole name, or a prefix that does not stop inside an identifier ("k_bin" is
        # not "k_bin_clear"; "k_pass1<11" is "k_pass1<11, 8>")
        nxt = name[len(kernel):len(kernel) + 1]
        if name.startswith(kernel) and not (nxt.isalnum() or nxt == "_"):
            v = dict(zip(cols, map(float, f[-len(cols):])))
            return {"traffic": v["total_MB"] * 1e6, "fetch": v["fetch_MB"] * 1e6, "write": v["write_MB"] * 1e6,
                    "valu_winst": v["valu_winst"], "valu_busy": v["valu%"] / 100.0}
    return None


def frame_kernels(logW=11, radix=8):
    """Kernel names of one forward frame (no habits, no absorption) for a plan."""
    fft = "<%d, %d>" % (logW, radix)
    return ("k_bin_clear", "k_bin", "k_tile_scan", "k_emit", "k_raster<false, false>", "k_pass1" + fft,
            "k_pass2" + fft, "k_pass3" + fft)


def frame_valu_floor_us(logW=11, radix=8):
    """Time the headline frame's kernels need at the chip's full VALU issue rate (their
    wave instructions x 4 cycles over 1024 SIMDs at 2.4 GHz), from the committed counter
    summary; None when that summary belongs to another build of the library."""
    frame = frame_kernels(logW, radix)
    try:
        lines = open(COUNTERS).read().splitlines()
    except OSError:
        return None
    stamp = [l for l in lines if l.startswith("# kernel library: sha1 ")]
    head = [l.split() for l in lines if l.startswith("kernel ")]
    if not stamp or stamp[0].split()[4] != kernel_hash() or not head:
        return None
    cols = head[0][1:]
    winst = {}
    for l in lines:
        f = l.split()
        if f and not l.startswith("#") and not l.startswith("kernel ") and len(f) > len(cols):
            winst[" ".join(f[:-len(cols)])] = dict(zip(cols, map(float, f[-len(cols):])))["valu_winst"]
    if not all(k in winst for k in frame):
        return None
    return sum(winst[k] for k in frame) * 4.0 / (1024 * 2.4e3)


def cpu_baseline(fr, budget_s=20.0):
    """The FP64 oracle on a bounded sample of the same workload, scaled to frames/s.

    Sample: one full noiseless frame (binning is not part of the oracle's
    definition; it rasterises every particle directly) plus the shot noise of a
    contiguous run of pixels, extrapolated to the frame's 2048^2 pixels.
    """
    import oracle
    t0 = time.perf_counter()
    opd = oracle.raster.opd(fr.soa, fr.H, fr.W)
    g = fr.globals4.astype(np.float64)
    o = oracle.Optics(mode=fr.optics.mode, na=fr.optics.na, shear_angle_rad=fr.optics.shear_angle_rad,
                      wavelength_um=fr.optics.wavelength_um, n_medium=fr.optics.n_medium,
                      pixel_um=fr.optics.pixel_um)
    I = oracle.optics.intensity(opd, o, g[0], g[1], g[2])
    t_render = time.perf_counter() - t0
    s = fr.optics.photons_mean / I.mean()
    flat = I.reshape(-1)
    t1 = time.perf_counter()
    m = 0
    while time.perf_counter() - t1 < max(1.0, budget_s - t_render) and m < flat.size:
        for p in range(m, min(m + 4096, flat.size)):
            oracle.noise.poisson_one(s * flat[p], p, 0, fr.optics.seed)
        m = min(m + 4096, flat.size)
    t_noise = (time.perf_counter() - t1) * flat.size / m
    per_frame = t_render + t_noise
    cpu, ncpu = host_cpu()
    return {"value": 1.0 / per_frame, "unit": "frames/s", "cores": 1, "kind": "oracle",
            "host_cpu": cpu, "host_logical_cores": ncpu,
            "sample": "1 full noiseless 2048^2 x 40k DIC frame (%.2f s) + Poisson noise of %d pixels "
                      "extrapolated to %d (%.1f s/frame)" % (t_render, m, flat.size, t_noise)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-steps", type=int, default=50)
    ap.add_argument("--no-extras", action="store_true", help="skip the backward, batch and inverse-solve legs")
    ap.add_argument("--legs", default="fft_vs_rocfft,multimodal,variants,backward,batch,stream,inverse",
                    help="comma-separated extra legs to run (default: all)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="after the timed run, one plain device-to-device copy of this many MiB "
                         "(reference dispatch for hardware byte counters)")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip training the learned initializer (600,000 rendered crops) and its comparison of "
                         "inverse solves (part of the inverse leg by default)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build runs on a single MI355X with no sharding "
              "or collectives (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2606_21381_amd import _lib, render, workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    fr = workloads.config1()
    H, W, n = fr.H, fr.W, fr.soa.shape[1]
    soa = torch.from_numpy(fr.soa).to(dev)
    g = torch.from_numpy(fr.globals4).to(dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    ws = torch.empty(render.workspace_size(H, W, n), dtype=torch.uint8, device=dev)

    def step():
        render.render(soa, H, W, fr.optics, g, out=out, workspace=ws)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    ev[0].record()
    for k in range(args.steps):
        step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = ev[0].elapsed_time(ev[-1]) / args.steps
    step_ms = np.array([ev[k].elapsed_time(ev[k + 1]) for k in range(args.steps)])

    # per-stage durations with HIP events on the launch stream (separate run)
    lib = _lib.load()
    ctx = render.context(dev)
    _lib.check(lib.osog_profile_enable(ctx, 1), "profile_enable")
    for _ in range(args.profile_steps):
        step()
    import ctypes
    st_ms = (ctypes.c_double * 10)()
    st_n = (ctypes.c_int64 * 10)()
    _lib.check(lib.osog_profile_read(ctx, st_ms, st_n), "profile_read")
    _lib.check(lib.osog_profile_enable(ctx, 0), "profile_disable")
    stage_us = {_lib.STAGES[k]: 1000.0 * st_ms[k] / st_n[k] for k in range(10) if st_n[k]}

    _, _, _, _, P = render.bin_pairs(soa, H, W)
    from paper_2606_21381_amd.render import band_columns
    kx_n = band_columns(H, W, fr.optics)
    alg = algorithmic_bytes(H, W, n, P, kx_n)
    dom = max((k for k in stage_us if k in alg), key=lambda k: stage_us[k])
    achieved = alg[dom] / (stage_us[dom] * 1e-6) / 1e9
    kname = {"binning": "k_bin", "raster": "k_raster", "pass1": "k_pass1", "pass2": "k_pass2",
             "pass3": "k_pass3"}[dom]
    cnt = measured_counters(kname)
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": round(cnt["traffic"]) if cnt else None,
            "algorithmic_bytes": alg[dom], "avg_us": round(stage_us[dom], 2),
            "valu_busy": round(cnt["valu_busy"], 3) if cnt else None}
    if dom == "raster":
        # the raster's time is set by its arithmetic pipeline, not by HBM: its roofline is FP32
        # arithmetic
        tests, clips = raster_work(fr.soa, H, W)
        flops = tests * RASTER_FLOP_PER_TEST + clips * RASTER_FLOP_PER_CLIP
        tflops = flops / (stage_us[dom] * 1e-6) / 1e12
        roof = {"bound": "alu", "kernel": dom, "achieved": round(tflops, 3), "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(tflops / FP32_PEAK_TFLOPS, 4),
                "traffic": round(cnt["traffic"]) if cnt else None,
                "algorithmic_flops": flops, "units": {"candidate_pixel_tests": tests, "prism_boundary_clips": clips,
                                                      "flop_per_test": RASTER_FLOP_PER_TEST,
                                                      "flop_per_clip": RASTER_FLOP_PER_CLIP},
                "avg_us": round(stage_us[dom], 2), "valu_busy": round(cnt["valu_busy"], 3) if cnt else None,
                "hbm_frac": round(achieved / HBM_PEAK_GBS, 4), "algorithmic_bytes": alg[dom]}
    total_alg = sum(alg.values())
    th, tw = render.get_tiling(dev)
    vf = frame_valu_floor_us(int(round(math.log2(W))), 8)
    res = {
        "metric": METRIC,
        "value": round(1000.0 / ms, 2),
        "unit": "frames/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded particle tables)",
        "config": {"workload": "dic2048_n40000", "height": H, "width": W, "particles": n,
                   "prisms": int((fr.soa[7] < 0.5).sum()), "mode": "DIC", "na": fr.optics.na,
                   "photons_mean": fr.optics.photons_mean, "pairs": P, "band_columns": kx_n},
        "particles_per_s": round(n * 1000.0 / ms, 1),
        "step_ms": {"mean": round(float(step_ms.mean()), 4), "std": round(float(step_ms.std()), 4),
                    "p50": round(float(np.percentile(step_ms, 50)), 4),
                    "p99": round(float(np.percentile(step_ms, 99)), 4)},
        "tiling": [th, tw],
        "stage_us": {k: round(v, 2) for k, v in stage_us.items()},
        "frame_alg_bytes": total_alg,
        "frame_alg_gbs": round(total_alg / (ms * 1e-3) / 1e9, 1),
        "frame_hbm_frac": round(total_alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "frame_hbm_target_frac": HBM_TARGET_FRAC,
        "frame_us_at_target": round(total_alg / (HBM_TARGET_FRAC * HBM_PEAK_GBS * 1e9) * 1e6, 2),
        # a floor from vector issue alone: the frame's kernels' VALU instructions at the full
        # issue rate, and that floor as a share of the measured frame time
        "frame_valu_floor_us": round(vf, 1) if vf else None,
        "frame_valu_frac": round(vf / (ms * 1e3), 4) if vf else None,
        "roofline": roof,
        "paper_context": "paper: 40,000 particles in under 50 ms on one NVIDIA A100 (1024^2 canvas)",
    }
    if not args.no_extras:
        legs = set(args.legs.split(","))
        progress("headline frame done: %.4f ms per frame" % ms)
        if "fft_vs_rocfft" in legs:
            res["fft_vs_rocfft"] = bench_fft_vs_rocfft(render, lib, ctx, soa, fr, g, dev)
            progress("leg fft_vs_rocfft done")
        if "multimodal" in legs:
            res["multimodal"] = bench_multimodal(render, soa, fr, dev)
            progress("leg multimodal done")
        if "variants" in legs:
            res["variants"] = bench_variants(render, fr, g, dev)
            progress("leg variants done")
        if "backward" in legs:
            res["backward"] = bench_backward(render, soa, g, fr, dev)
            progress("leg backward done")
        if "batch" in legs:
            res["batch"] = bench_batch(render, dev)
            progress("leg batch done")
        if "stream" in legs:
            res["stream"] = bench_stream(render, fr, dev)
            progress("leg stream done")
        if "inverse" in legs:
            res["inverse"] = bench_inverse(dev, learned=not args.no_learned)
            progress("leg inverse done")
    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        res["calib_copy_bytes"] = nb
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(fr)
    print(json.dumps(res), flush=True)


def bench_fft_vs_rocfft(render, lib, ctx, soa, fr, g, dev, reps=50):
    """The imaging chain of a noiseless headline frame (passes 1-3: exp(i k OPD), banded
    row DFT, column DFT x transfer x inverse column DFT, inverse row DFT, |E|^2) against
    the same chain through torch.fft (rocFFT): exp(i k OPD), dense FFT2, multiply by a
    full-grid transfer array, IFFT2, |E|^2.  The transfer values do not change the
    library FFT's time, so a unit-modulus array stands in for them here (the numerics of
    the two chains are compared in the forward tests)."""
    import ctypes
    from dataclasses import replace

    import torch
    from paper_2606_21381_amd import _lib
    H, W = fr.H, fr.W
    opt0 = replace(fr.optics, photons_mean=0.0)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    _, opd = render.render(soa, H, W, opt0, g, want_opd=True)
    for _ in range(5):
        render.render(soa, H, W, opt0, g, out=out)
    torch.cuda.synchronize()
    _lib.check(lib.osog_profile_enable(ctx, 1), "profile_enable")
    for _ in range(reps):
        render.render(soa, H, W, opt0, g, out=out)
    st_ms = (ctypes.c_double * 10)()
    st_n = (ctypes.c_int64 * 10)()
    _lib.check(lib.osog_profile_read(ctx, st_ms, st_n), "profile_read")
    _lib.check(lib.osog_profile_enable(ctx, 0), "profile_disable")
    us = {_lib.STAGES[k]: 1000.0 * st_ms[k] / st_n[k] for k in range(5) if st_n[k]}
    chain_us = us["pass1"] + us["pass2"] + us["pass3"]
    k = 2.0 * math.pi / fr.optics.wavelength_um
    gen = torch.Generator(device=dev)
    gen.manual_seed(5)
    Hf = torch.polar(torch.ones((H, W), device=dev),
                     (2.0 * math.pi) * torch.rand((H, W), device=dev, generator=gen))

    def chain():
        E = torch.fft.ifft2(torch.fft.fft2(torch.polar(torch.ones_like(opd), k * opd)) * Hf)
        return E.real * E.real + E.imag * E.imag

    for _ in range(5):
        chain()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        chain()
    e1.record()
    torch.cuda.synchronize()
    roc_us = 1000.0 * e0.elapsed_time(e1) / reps
    return {"workload": "dic2048_n40000 noiseless imaging chain", "library_passes_us": round(chain_us, 2),
            "library_stage_us": {k2: round(us[k2], 2) for k2 in ("pass1", "pass2", "pass3")},
            "rocfft_chain_us": round(roc_us, 2), "speedup": round(roc_us / chain_us, 2)}


def bench_multimodal(render, soa, fr, dev, reps=20):
    """Brightfield, DIC (with the frame's noise) and oblique images of the headline
    particle table: one osog_render_multi call against three osog_render calls."""
    import torch
    from paper_2606_21381_amd import workloads
    opts = [workloads.OpticsSpec(mode=workloads.BRIGHTFIELD, na=0.5), fr.optics,
            workloads.OpticsSpec(mode=workloads.OBLIQUE, na=0.5, tilt_fx=0.3 * 0.5 / 0.55)]
    g = torch.tensor([[float(fr.globals4[0]), 0, 0, 0], list(map(float, fr.globals4)),
                      [float(fr.globals4[0]), 0, 0, 0]], dtype=torch.float32, device=dev)
    outs = [torch.empty((fr.H, fr.W), dtype=torch.float32, device=dev) for _ in opts]

    def multi():
        render.render_multi(soa, fr.H, fr.W, opts, g, out=outs)

    def singles():
        for k, o in enumerate(opts):
            render.render(soa, fr.H, fr.W, o, g[k], out=outs[k])

    res = {}
    for name, fn in (("multi", multi), ("three_singles", singles)):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        res[name + "_ms"] = round(e0.elapsed_time(e1) / reps, 4)
    res["workload"] = "dic2048_n40000 as brightfield + DIC + oblique"
    res["images_per_s"] = round(3000.0 / res["multi_ms"], 1)
    return res


def bench_variants(render, fr, g, dev, reps=20):
    """The headline frame with Beer-Lambert absorption (a seeded dmu row), as Eq. 5's
    literal (incoherent) DIC, and with a third of its particles as polyhedral habits:
    ms per frame of each, with the frame's noise."""
    import numpy as np
    import torch
    from dataclasses import replace
    from paper_2606_21381_amd import workloads
    rng = np.random.Generator(np.random.PCG64(11))
    soa8 = torch.from_numpy(fr.soa).to(dev)
    soa9 = torch.from_numpy(workloads.f32(workloads.with_absorption(rng, fr.soa.astype(np.float64)))).to(dev)
    # a third of the particles as polyhedral habits (octahedra, tetragonal bipyramids, one with topography)
    hab = fr.soa.astype(np.float64).copy()
    sel = rng.permutation(hab.shape[1])[: hab.shape[1] // 3]
    hab[:, sel] = workloads.habits_table(rng, sel.size, fr.H, fr.W, 3)
    soa_h = torch.from_numpy(workloads.f32(hab)).to(dev)
    habits = [workloads.habit_octahedron(), workloads.habit_tetragonal(0.5),
              workloads.habit_tetragonal(0.3, topo_amplitude_um=0.15, topo_cell_px=4.0)]
    frc = workloads.config1_clustered()
    soa_c = torch.from_numpy(frc.soa).to(dev)
    cases = {"absorbing_dic": (soa9, replace(fr.optics, absorption=1)),
             "incoherent_dic": (soa8, replace(fr.optics, mode=workloads.DIC_INCOHERENT)),
             "habits_dic": (soa_h, fr.optics),
             "uniform_dic": (soa8, fr.optics),
             "clustered_dic": (soa_c, frc.optics)}
    res = {"workload": "dic2048_n40000 (absorbing: dmu ~ U[0, 0.4] 1/um; habits: a third of the particles "
                       "as octahedra / tetragonal bipyramids, one habit with micro-topography; clustered: the "
                       "40,000 centres in 64 Gaussian clusters of sigma 25 px)"}
    for name, (s, o) in cases.items():
        if name == "habits_dic":
            render.set_habits(habits, 7)
        out = torch.empty((fr.H, fr.W), dtype=torch.float32, device=dev)
        ws = torch.empty(render.workspace_size(fr.H, fr.W, fr.soa.shape[1], o.mode == workloads.DIC_INCOHERENT),
                         dtype=torch.uint8, device=dev)
        for _ in range(3):
            render.render(s, fr.H, fr.W, o, g, out=out, workspace=ws)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            render.render(s, fr.H, fr.W, o, g, out=out, workspace=ws)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms_per_frame": round(ms, 4), "frames_per_s": round(1000.0 / ms, 1)}
        if name in ("uniform_dic", "clustered_dic"):  # per-stage times: does crowding slow the raster?
            import ctypes
            from paper_2606_21381_amd import _lib
            lib, ctx = _lib.load(), render.context(dev)
            _lib.check(lib.osog_profile_enable(ctx, 1), "profile_enable")
            for _ in range(reps):
                render.render(s, fr.H, fr.W, o, g, out=out, workspace=ws)
            st_ms, st_n = (ctypes.c_double * 10)(), (ctypes.c_int64 * 10)()
            _lib.check(lib.osog_profile_read(ctx, st_ms, st_n), "profile_read")
            _lib.check(lib.osog_profile_enable(ctx, 0), "profile_disable")
            res[name]["stage_us"] = {_lib.STAGES[k]: round(1000.0 * st_ms[k] / st_n[k], 2) for k in range(5) if st_n[k]}
        if name == "habits_dic":
            render.set_habits([], 0)
    return res


def bench_backward(render, soa, g, fr, dev, reps=20):
    """ms per adjoint call (forward recompute + adjoint) at the headline frame."""
    import torch
    gi = torch.randn(fr.H, fr.W, device=dev)
    for _ in range(3):
        render.render_backward(soa, fr.H, fr.W, fr.optics, g, gi)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        render.render_backward(soa, fr.H, fr.W, fr.optics, g, gi)
    e1.record()
    torch.cuda.synchronize()
    return {"ms_per_backward": round(e0.elapsed_time(e1) / reps, 4), "workload": "dic2048_n40000"}


def bench_batch(render, dev, reps=10):
    """64 frames of 512/1024/2048^2, 100..40000 particles, DIC + oblique, one HIP graph launch."""
    import torch
    from paper_2606_21381_amd import autotune, workloads
    frs = workloads.config2()
    fr = [(torch.from_numpy(x.soa).to(dev), x.H, x.W, x.optics, torch.from_numpy(x.globals4).to(dev)) for x in frs]
    # autotune one representative frame per canvas size (largest particle count of that size)
    reps_by_size = {}
    for x, f in zip(frs, fr):
        k = (x.H, x.W)
        if k not in reps_by_size or f[0].shape[1] > reps_by_size[k][0].shape[1]:
            reps_by_size[k] = (f[0], x.optics, f[4])
    choices = autotune.tune_sizes(reps_by_size, reps=3, device=dev)
    b = render.Batch(fr)
    b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    lats = []
    e0.record()
    for _ in range(reps):
        b.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    for _ in range(3):
        b.run()
        torch.cuda.synchronize()
        lats.append(b.latencies_ms())
    lat = np.concatenate(lats)
    # the tuned plans stay in the context: put the default plan back so that later legs
    # (the stream of headline frames) run the headline frame's plan
    th, tw = render.get_tiling(dev)
    lib, ctx = render._lib.load(), render.context(dev)
    for (hh, ww) in reps_by_size:
        render._lib.check(lib.osog_set_size_tiling(ctx, hh, ww, th, tw), "osog_set_size_tiling")
        render._lib.check(lib.osog_set_size_radix(ctx, hh, ww, 8), "osog_set_size_radix")
    px = sum(x.H * x.W for x in frs)
    parts = sum(x.soa.shape[1] for x in frs)
    return {"workload": "batch64_mixed", "frames": len(frs), "ms_per_batch": round(ms, 4),
            "frames_per_s": round(len(frs) * 1000.0 / ms, 1), "px_per_s": round(px * 1000.0 / ms, 1),
            "particles_per_s": round(parts * 1000.0 / ms, 1),
            "latency_p50_ms": round(float(np.percentile(lat, 50)), 4),
            "latency_p99_ms": round(float(np.percentile(lat, 99)), 4),
            "error_flag": b.error_flag(), "autotune": choices}


def bench_stream(render, fr, dev, frames=8, reps=10):
    """The headline frame rendered as a stream: `frames` copies of it (each with its own
    noise seed) per batch graph launch, so one frame's binning and raster overlap another's
    FFT passes on the concurrent branches.  Reported beside the single-render rate, which
    stays the headline value."""
    import torch
    from dataclasses import replace
    soa = torch.from_numpy(fr.soa).to(dev)
    g = torch.from_numpy(fr.globals4).to(dev)
    items = [(soa, fr.H, fr.W, replace(fr.optics, seed=fr.optics.seed + k), g) for k in range(frames)]
    b = render.Batch(items)
    b.run()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"workload": "dic2048_n40000 x %d per batch launch" % frames, "ms_per_batch": round(ms, 4),
            "frames_per_s": round(frames * 1000.0 / ms, 1), "error_flag": b.error_flag()}


def progress(*parts):
    """One line on stderr when a leg (or one of its targets) is done."""
    print("bench:", *parts, file=sys.stderr, flush=True)


def bench_inverse(dev, learned=True, learned_targets=10, learned_samples=600_000):
    """1024^2 DIC, 500 prisms (seed 3): the hybrid solve (Adam from the perturbed start,
    angles held until the second-order polish); time to e <= 1e-3.  Then, when
    `learned`, the learned initializer trained on engine-rendered crops against the
    default start on `learned_targets` further targets (seeds 300..)."""
    import torch
    from paper_2606_21381_amd import inverse, workloads
    prob = workloads.config3()
    target, start, truth = inverse.problem_tensors(prob, dev)
    inverse.solve(target, inverse.problem_tensors(prob, dev)[1], truth, prob.target.H, prob.target.W,
                  prob.target.optics, inverse.SolverConfig(steps=3))  # warm-up
    res = inverse.solve_hybrid(target, start, truth, prob.target.H, prob.target.W, prob.target.optics)
    a = res.adam
    out = {"workload": "dic1024_n500 (seed 3): Adam %d steps (globals first, angles held) + polish" % a.steps,
           "time_to_1e-3_s": res.time_to_target_s, "glob_time_to_1e-3_s": res.time_to_glob_target_s,
           "final_error": res.final_e, "final_error_glob": res.final_e_glob, "final_error_part": res.final_e_part,
           "final_loss": res.final_loss, "total_s": round(res.total_s, 3),
           "adam_s": round(float(a.time_s[-1]), 3), "adam_steps_per_s": round(len(a.loss) / float(a.time_s[-1]), 1),
           "adam_final_error": float(a.error[-1]),
           "polish_stages": [(tag.split()[0], round(t, 3), float("%.3g" % e)) for tag, t, e, _ in res.trace]}
    if learned:
        from paper_2606_21381_amd import cnn
        def log(k, info):
            if isinstance(info, dict) and "seed" in info:
                progress("learned vs default, target seed %d: fallback %s, time to 1e-3 %s / %s s" % (
                    info["seed"], info["fallback"], info["default"]["time_to_1e-3_s"],
                    info["learned"]["time_to_1e-3_s"]))
            elif k % 500 == 0:
                progress("learned initializer training step", k)

        rep = cnn.compare(dev, samples=learned_samples, n_targets=learned_targets, log=log)
        rep["targets"] = [{"seed": r["seed"], "fallback": r["fallback"],
                           "default": {k: r["default"][k] for k in ("time_to_1e-3_s", "glob_time_to_1e-3_s", "final_e")},
                           "learned": {k: r["learned"][k] for k in ("time_to_1e-3_s", "glob_time_to_1e-3_s", "final_e")}}
                          for r in rep["targets"]]
        out["learned"] = rep
    return out


if __name__ == "__main__":
    main()
