"""GPU adjoint against FP64 central finite differences of the oracle.

Loss L = sum(w * I) for fixed random weights w, so dL/dtheta = <w, dI/dtheta>.
Tolerance (per parameter row): relative error <= 1e-3 on components with
|g| > 1e-3 max|g| of that row, cosine >= 0.99999 over the row; components the
oracle flags as non-smooth (an edge crossing a pixel boundary inside the
stencil) are excluded.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_2606_21381_amd import workloads
from tests.gpu_util import dev_globals, dev_soa, need_gpu, oracle_optics, say

pytestmark = pytest.mark.gpu


def case(seed, n, size, kinds, mode=workloads.DIC):
    rng = np.random.Generator(np.random.PCG64(seed))
    if kinds == "prism":
        s = workloads.prisms(rng, n, size, size)
        s[3] = rng.uniform(3, 12, n)
        s[4] = s[3]
    elif kinds == "ellipsoid":
        s = workloads.ellipsoids(rng, n, size, size)
    else:
        s = workloads.mixed(rng, n, size, size)
    s[0] = rng.uniform(8, size - 8, n)
    s[1] = rng.uniform(8, size - 8, n)
    soa = workloads.f32(s)
    if mode == workloads.DIC:
        opt = workloads.dic_optics(0.0)
        g = np.array([rng.uniform(-2, 2), rng.uniform(0.8, 1.2), (math.pi / 2) * rng.uniform(0.8, 1.2), 0], np.float32)
    elif mode == workloads.OBLIQUE:
        opt = workloads.OpticsSpec(mode=mode, na=0.5, tilt_fx=0.3 * 0.5 / 0.55)
        g = np.array([rng.uniform(-2, 2), 0, 0, 0], np.float32)
    else:
        opt = workloads.OpticsSpec(mode=mode, na=0.4)
        g = np.array([rng.uniform(-2, 2), 0, 0, 0], np.float32)
    w = rng.normal(size=(size, size))
    return soa, opt, g, w


def gpu_grads(soa, opt, g, w, size):
    from paper_2606_21381_amd import render
    gs, gg = render.render_backward(dev_soa(soa), size, size, opt, dev_globals(g),
                                    torch.from_numpy(w.astype(np.float32)).cuda())
    torch.cuda.synchronize()
    return gs.cpu().double().numpy(), gg.cpu().double().numpy()


def compare_row(name, got, ref, flags, rel=1e-3, cos_min=0.99999):
    keep = ~flags
    got, ref = got[keep], ref[keep]
    scale = np.max(np.abs(ref)) if ref.size else 0.0
    if scale == 0.0:
        assert np.max(np.abs(got)) < 1e-6, name
        return 0.0, 1.0
    big = np.abs(ref) > 1e-3 * scale
    err = np.max(np.abs(got[big] - ref[big]) / np.abs(ref[big]))
    cos = float(np.dot(got, ref) / (np.linalg.norm(got) * np.linalg.norm(ref)))
    say("  %-6s max rel err %.2e  cosine %.8f  (%d comps, %d flagged)" % (name, err, cos, big.sum(), (~keep).sum()))
    assert err <= rel and cos >= cos_min, name
    return err, cos


ROWS = ["cx", "cy", "angle", "a", "b", "height", "dn"]


@pytest.mark.parametrize("mode", [workloads.DIC, workloads.BRIGHTFIELD, workloads.OBLIQUE])
def test_prism_gradients_vs_fd_64x64_8_particles(mode):
    need_gpu()
    soa, opt, g, w = case(3 + mode, 8, 64, "prism", mode)
    gs, gg = gpu_grads(soa, opt, g, w, 64)
    rs, rg, fs, fg = oracle.grad.fd_gradients(soa, 64, 64, oracle_optics(opt), g, w)
    say("mode %d, 8 prisms on 64x64" % mode)
    for r, name in enumerate(ROWS):
        if name == "b":   # square prisms: a and b act separately here (half-widths of a rectangle)
            pass
        compare_row(name, gs[r], rs[r], fs[r])
    nglob = 3 if mode == workloads.DIC else 1
    for k in range(nglob):
        e = abs(gg[k] - rg[k]) / max(abs(rg[k]), 1e-12)
        say("  global %d: gpu %.6e fd %.6e rel %.2e" % (k, gg[k], rg[k], e))
        assert e <= 1e-3
    assert gs[7].max() == 0 and gs[7].min() == 0 and gg[3] == 0


def test_ellipsoid_gradients_vs_fd():
    need_gpu()
    soa, opt, g, w = case(21, 6, 64, "ellipsoid")
    gs, gg = gpu_grads(soa, opt, g, w, 64)
    rs, rg, fs, fg = oracle.grad.fd_gradients(soa, 64, 64, oracle_optics(opt), g, w)
    say("DIC, 6 ellipsoids on 64x64 (centre-sampled: 1/sqrt(1-q) near the rim)")
    for r, name in enumerate(ROWS):
        compare_row(name, gs[r], rs[r], fs[r], rel=2e-2, cos_min=0.9999)
    for k in range(3):
        assert abs(gg[k] - rg[k]) / max(abs(rg[k]), 1e-12) <= 1e-3


def test_global_gradients_vs_fd_256():
    need_gpu()
    soa, opt, g, w = case(31, 64, 256, "mixed")
    gs, gg = gpu_grads(soa, opt, g, w, 256)
    rs, rg, fs, fg = oracle.grad.fd_gradients(soa, 256, 256, oracle_optics(opt), g, w, rows=())
    for k in range(3):
        e = abs(gg[k] - rg[k]) / max(abs(rg[k]), 1e-12)
        say("256^2 global %d: gpu %.6e fd %.6e rel %.2e" % (k, gg[k], rg[k], e))
        assert e <= 1e-3


def test_backward_deterministic_and_autograd():
    need_gpu()
    from paper_2606_21381_amd import render
    soa, opt, g, w = case(41, 300, 256, "mixed")
    a = gpu_grads(soa, opt, g, w, 256)
    b = gpu_grads(soa, opt, g, w, 256)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    s = dev_soa(soa).requires_grad_(True)
    gl = dev_globals(g).requires_grad_(True)
    I = render.render_diff(s, gl, 256, 256, opt)
    (I * torch.from_numpy(w.astype(np.float32)).cuda()).sum().backward()
    torch.cuda.synchronize()
    assert np.array_equal(s.grad.cpu().double().numpy(), a[0])
    assert np.array_equal(gl.grad.cpu().double().numpy(), a[1])


@pytest.mark.parametrize("kinds,mode", [("mixed", workloads.DIC), ("mixed", workloads.OBLIQUE)])
def test_dot_product_random_direction(kinds, mode):
    """<J v, w> = <v, J^T w> along one random direction v over every particle
    attribute and the three optical globals at once: J v by FP64 central
    differences of the oracle image, J^T w by the GPU adjoint."""
    need_gpu()
    soa, opt, g, w = case(21 + mode, 10, 64, kinds, mode)
    rng = np.random.Generator(np.random.PCG64(99))
    scale = np.array([1.0, 1.0, 0.1, 1.0, 1.0, 0.3, 0.005])[:, None]  # px, px, rad, px, px, um, 1
    v_soa = rng.uniform(-1, 1, (7, soa.shape[1])) * scale
    v_g = rng.uniform(-1, 1, 3) * np.array([0.3, 0.1, 0.1]) if mode == workloads.DIC else \
        np.array([rng.uniform(-0.3, 0.3), 0.0, 0.0])
    gs, gg = gpu_grads(soa, opt, g, w, 64)
    adj = float(np.sum(gs[:7] * v_soa) + np.dot(gg[:3], v_g))
    o = oracle_optics(opt)
    s64 = soa.astype(np.float64)
    g64 = g.astype(np.float64)
    vals = []
    for eps in (1e-5, 5e-6):
        sp, sm = s64.copy(), s64.copy()
        sp[:7] += eps * v_soa
        sm[:7] -= eps * v_soa
        gp, gm = g64.copy(), g64.copy()
        gp[:3] += eps * v_g
        gm[:3] -= eps * v_g
        vals.append((oracle.grad.loss(sp, 64, 64, o, gp, w) - oracle.grad.loss(sm, 64, 64, o, gm, w)) / (2 * eps))
    fd = vals[0]
    say("dot product (%s, mode %d): <Jv,w> %.9e (eps/2: %.9e), <v,J^T w> %.9e, rel %.2e" % (
        kinds, mode, vals[0], vals[1], adj, abs(adj - fd) / abs(fd)))
    assert abs(vals[0] - vals[1]) <= 1e-4 * abs(fd)      # the difference quotient has converged
    assert abs(adj - fd) <= 1e-3 * abs(fd)
