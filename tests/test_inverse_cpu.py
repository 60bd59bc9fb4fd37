"""Host logic of the inverse solver: error metric, optimiser loop, bookkeeping.

The renderer is injected as a small differentiable torch function so the loop
runs on the CPU; the product path always renders through libosog.
"""
import math

import numpy as np
import torch

from paper_2606_21381_amd import inverse


def make(n=5, seed=0):
    g = torch.Generator().manual_seed(seed)
    x = torch.rand(n, generator=g) * 50
    y = torch.rand(n, generator=g) * 50
    a = torch.rand(n, generator=g) * math.pi
    w = 3 + torch.rand(n, generator=g) * 5
    h = torch.ones(n)
    glob = torch.tensor([0.03, -0.8, 1.0, math.pi / 2])
    return x, y, a, w, h, glob


def test_parameter_error_definition():
    x, y, a, w, h, glob = make()
    truth = inverse.Truth(x, y, a, w, glob)
    p = inverse.Params(x, y, a, w, h, glob)
    assert float(inverse.parameter_error(p, truth)) == 0.0
    with torch.no_grad():
        p.x[2] += 0.3                      # 0.3 px / 3 px = 0.1
    assert abs(float(inverse.parameter_error(p, truth)) - 0.1) < 1e-6
    with torch.no_grad():
        p.x[2] -= 0.3
        p.angle[1] += math.pi / 2 + 0.01   # a square prism's angle counts modulo pi/2
    assert abs(float(inverse.parameter_error(p, truth)) - 0.05) < 1e-4
    with torch.no_grad():
        p.angle[1] -= math.pi / 2 + 0.01
        p.dz[0] = -0.8 + 0.05              # dz error relative to max(|dz*|, 0.5) = 0.8
    assert abs(float(inverse.parameter_error(p, truth)) - 0.0625) < 1e-6
    t0 = inverse.Truth(x, y, a, w, torch.tensor([0.03, 0.01, 1.0, math.pi / 2]))
    p2 = inverse.Params(x, y, a, w, h, torch.tensor([0.03, 0.06, 1.0, math.pi / 2]))
    assert abs(float(inverse.parameter_error(p2, t0)) - 0.1) < 1e-6  # floor 0.5 um for dz


def test_solver_converges_on_a_smooth_toy_model():
    x, y, a, w, h, glob = make(4)
    truth = inverse.Truth(x, y, a, w, glob)
    A = torch.randn(64, 8 * 4 + 4, generator=torch.Generator().manual_seed(1), dtype=torch.float64)

    def toy(soa, g):  # linear "image" of the parameters: a convex quadratic loss
        v = torch.cat([soa.reshape(-1), g]).double()
        return (A @ v).float()

    target = toy(inverse.Params(x, y, a, w, h, glob).soa(), inverse.Params(x, y, a, w, h, glob).globals4()).detach()
    start = inverse.Params(x + 1.0, y - 1.0, a + 0.1, w + 0.5, h,
                           glob * torch.tensor([1.1, 0.9, 1.1, 0.95]))
    cfg = inverse.SolverConfig(steps=600, lr_pos=0.05, lr_angle=0.01, lr_width=0.05, lr_dn=1e-3,
                               lr_dz=0.01, lr_shear=0.01, lr_bias=0.01, target_error=1e-2)
    res = inverse.solve(target, start, truth, 8, 8, None, cfg, render_fn=toy)
    assert res.error.shape == (601,) and res.loss.shape == (600,) and res.time_s.shape == (600,)
    assert res.error[0] > 0.1
    assert res.steps_to_target is not None and res.error[res.steps_to_target] <= 1e-2
    assert res.time_to_target_s == res.time_s[res.steps_to_target - 1]
    assert np.all(np.diff(res.time_s) >= 0)
    assert res.loss[-1] < 1e-3 * res.loss[0]


def test_curriculum_stages():
    from paper_2606_21381_amd import inverse
    cfg = inverse.SolverConfig(globals_first=60)
    assert inverse.stage_groups(cfg, 0) == frozenset(("dn", "dz", "shear", "bias"))
    assert inverse.stage_groups(cfg, 60) == frozenset(inverse.GROUPS)
    cur = inverse.SolverConfig(curriculum=((10, ("dz",)), (5, ("position", "width")), (1, ("bias",))))
    assert inverse.stage_groups(cur, 9) == frozenset(("dz",))
    assert inverse.stage_groups(cur, 10) == frozenset(("position", "width"))
    assert inverse.stage_groups(cur, 15) == frozenset(("bias",))
    assert inverse.stage_groups(cur, 1000) == frozenset(("bias",))


def _toy_model(H=64, W=64, n=6):
    """A smooth stand-in for the renderer: oriented Gaussian blobs (long axis w, short
    axis (0.5 + 0.1 shear) w) scaled by dn, each with a round halo of twice its width
    weighted by dz, on a background set by the bias (every global has its own
    signature); gradients by autograd."""
    from paper_2606_21381_amd import polish
    jj, ii = torch.meshgrid(torch.arange(W, dtype=torch.float64), torch.arange(H, dtype=torch.float64), indexing="xy")

    def render(x, y, a, w, glob):
        x, y, a, w, glob = (t.double() for t in (x, y, a, w, glob))
        dx = jj[None] - x[:, None, None]
        dy = ii[None] - y[:, None, None]
        c, s = torch.cos(a)[:, None, None], torch.sin(a)[:, None, None]
        u, v = c * dx + s * dy, -s * dx + c * dy
        ww = w[:, None, None]
        sv = (0.5 + 0.1 * glob[2]) * ww
        blobs = torch.exp(-(u * u) / (ww * ww) - (v * v) / (sv * sv))
        halo = torch.exp(-(dx * dx + dy * dy) / (4.0 * ww * ww))
        return (glob[3] + 30.0 * glob[0] * blobs.sum(0) + 0.2 * glob[1] * halo.sum(0)).float()

    def grad(x, y, a, w, glob, gI):
        v = [t.detach().clone().requires_grad_(True) for t in (x, y, a, w, glob)]
        (render(*v).double() * gI.double()).sum().backward()
        return torch.stack([v[0].grad, v[1].grad, v[2].grad, v[3].grad]).float(), v[4].grad.float()

    return polish.Model(H, W, None, torch.ones(n), render_fn=render, grad_fn=grad), render


def test_polish_recovers_a_toy_problem():
    """Angle search plus Gauss-Newton-CG from a start 0.15 rad, 0.3 px and 5 % off the
    truth of six well-separated blobs: every parameter within 1e-3 of its scale."""
    from paper_2606_21381_amd import polish
    torch.manual_seed(0)
    model, render = _toy_model()
    x = torch.tensor([12.0, 30.0, 50.0, 14.0, 33.0, 52.0])
    y = torch.tensor([12.0, 14.0, 11.0, 45.0, 50.0, 47.0])
    a = torch.tensor([0.3, 1.0, 2.0, 0.6, 1.4, 2.6])
    w = torch.tensor([3.0, 4.0, 3.5, 4.5, 3.2, 3.8])
    g = torch.tensor([0.03, 0.5, 0.2, 1.0])
    target = render(x, y, a, w, g)
    pert = torch.tensor([1.0, -1.0, 1.0, -1.0, 1.0, -1.0])
    pc = polish.PolishConfig(iters=12, margin_px=6.0, separation_px=6.0, eps=(0.01, 0.01, 0.002, 0.01),
                             eps_glob=(1e-4, 0.01, 0.01, 0.01), angle_span=0.3, angle_steps=31, research_w_max=10.0)
    res = polish.polish(target, model, x + 0.3 * pert, y - 0.3 * pert, a + 0.15 * pert, w * 1.05,
                        g * torch.tensor([1.05, 0.95, 1.05, 1.02]), pc)
    xr, yr, ar, wr, gr = res[:5]
    da = torch.remainder(ar - a + math.pi / 4, math.pi / 2) - math.pi / 4
    assert float((xr - x).abs().max()) < 3e-3 and float((yr - y).abs().max()) < 3e-3
    assert float(da.abs().max()) < 2e-4 and float((wr - w).abs().max()) < 3e-3
    assert float(((gr - g).abs() / g.abs()).max()) < 1e-3


def test_colouring_keeps_colours_apart():
    from paper_2606_21381_amd import polish
    rng = np.random.default_rng(1)
    x, y, w = rng.uniform(0, 256, 60), rng.uniform(0, 256, 60), rng.uniform(3, 8, 60)
    color, bounds = polish.color_windows(x, y, w, 256, 256, 5.0, 20.0)
    sep = w * math.sqrt(2) + 20.0
    for i in range(60):
        same = (color == color[i]) & (np.arange(60) != i)
        assert not np.any(same & (np.abs(x - x[i]) < sep + sep[i]) & (np.abs(y - y[i]) < sep + sep[i]))
    assert np.all(bounds[:, 0] <= bounds[:, 1]) and np.all(bounds[:, 0] >= 0) and np.all(bounds[:, 1] <= 255)


def test_reseed_returns_a_displaced_particle():
    """A blob left 2 px and 3 px off in x and y, its width 1.5 px too large, is moved
    back onto its truth by one re-seed (a grid point), and the particles already at
    their truth stay where they are."""
    from paper_2606_21381_amd import polish
    model, render = _toy_model()
    x = torch.tensor([12.0, 30.0, 50.0, 14.0, 33.0, 52.0])
    y = torch.tensor([12.0, 14.0, 11.0, 45.0, 50.0, 47.0])
    a = torch.tensor([0.3, 1.0, 2.0, 0.6, 1.4, 2.6])
    w = torch.tensor([3.0, 4.0, 3.5, 4.5, 3.2, 3.8])
    g = torch.tensor([0.03, 0.5, 0.2, 1.0])
    target = render(x, y, a, w, g)
    xs, ys, ws = x.clone(), y.clone(), w.clone()
    xs[1] += 2.0
    ys[1] -= 3.0
    ws[1] += 1.5
    pc = polish.PolishConfig(margin_px=6.0, separation_px=6.0)
    xr, yr, ar, wr, moved = polish.reseed(model, target, xs, ys, a.clone(), ws, g, pc)
    assert moved == 1
    assert torch.equal(xr, x) and torch.equal(yr, y) and torch.equal(wr, w) and torch.equal(ar, a)
    # at the truth nothing is selected or moved
    assert polish.reseed(model, target, x, y, a, w, g, pc)[4] == 0


def test_blurred_start_runs_and_converges():
    """The optional coarse start (blurred residuals for the first steps) moves blobs
    4 px off back onto their truth; it needs the pixel loss."""
    H = W = 48
    ii = torch.arange(H, dtype=torch.float32)[:, None]
    jj = torch.arange(W, dtype=torch.float32)[None, :]

    def blobs(soa, g):
        I = torch.zeros(H, W)
        for k in range(soa.shape[1]):
            I = I + torch.exp(-((ii - soa[1, k]) ** 2 + (jj - soa[0, k]) ** 2) / 8.0)
        return I * g[0] * 30

    x, y = torch.tensor([10.0, 25.0, 38.0]), torch.tensor([12.0, 30.0, 20.0])
    a, w, h = torch.zeros(3), torch.full((3,), 3.0), torch.ones(3)
    glob = torch.tensor([0.03, -0.8, 1.0, math.pi / 2])
    truth = inverse.Truth(x, y, a, w, glob)
    p = inverse.Params(x, y, a, w, h, glob)
    target = blobs(p.soa(), p.globals4()).detach()
    start = inverse.Params(x + 4.5, y - 4.0, a, w, h, glob)
    cfg = inverse.SolverConfig(steps=300, lr_pos=0.2, curriculum=((300, ("position",)),),
                               blur_steps=150, blur_radius=4, target_error=1e-2)
    res = inverse.solve(target, start, truth, H, W, None, cfg, render_fn=blobs)
    assert res.steps_to_target is not None and res.error[-1] < 1e-3
    bad = inverse.SolverConfig(steps=3, loss="spectral", blur_steps=2, blur_radius=2)
    try:
        inverse.solve(target, inverse.Params(x, y, a, w, h, glob), truth, H, W, None, bad, render_fn=blobs)
    except ValueError:
        pass
    else:
        raise AssertionError("a blurred start with the spectral loss must be refused")


def test_reseed_uncrosses_a_swapped_pair():
    """Two overlapping blobs of different heights whose centres were exchanged are
    put back by the re-seed's pair exchange."""
    from paper_2606_21381_amd import polish
    H = W = 64
    jj, ii = torch.meshgrid(torch.arange(W, dtype=torch.float64), torch.arange(H, dtype=torch.float64), indexing="xy")
    height = torch.tensor([1.0, 2.5, 1.0])

    def render(x, y, a, w, glob):
        x, y, w = (t.double() for t in (x, y, w))
        dx = jj[None] - x[:, None, None]
        dy = ii[None] - y[:, None, None]
        ww = w[:, None, None]
        return (height.double()[:, None, None] * torch.exp(-(dx * dx + dy * dy) / (ww * ww))).sum(0).float()

    model = polish.Model(H, W, None, height, render_fn=render, grad_fn=lambda *args: None)
    x = torch.tensor([30.0, 33.0, 10.0])
    y = torch.tensor([30.0, 32.0, 50.0])
    a = torch.zeros(3)
    w = torch.tensor([4.0, 4.0, 3.0])
    g = torch.zeros(4)
    target = render(x, y, a, w, g)
    xs, ys = x[[1, 0, 2]], y[[1, 0, 2]]
    pc = polish.PolishConfig(margin_px=6.0, separation_px=6.0, reseed_px=0, reseed_dw=(0.0,))
    xr, yr, ar, wr, moved = polish.reseed(model, target, xs, ys, a.clone(), w.clone(), g, pc)
    assert moved >= 2
    assert torch.equal(xr, x) and torch.equal(yr, y)
