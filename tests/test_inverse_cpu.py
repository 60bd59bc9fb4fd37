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
