"""Inverse rendering by gradient descent through the hand-written adjoint.

The paper calibrates its simulator by back-propagating an image loss through
the renderer (Sec. IV.B).  Here the target is a pixel-aligned, noiseless DIC
frame rendered from known prisms, and Adam recovers the shared dn, the defocus,
the DIC shear and bias, and every prism's centre, angle and half-width from a
perturbed start, minimising the mean squared image error.

Schedule (a curriculum of stages, each naming the parameter groups that move):
by default for the first ``globals_first`` steps only the four globals move (the
per-particle parameters would otherwise drift to compensate for 20 % errors in
dn, defocus, shear and bias, and some settle in other basins); then everything
moves, with a cosine decay of every rate over the last part of the run.  Optionally
the first ``blur_steps`` steps compare blurred residuals (a coarse start).

Losses: the mean squared image error for a pixel-aligned target, or the
spectral loss of Eq. 8 (log amplitudes of the 2-D DFT, eps = ``spectral_eps``
times the target's DC term) for a target that cannot be aligned pixel by pixel
-- another placement of particles with the same statistics.  Against such a
target only the optical globals are defined, so its curriculum freezes the
geometry (the paper's calibration of blur-like optical parameters from
unaligned micrographs, Sec. IV.B).

Parameter error (how "1e-3 relative parameter error" is measured):
  e = max(e_glob, e_part)
  e_glob = max over dn, dz, shear, bias of |p - p*| / max(|p*|, floor)
           (floor 0.5 um for dz, whose true value can be near 0; none otherwise)
  e_part = max over prisms of |dx| / 3 px, |dy| / 3 px, |d angle mod pi/2| / 0.2 rad,
           |dw| / 3 px   (each per-particle error relative to its perturbation scale;
           a square prism's angle is defined modulo pi/2)

Nothing here computes the image: every forward and backward call goes through
``render.RenderFn`` (libosog).  A different differentiable ``render_fn`` can be
injected, which the CPU tests use to check the optimiser logic.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import torch

GLOBAL_NAMES = ("dn", "dz", "shear", "bias")


@dataclass
class SolverConfig:
    steps: int = 500
    lr_pos: float = 0.08       # px
    lr_angle: float = 0.008    # rad
    lr_width: float = 0.08     # px
    lr_dn: float = 4e-4
    lr_dz: float = 0.03        # um
    lr_shear: float = 0.01     # px
    lr_bias: float = 0.01      # rad
    betas: tuple = (0.9, 0.99)
    decay_after: float = 0.6   # fraction of the steps after which the rates decay
    decay_to: float = 0.1      # final rate multiplier (cosine)
    target_error: float = 1e-3
    width_floor: float = 1.0   # half-width kept >= 1 px
    globals_first: int = 60    # steps during which only dn, dz, shear, bias move
    # explicit curriculum: ((steps, groups), ...) with groups from GROUPS; overrides
    # globals_first when given (the last stage lasts to the end)
    curriculum: Optional[tuple] = None
    loss: str = "mse"          # "mse" (pixel-aligned target) or "spectral" (Eq. 8)
    spectral_eps: float = 1e-4 # eps of the spectral loss, relative to the target's DC term
    # coarse start: for the first blur_steps steps the pixel loss compares the residual
    # I - target after two box blurs of radius r = blur_radius px (close to a Gaussian of
    # sigma = sqrt(((2 r + 1)^2 - 1) / 6) px, 5.3 px for r = 6), which widens each
    # particle's basin of attraction
    blur_steps: int = 0
    blur_radius: int = 0
    # replay each step as one captured HIP graph (one per curriculum stage) when the
    # target is on the GPU; the eager loop issues ~50 launches per step and is bound by
    # the host.  The steps compute the same values either way.
    graph: bool = True


@dataclass
class Truth:
    x: torch.Tensor
    y: torch.Tensor
    angle: torch.Tensor
    width: torch.Tensor
    globals4: torch.Tensor     # dn, dz, shear, bias


@dataclass
class SolveResult:
    steps: int
    error: np.ndarray          # e per step (after the update), len = steps + 1 (index 0 = start)
    loss: np.ndarray           # per step (before the update)
    time_s: np.ndarray         # GPU time since the start of step 0, per step end
    steps_to_target: Optional[int]
    time_to_target_s: Optional[float]
    final: dict = field(default_factory=dict)
    error_glob: Optional[np.ndarray] = None   # e_glob per step, len = steps + 1
    error_part: Optional[np.ndarray] = None   # e_part per step, len = steps + 1
    steps_to_glob_target: Optional[int] = None
    time_to_glob_target_s: Optional[float] = None
    graphed: bool = False                     # steps replayed from captured graphs


class Params(torch.nn.Module):
    """Unknowns of the inverse problem; builds the SoA table and the globals."""

    def __init__(self, x, y, angle, width, height, glob):
        super().__init__()
        self.x = torch.nn.Parameter(x.clone())
        self.y = torch.nn.Parameter(y.clone())
        self.angle = torch.nn.Parameter(angle.clone())
        self.width = torch.nn.Parameter(width.clone())
        self.dn = torch.nn.Parameter(glob[0:1].clone())
        self.dz = torch.nn.Parameter(glob[1:2].clone())
        self.shear = torch.nn.Parameter(glob[2:3].clone())
        self.bias = torch.nn.Parameter(glob[3:4].clone())
        self.register_buffer("height", height.clone())

    def soa(self) -> torch.Tensor:
        n = self.x.shape[0]
        return torch.stack([self.x, self.y, self.angle, self.width, self.width, self.height,
                            self.dn.expand(n), torch.zeros_like(self.x)])

    def globals4(self) -> torch.Tensor:
        return torch.cat([self.dz, self.shear, self.bias, torch.zeros_like(self.dz)])

    def glob(self) -> torch.Tensor:
        return torch.cat([self.dn, self.dz, self.shear, self.bias])


def error_floor(device) -> torch.Tensor:
    """Denominator floor of e_glob per global (dn, dz, shear, bias)."""
    return torch.tensor([0.0, 0.5, 0.0, 0.0], device=device, dtype=torch.float32)


def parameter_errors(p: Params, truth: Truth, floor: Optional[torch.Tensor] = None):
    """(e_glob, e_part) on the device (see the module docstring).  ``floor``: a
    precomputed error_floor (needed inside a graph capture, which allows no
    host-to-device copy)."""
    g = p.glob()
    if floor is None:
        floor = error_floor(g.device)
    e_glob = ((g - truth.globals4).abs() / torch.maximum(truth.globals4.abs(), floor)).max()
    da = torch.remainder(p.angle - truth.angle + math.pi / 4, math.pi / 2) - math.pi / 4
    e_part = torch.stack([((p.x - truth.x).abs() / 3.0).max(), ((p.y - truth.y).abs() / 3.0).max(),
                          (da.abs() / 0.2).max(), ((p.width - truth.width).abs() / 3.0).max()]).max()
    return e_glob, e_part


def parameter_error(p: Params, truth: Truth) -> torch.Tensor:
    """e = max(e_glob, e_part) on the device (see the module docstring)."""
    e_glob, e_part = parameter_errors(p, truth)
    return torch.maximum(e_glob, e_part)


GROUPS = ("position", "angle", "width", "dn", "dz", "shear", "bias")


def stage_groups(cfg: SolverConfig, k: int) -> frozenset:
    """Parameter groups that move at step k."""
    if cfg.curriculum is None:
        return frozenset(GROUPS[3:]) if k < cfg.globals_first else frozenset(GROUPS)
    end = 0
    for n, groups in cfg.curriculum:
        end += n
        if k < end:
            return frozenset(groups)
    return frozenset(cfg.curriculum[-1][1])


def _params_of(p: "Params", group: str):
    return {"position": (p.x, p.y), "angle": (p.angle,), "width": (p.width,), "dn": (p.dn,),
            "dz": (p.dz,), "shear": (p.shear,), "bias": (p.bias,)}[group]


def _lr_groups(p: Params, cfg: SolverConfig):
    return [
        {"params": [p.x, p.y], "lr": cfg.lr_pos},
        {"params": [p.angle], "lr": cfg.lr_angle},
        {"params": [p.width], "lr": cfg.lr_width},
        {"params": [p.dn], "lr": cfg.lr_dn},
        {"params": [p.dz], "lr": cfg.lr_dz},
        {"params": [p.shear], "lr": cfg.lr_shear},
        {"params": [p.bias], "lr": cfg.lr_bias},
    ]


_side_streams = {}


def _warmup_stream(dev) -> "torch.cuda.Stream":
    """One warm-up stream per device, reused by every solve (the renderer keeps a
    workspace per stream, so a fresh stream per solve would add one each time)."""
    key = torch.device(dev).index
    if key not in _side_streams:
        _side_streams[key] = torch.cuda.Stream(device=dev)
    return _side_streams[key]


def _graph_memsets(g) -> int:
    """Memset nodes in a captured graph.  A step graph must hold kernels and copies
    only (a memset node is replayed as recorded, and such nodes have left wrong
    values on replays after the first), so one that holds a memset is not used."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so")
    graph = ctypes.c_void_p(g.raw_cuda_graph())
    n = ctypes.c_size_t(0)
    if hip.hipGraphGetNodes(graph, None, ctypes.byref(n)) != 0:
        raise RuntimeError("hipGraphGetNodes failed")
    nodes = (ctypes.c_void_p * max(n.value, 1))()
    if hip.hipGraphGetNodes(graph, nodes, ctypes.byref(n)) != 0:
        raise RuntimeError("hipGraphGetNodes failed")
    kinds = ctypes.c_int(-1)
    memsets = 0
    for i in range(n.value):
        if hip.hipGraphNodeGetType(ctypes.c_void_p(nodes[i]), ctypes.byref(kinds)) != 0:
            raise RuntimeError("hipGraphNodeGetType failed")
        memsets += kinds.value == 2  # hipGraphNodeTypeMemset
    return memsets


def solve(target: torch.Tensor, start: Params, truth: Optional[Truth], H: int, W: int, optics,
          cfg: SolverConfig = SolverConfig(),
          render_fn: Optional[Callable] = None) -> SolveResult:
    """Adam on L = mean((I(theta) - target)^2) (or the spectral loss, cfg.loss);
    returns error/loss/time traces.

    ``start`` is modified in place.  Errors and losses stay on the GPU during
    the loop (no host synchronisation per step); per-step GPU times come from
    events recorded on the current stream.  On the GPU (``cfg.graph``) every
    step is one replay of a captured graph of the whole step (forward, loss,
    adjoint, Adam, clamp, errors), captured once per curriculum stage after
    three eager warm-up steps whose effect on the parameters and on Adam's state
    is undone; the rates of the cosine decay live in a device tensor that each
    step rewrites.  If a captured graph holds a memset node the solve runs eager.
    """
    if cfg.blur_steps > 0 and (cfg.loss != "mse" or cfg.blur_radius < 1):
        raise ValueError("blur_steps needs the mse loss and blur_radius >= 1")
    if render_fn is None:
        from .render import render_diff

        def render_fn(soa, g):
            return render_diff(soa, g, H, W, optics)

    if cfg.loss == "spectral":
        from .render import spectral_loss_diff, spectral_target
        eps = cfg.spectral_eps * float(target.double().sum())
        tl = spectral_target(target, eps)

        def loss_fn(I):
            return spectral_loss_diff(I, tl, eps)
    elif cfg.loss == "mse":
        inv_n = 1.0 / target.numel()
        rb = cfg.blur_radius

        def loss_fn(I, blurred=False):  # row sums, then their sum: no grid-wide reduction
            r = I - target
            if blurred:
                q = r.reshape(1, 1, *r.shape[-2:])
                for _ in range(2):
                    q = torch.nn.functional.avg_pool2d(q, 2 * rb + 1, stride=1, padding=rb)
                r = q.reshape(r.shape)
            return torch.sum(torch.sum(r ** 2, dim=-1)) * inv_n
    else:
        raise ValueError("loss must be 'mse' or 'spectral'")
    dev = target.device
    on_gpu = target.is_cuda
    groups = _lr_groups(start, cfg)
    base = [g["lr"] for g in groups]
    if on_gpu:  # rates as views of one device tensor, rewritten in place by the decay
        base_t = torch.tensor(base, dtype=torch.float32, device=dev)
        lr_all = base_t.clone()
        for k, g in enumerate(groups):
            g["lr"] = lr_all[k]
        opt = torch.optim.Adam(groups, betas=cfg.betas, capturable=True, foreach=True)
    else:
        opt = torch.optim.Adam(groups, betas=cfg.betas)
    losses = torch.zeros(cfg.steps, device=dev)
    errors = torch.zeros((cfg.steps + 1, 2), device=dev)
    static_loss = torch.zeros((), device=dev)
    static_err = torch.zeros(2, device=dev)
    floor = error_floor(dev)
    k0 = int(cfg.decay_after * cfg.steps)

    def rate_mult(k):  # cosine decay of every group's rate over the last part of the run
        if k < k0:
            return 1.0
        f = (k - k0) / max(1, cfg.steps - k0)
        return cfg.decay_to + (1 - cfg.decay_to) * 0.5 * (1 + math.cos(math.pi * f))

    def set_rates(k):
        m = rate_mult(k)
        if on_gpu:
            torch.mul(base_t, m, out=lr_all)
        else:
            for g, b in zip(opt.param_groups, base):
                g["lr"] = b * m

    def body(moving, blurred=False):
        opt.zero_grad(set_to_none=True)
        I = render_fn(start.soa(), start.globals4())
        loss = loss_fn(I, blurred) if blurred else loss_fn(I)
        loss.backward()
        for grp in GROUPS:  # frozen groups keep their values (and Adam state)
            if grp not in moving:
                for q in _params_of(start, grp):
                    q.grad = None
        opt.step()
        with torch.no_grad():
            start.width.clamp_(min=cfg.width_floor)
            static_loss.copy_(loss.detach())
            if truth is not None:
                static_err.copy_(torch.stack(parameter_errors(start, truth, floor)))

    graphs = None
    def key(k):  # what one step does: the groups that move and whether the loss is blurred
        return stage_groups(cfg, k), k < cfg.blur_steps

    stages = sorted({key(k) for k in range(cfg.steps)}, key=lambda f: (sorted(f[0]), f[1]))
    if on_gpu and cfg.graph and cfg.steps > 0:
        saved = [q.detach().clone() for q in start.parameters()]
        side = _warmup_stream(dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):  # warm-up: creates Adam's state and the allocator's blocks
            for i in range(3):
                body(frozenset(GROUPS), i == 0 and cfg.blur_steps > 0)
        torch.cuda.current_stream(dev).wait_stream(side)
        graphs, pool = {}, None
        for st in stages:
            g = torch.cuda.CUDAGraph(keep_graph=True)
            with torch.cuda.graph(g, pool=pool):
                body(*st)
            pool = g.pool()
            g.instantiate()
            if _graph_memsets(g):
                graphs = None
                break
            graphs[st] = g
        with torch.no_grad():  # undo the warm-up and capture steps
            for q, v in zip(start.parameters(), saved):
                q.copy_(v)
            for st in opt.state.values():
                for v in st.values():
                    if torch.is_tensor(v):
                        v.zero_()
    timing = on_gpu
    events = [torch.cuda.Event(enable_timing=True) for _ in range(cfg.steps + 1)] if timing else None
    t_host = []
    with torch.no_grad():
        if truth is not None:
            errors[0] = torch.stack(parameter_errors(start, truth))
    if timing:
        events[0].record()
    t0 = time.perf_counter()
    for k in range(cfg.steps):
        if k >= k0 or k == 0:
            set_rates(k)
        if graphs is not None:
            graphs[key(k)].replay()
        else:
            body(*key(k))
        losses[k].copy_(static_loss)
        if truth is not None:
            errors[k + 1].copy_(static_err)
        if timing:
            events[k + 1].record()
        else:
            t_host.append(time.perf_counter() - t0)
    if timing:
        torch.cuda.synchronize()
        times = np.array([events[0].elapsed_time(e) / 1000.0 for e in events[1:]])
    else:
        times = np.array(t_host)
    eg = errors.cpu().numpy()
    err = eg.max(axis=1)
    hit = np.nonzero(err[1:] <= cfg.target_error)[0] if truth is not None else np.array([])
    hitg = np.nonzero(eg[1:, 0] <= cfg.target_error)[0] if truth is not None else np.array([])
    return SolveResult(cfg.steps, err, losses.cpu().numpy(), times,
                       int(hit[0]) + 1 if hit.size else None, float(times[hit[0]]) if hit.size else None,
                       {k: float(v) for k, v in zip(GLOBAL_NAMES, start.glob().detach().cpu().numpy())},
                       eg[:, 0], eg[:, 1], int(hitg[0]) + 1 if hitg.size else None,
                       float(times[hitg[0]]) if hitg.size else None, graphs is not None)


def problem_tensors(prob, device):
    """(target image, Params at the perturbed start, Truth) for a workloads.InverseProblem."""
    from .render import render
    tf, inf = prob.target, prob.init
    soa_t = torch.from_numpy(tf.soa).to(device)
    g_t = torch.from_numpy(tf.globals4).to(device)
    target = render(soa_t, tf.H, tf.W, tf.optics, g_t)
    s0 = torch.from_numpy(inf.soa).to(device)
    glob0 = torch.tensor([float(inf.soa[6, 0]), *[float(v) for v in inf.globals4[:3]]],
                         dtype=torch.float32, device=device)
    start = Params(s0[0], s0[1], s0[2], s0[3], s0[5], glob0).to(device)
    truth = Truth(soa_t[0], soa_t[1], soa_t[2], soa_t[3],
                  torch.tensor([float(tf.soa[6, 0]), *[float(v) for v in tf.globals4[:3]]],
                               dtype=torch.float32, device=device))
    return target, start, truth


@dataclass
class HybridResult:
    """Adam, then the second-order polish (polish.py).  Times are seconds since the
    start of Adam's first step (GPU events for Adam, wall clock after it)."""
    adam: SolveResult
    trace: list                               # polish stages: (tag, time_s, e, e_glob)
    time_to_target_s: Optional[float]
    time_to_glob_target_s: Optional[float]    # e_glob <= target (the four globals)
    final_loss: float
    final_e: Optional[float]
    final_e_glob: Optional[float]
    final_e_part: Optional[float]
    total_s: float
    final: dict = field(default_factory=dict)


def hybrid_config(steps: int = 500, globals_steps: int = 60) -> SolverConfig:
    """Adam schedule of the hybrid solve: the globals alone, then centres, widths and
    globals; the angles stay at their start (inside +-0.2 rad of the truth, the bracket
    the polish's angle search covers) until the polish."""
    glob = ("dn", "dz", "shear", "bias")
    return SolverConfig(steps=steps, curriculum=((globals_steps, glob), (steps - globals_steps, ("position", "width") + glob)))


def solve_hybrid(target: torch.Tensor, start: Params, truth: Optional[Truth], H: int, W: int, optics,
                 cfg: Optional[SolverConfig] = None, pc=None) -> HybridResult:
    """Adam (``cfg``, by default hybrid_config()) then polish.polish (``pc``) from
    Adam's state; ``start`` ends at the solution.  With a truth, e after every Adam
    step and every polish stage is recorded (the truth never steers the solve)."""
    from . import polish
    cfg = cfg or hybrid_config()
    pc = pc or polish.PolishConfig()
    res = solve(target, start, truth, H, W, optics, cfg)
    torch.cuda.synchronize(target.device)
    t_adam = float(res.time_s[-1]) if len(res.time_s) else 0.0
    model = polish.Model(H, W, optics, start.height.detach())
    floor = error_floor(target.device)

    glob_err = []

    def error_fn(x, y, a, w, glob):
        tmp = Params(x, y, a, w, start.height.detach(), glob)
        eg, ep = parameter_errors(tmp, truth, floor)
        glob_err.append(float(eg))
        return float(torch.maximum(eg, ep))

    t0 = time.perf_counter()
    with torch.no_grad():
        x, y, a, w, glob = (t.detach().clone() for t in (start.x, start.y, start.angle, start.width, start.glob()))
        x, y, a, w, glob, trace = polish.polish(target, model, x, y, a, w, glob, pc,
                                                error_fn=error_fn if truth is not None else None,
                                                clock=lambda: t_adam + time.perf_counter() - t0)
        torch.cuda.synchronize(target.device)
        total = t_adam + time.perf_counter() - t0
        for q, v in ((start.x, x), (start.y, y), (start.angle, a), (start.width, w)):
            q.copy_(v)
        for q, v in zip((start.dn, start.dz, start.shear, start.bias), glob):
            q.fill_(float(v))
    trace = [(tag, t, e, eg) for (tag, t, e), eg in zip(trace, glob_err)] if truth is not None else trace
    hit, hitg = res.time_to_target_s, res.time_to_glob_target_s
    for _, t, e, eg in (trace if truth is not None else []):
        if hit is None and e <= cfg.target_error:
            hit = t
        if hitg is None and eg <= cfg.target_error:
            hitg = t
    fe = fg = fp = None
    if truth is not None:
        eg, ep = parameter_errors(start, truth)
        fe, fg, fp = float(torch.maximum(eg, ep)), float(eg), float(ep)
    with torch.no_grad():
        I = model.render(start.x, start.y, start.angle, start.width, start.glob())
        final_loss = float(torch.mean((I.double() - target.double()) ** 2))
    return HybridResult(res, trace, hit, hitg, final_loss, fe, fg, fp, total,
                        {k: float(v) for k, v in zip(GLOBAL_NAMES, start.glob().detach().cpu().numpy())})
