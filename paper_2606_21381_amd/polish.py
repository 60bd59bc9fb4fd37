"""Second-order finish of the inverse solve: bracketed angle search and
Gauss-Newton steps on the image loss.

The paper calibrates its simulator by gradient descent through the renderer
(Sec. IV.B).  Adam reaches the truth's neighbourhood, but the angles of small
prisms barely change the image (a 3 px prism turned by 0.1 rad changes the loss
by ~1e-9) and end in shallow side minima, and the defocus converges slowly.
This module finishes from Adam's state with two tools that use only the
library's forward render and hand-written adjoint:

* Angle search.  For every particle, the image loss inside its window (its box
  widened by the optical spread) is evaluated at evenly spaced angles across a
  bracket around the current angle, and the best one is kept.  Particles are
  coloured so that windows of one colour do not overlap; one render per
  (colour, candidate angle) then serves every particle of that colour.
* Gauss-Newton by preconditioned conjugate gradients.  The gradient J^T r is
  exact (the adjoint); products with J^T J take one forward-difference render
  (J v) and one adjoint call (J^T u); the preconditioner is J^T J restricted to
  4 x 4 blocks, one per particle (x, y, angle, half-width), with J's columns from
  forward differences (one render per colour and parameter), and one 4 x 4 block
  for the globals (dn, dz, shear, bias).  A step is kept only if the full loss
  decreases, and the damping adapts (Marquardt's rule).  (A block-diagonal
  variant, ``method = "block"``, alternates particle and global block steps.)
* Colouring.  Particles of one colour move together in the searches and the
  forward differences, so they are kept ``separation_px`` further apart than
  their boxes: a particle's optical influence (defocus, DIC shear, the band
  limit's ringing) reaches tens of pixels past its box, and with windows merely
  disjoint the neighbours' changes dominated a small prism's window loss.
  Repeated searches turn only prisms narrower than ``research_w_max``: the large
  ones' angles are well determined, and turning them leaves far-reaching residuals.
  They scan a whole period of the square's angle (+-pi/4), since a small prism's
  first search, made while the positions were still off, can end in a side minimum
  more than the first bracket away from the truth.
* Closing angle search.  The repeated searches leave the small prisms' angles on a
  grid of a few 1e-3 rad, and the Gauss-Newton steps barely move them; when the
  steps end above the loss floor, those angles are searched once more over
  brackets of +-``final_span`` and a tenth of it.
* Re-seeding.  When the Gauss-Newton steps end above the loss floor, the
  particles whose window loss exceeds ``reseed_factor`` times the median are
  moved, colour by colour, to the best point of a grid around their state
  (centre offsets of whole pixels up to ``reseed_px``, half-width offsets
  ``reseed_dw``, the angle as it is or turned by pi/4), scored by the window loss;
  then the polish starts again from there.  This lets a particle that Adam left a
  few pixels from its truth, in a side minimum of its window, leave it.  The same
  stage tries exchanging the centres (or centres, angles and half-widths) of
  neighbouring particles closer than 1.5 times the larger half-width: their
  heights differ, so a pair that Adam crossed over fits the image nearly but not
  exactly, and no small step uncrosses it.

Nothing here computes an image: every render and gradient goes through libosog
(or the injected functions the CPU tests use).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, replace
from typing import Callable, Optional

import numpy as np
import torch


@dataclass
class PolishConfig:
    iters: int = 20               # Gauss-Newton steps at most
    margin_px: float = 12.0       # window = particle box widened by the optical spread
    separation_px: float = 40.0   # particles of one colour (moved together) are this much further apart
    eps: tuple = (0.02, 0.02, 0.004, 0.02)          # forward-difference steps: x, y [px], angle [rad], width [px]
    eps_glob: tuple = (1e-5, 0.004, 0.002, 0.002)   # dn, dz [um], shear [px], bias [rad]
    angle_span: float = 0.3       # angle search over [-span, +span] around the current angle
    angle_steps: int = 61
    angle_refine: int = 2         # further searches, each over a bracket 1/10 as wide
    lam0: float = 1e-3            # initial damping (relative to the block diagonal)
    target_error: float = 1e-3
    loss_tol: float = 1e-15       # stop once the mean squared image error is below loss_tol x mean(target^2)
    method: str = "cg"            # "cg": Gauss-Newton by preconditioned CG; "block": block steps only
    cg_iters: int = 20            # conjugate-gradient iterations per Gauss-Newton step
    search_every: int = 3         # repeat the angle search every this many steps (0: only at the start)
    research_span: float = math.pi / 4  # bracket of the repeated searches (a full period of a square)
    research_refine: int = 1      # further repeated searches, each over a bracket 1/10 as wide
    research_w_max: float = 5.0   # the repeated searches turn only prisms narrower than this [px]
    final_span: float = 3e-3      # closing search of those prisms' angles over +-final_span [rad]
    final_refine: int = 1         # further closing searches, each over a bracket 1/10 as wide
    # parameter scales of the CG's unknowns: x, y [px], angle [rad], width [px]; dn, dz, shear, bias
    scale: tuple = (1.0, 1.0, 0.1, 1.0)
    scale_glob: tuple = (1e-3, 0.1, 0.05, 0.05)
    jvp_eps: float = 0.01         # forward-difference step of J v along the scaled unit direction
    reseed_rounds: int = 1        # re-seed and polish again at most this many times
    reseed_factor: float = 10.0   # re-seed particles whose window loss exceeds this times the median
    reseed_px: int = 3            # centre offsets -reseed_px .. reseed_px px in x and y
    reseed_dw: tuple = (-1.5, 0.0, 1.5)  # half-width offsets [px]


class Model:
    """Forward render and adjoint of the inverse problem's parameterisation: n prisms
    with (x, y, angle, half-width) each, known heights, one shared dn, and the
    globals dz, shear, bias.  ``render(x, y, a, w, glob)`` -> image; ``grad(x, y, a,
    w, glob, gI)`` -> (d/d(x, y, a, w) as [4, n], d/d(dn, dz, shear, bias) as [4])
    for dL/dI = gI."""

    def __init__(self, H: int, W: int, optics, height: torch.Tensor,
                 render_fn: Optional[Callable] = None, grad_fn: Optional[Callable] = None):
        self.H, self.W, self.optics = H, W, optics
        self.height = height
        self.n = height.shape[0]
        self._render_fn = render_fn
        self._grad_fn = grad_fn
        dev = height.device
        if render_fn is None:
            from . import render as R
            self._R = R
            self._out = torch.empty((H, W), dtype=torch.float32, device=dev)
            self._ws = torch.empty(R.workspace_size(H, W, self.n), dtype=torch.uint8, device=dev)
            self._ws_b = torch.empty(R.workspace_size(H, W, self.n, with_backward=True), dtype=torch.uint8,
                                     device=dev)

    def soa(self, x, y, a, w, glob):
        n = self.n
        return torch.stack([x, y, a, w, w, self.height, glob[0].expand(n), torch.zeros_like(x)]).contiguous()

    @staticmethod
    def g4(glob):
        return torch.stack([glob[1], glob[2], glob[3], torch.zeros_like(glob[0])]).contiguous()

    def render(self, x, y, a, w, glob) -> torch.Tensor:
        if self._render_fn is not None:
            return self._render_fn(x, y, a, w, glob)
        return self._R.render(self.soa(x, y, a, w, glob), self.H, self.W, self.optics, self.g4(glob),
                              out=self._out, workspace=self._ws).clone()

    def grad(self, x, y, a, w, glob, gI):
        if self._grad_fn is not None:
            return self._grad_fn(x, y, a, w, glob, gI)
        gs, gg = self._R.render_backward(self.soa(x, y, a, w, glob), self.H, self.W, self.optics, self.g4(glob),
                                         gI.contiguous(), workspace=self._ws_b)
        gp = torch.stack([gs[0, :self.n], gs[1, :self.n], gs[2, :self.n], gs[3, :self.n] + gs[4, :self.n]])
        ggl = torch.stack([gs[6, :self.n].sum(), gg[0], gg[1], gg[2]])
        return gp, ggl


def color_windows(x, y, w, H, W, margin, separation=None):
    """Greedy colouring of the particles so that particles of one colour are apart by
    more than their boxes (half-side w sqrt 2) widened by `separation` each (default
    `margin`): a particle's optical influence reaches well past its own box, and
    particles of one colour move together.  Returns (colour per particle, window
    bounds [n, 4] -- the box widened by `margin`, clipped to the canvas, inclusive
    x0, x1, y0, y1 -- over which per-particle sums are taken)."""
    x, y, w = (np.asarray(v, dtype=np.float64) for v in (x, y, w))
    ext = w * math.sqrt(2.0) + margin
    x0 = np.clip(np.floor(x - ext), 0, W - 1).astype(int)
    x1 = np.clip(np.ceil(x + ext), 0, W - 1).astype(int)
    y0 = np.clip(np.floor(y - ext), 0, H - 1).astype(int)
    y1 = np.clip(np.ceil(y + ext), 0, H - 1).astype(int)
    sep = w * math.sqrt(2.0) + (margin if separation is None else separation)
    n = x.shape[0]
    order = np.argsort(-ext, kind="stable")
    color = -np.ones(n, dtype=int)
    for i in order:
        clash = (np.abs(x - x[i]) < sep + sep[i]) & (np.abs(y - y[i]) < sep + sep[i]) & (color >= 0)
        used = set(color[clash].tolist())
        c = 0
        while c in used:
            c += 1
        color[i] = c
    return color, np.stack([x0, x1, y0, y1], axis=1)


class Windows:
    """Per colour: the flat indices of the pixels inside that colour's windows and
    the particle each belongs to (for per-particle sums by index_add)."""

    def __init__(self, color, bounds, H, W, device):
        self.n = color.shape[0]
        self.colors = []
        for c in range(int(color.max()) + 1 if color.size else 0):
            members = np.nonzero(color == c)[0]
            pix, own = [], []
            for i in members:
                x0, x1, y0, y1 = bounds[i]
                ii, jj = np.meshgrid(np.arange(y0, y1 + 1), np.arange(x0, x1 + 1), indexing="ij")
                pix.append((ii * W + jj).reshape(-1))
                own.append(np.full(ii.size, i))
            self.colors.append((torch.as_tensor(members, device=device),
                                torch.as_tensor(np.concatenate(pix), device=device),
                                torch.as_tensor(np.concatenate(own), device=device)))

    def sums(self, c, img_flat):
        """Per-particle sums of img over colour c's windows (length n, zero elsewhere)."""
        _, pix, own = self.colors[c]
        out = torch.zeros(self.n, dtype=torch.float64, device=img_flat.device)
        return out.index_add_(0, own, img_flat[pix].double())


def _loss(I, target):
    return float(torch.mean((I.double() - target.double()) ** 2))


def angle_search(model: Model, target, x, y, a, w, glob, win: Windows, span: float, steps: int,
                 only: Optional[torch.Tensor] = None):
    """Per particle, the angle in [a - span, a + span] (steps values) that minimises the
    image loss inside its window, the other particles of its colour moved alike.
    ``only`` (bool [n]): search these particles and keep the others' angles (a
    turned large particle leaves residuals whose tails reach far)."""
    tf = target.reshape(-1)
    offs = torch.linspace(-span, span, steps, device=a.device)
    best_a = a.clone()
    for c, (members, _, _) in enumerate(win.colors):
        if only is not None:
            members = members[only[members]]
            if members.numel() == 0:
                continue
        best = torch.full((model.n,), float("inf"), dtype=torch.float64, device=a.device)
        for d in offs:
            ac = a.clone()
            ac[members] += d
            r = model.render(x, y, ac, w, glob).reshape(-1) - tf
            s = win.sums(c, r * r)
            better = s < best
            better_m = torch.zeros_like(better)
            better_m[members] = better[members]
            best = torch.where(better_m, s, best)
            best_a = torch.where(better_m, ac, best_a)
    return best_a


def reseed(model: Model, target, x, y, a, w, glob, pc: PolishConfig):
    """Moves every particle whose window loss exceeds pc.reseed_factor times the
    median to the best point of its grid (centre offsets in whole pixels up to
    pc.reseed_px, half-width offsets pc.reseed_dw, angle offsets 0 and pi/4), scored
    by the window loss with the other particles of its colour moved alike; keeps a
    particle where no grid point lowers its window loss.  Then, for every pair of
    particles closer than 1.5 times the larger half-width, keeps the exchange of their
    centres (or of centres, angles and half-widths) if it lowers the loss over the
    pair's joint window.  Returns (x, y, a, w, moved)."""
    color, bounds = color_windows(x.detach().cpu().numpy(), y.detach().cpu().numpy(),
                                  w.detach().cpu().numpy(), model.H, model.W, pc.margin_px, pc.separation_px)
    win = Windows(color, bounds, model.H, model.W, x.device)
    tf = target.reshape(-1)
    r = model.render(x, y, a, w, glob).reshape(-1) - tf
    s = torch.zeros(model.n, dtype=torch.float64, device=x.device)
    for c in range(len(win.colors)):
        s += win.sums(c, r * r)
    bad = s > float(torch.median(s)) * pc.reseed_factor
    R = pc.reseed_px
    grid = [(dx, dy, dw, da) for dx in range(-R, R + 1) for dy in range(-R, R + 1)
            for dw in pc.reseed_dw for da in (0.0, math.pi / 4)]
    best = s.clone()
    bx, by, ba, bw = x.clone(), y.clone(), a.clone(), w.clone()
    for c, (members, _, _) in enumerate(win.colors):
        m = members[bad[members]]
        if m.numel() == 0:
            continue
        for dx, dy, dw, da in grid:
            xc, yc, ac, wc = x.clone(), y.clone(), a.clone(), w.clone()
            xc[m] += dx
            yc[m] += dy
            ac[m] += da
            wc[m] = torch.clamp(wc[m] + dw, min=1.0)
            rc = model.render(xc, yc, ac, wc, glob).reshape(-1) - tf
            sc = win.sums(c, rc * rc)
            better = torch.zeros_like(bad)
            better[m] = sc[m] < best[m]
            best = torch.where(better, sc, best)
            bx, by = torch.where(better, xc, bx), torch.where(better, yc, by)
            ba, bw = torch.where(better, ac, ba), torch.where(better, wc, bw)
    moved = int(((bx != x) | (by != y) | (ba != a) | (bw != w)).sum())
    x, y, a, w = bx, by, ba, bw
    # exchanges within close pairs, scored by the loss over the pair's joint window
    xn, yn, wn = (v.detach().cpu().numpy().astype(np.float64) for v in (x, y, w))
    dist = np.hypot(xn[:, None] - xn[None], yn[:, None] - yn[None])
    close = (dist < 1.5 * np.maximum(wn[:, None], wn[None])) & np.triu(np.ones_like(dist, dtype=bool), 1)
    tg = target.reshape(model.H, model.W).double()
    I = model.render(x, y, a, w, glob).reshape(model.H, model.W)
    for i, j in np.argwhere(close).tolist():
        ext = pc.margin_px + 1.5 * max(wn[i], wn[j])
        x0 = max(0, math.floor(min(xn[i], xn[j]) - ext))
        x1 = min(model.W - 1, math.ceil(max(xn[i], xn[j]) + ext))
        y0 = max(0, math.floor(min(yn[i], yn[j]) - ext))
        y1 = min(model.H - 1, math.ceil(max(yn[i], yn[j]) + ext))

        def pair_loss(img):
            r = img[y0:y1 + 1, x0:x1 + 1].double() - tg[y0:y1 + 1, x0:x1 + 1]
            return float((r * r).sum())

        best_l, best_s = pair_loss(I), None
        for whole in (False, True):
            xc, yc, ac, wc = x.clone(), y.clone(), a.clone(), w.clone()
            xc[[i, j]], yc[[i, j]] = x[[j, i]], y[[j, i]]
            if whole:
                ac[[i, j]], wc[[i, j]] = a[[j, i]], w[[j, i]]
            Ic = model.render(xc, yc, ac, wc, glob).reshape(model.H, model.W)
            lc = pair_loss(Ic)
            if lc < best_l:
                best_l, best_s = lc, (xc, yc, ac, wc, Ic)
        if best_s is not None:
            x, y, a, w, I = best_s
            xn, yn, wn = (v.detach().cpu().numpy().astype(np.float64) for v in (x, y, w))
            moved += 2
    return x, y, a, w, moved


def particle_blocks(model: Model, I, x, y, a, w, glob, win: Windows, eps):
    """Gauss-Newton blocks J_i^T J_i [n, 4, 4] (sum of squared-residual convention:
    the curvature of sum r^2 / 2) from forward differences, one render per colour
    and parameter."""
    n = model.n
    A = torch.zeros((n, 4, 4), dtype=torch.float64, device=x.device)
    If = I.reshape(-1)
    for c, (members, _, _) in enumerate(win.colors):
        J = []
        for k, e in enumerate(eps):
            v = [x.clone(), y.clone(), a.clone(), w.clone()]
            v[k][members] += e
            J.append((model.render(*v, glob).reshape(-1) - If) / e)
        for p in range(4):
            for q in range(p, 4):
                s = win.sums(c, J[p] * J[q])
                A[members, p, q] = s[members]
                A[members, q, p] = s[members]
    return A


def global_block(model: Model, I, x, y, a, w, glob, eps_glob):
    If = I.reshape(-1).double()
    J = []
    for k, e in enumerate(eps_glob):
        g = glob.clone()
        g[k] += e
        J.append((model.render(x, y, a, w, g).reshape(-1).double() - If) / e)
    J = torch.stack(J)
    return J @ J.T


def _lm_solve(A, g, lam):
    """(A + lam diag(A) + tiny I) d = -g, batched over leading dimensions."""
    d = torch.diagonal(A, dim1=-2, dim2=-1)
    M = A + torch.diag_embed(lam * d + 1e-12 * (1.0 + d))
    return -torch.linalg.solve(M, g.unsqueeze(-1)).squeeze(-1)


def _pack(x, y, a, w, glob):
    return torch.cat([x, y, a, w, glob]).double()


def _unpack(v, n):
    v = v.float()
    return v[:n], v[n:2 * n], v[2 * n:3 * n], v[3 * n:4 * n], v[4 * n:4 * n + 4]


def gn_cg_step(model: Model, target, x, y, a, w, glob, I, win: Windows, pc: PolishConfig, lam: float):
    """One Gauss-Newton step by preconditioned conjugate gradients on
    (J^T J + lam D) d = -J^T r in scaled unknowns u = theta / sigma.  J v is a
    forward difference of the render along sigma v; J^T u is the adjoint; the
    preconditioner is the block diagonal (per-particle 4 x 4 blocks and the global
    block, from forward differences).  Returns the step d in natural units."""
    n, N = model.n, target.numel()
    sig = torch.cat([torch.full((n,), float(s_), device=x.device) for s_ in pc.scale] +
                    [torch.tensor(pc.scale_glob, device=x.device)]).double()
    theta = _pack(x, y, a, w, glob)
    If = I.reshape(-1)
    r = If - target.reshape(-1)

    def jt(u_img):  # J^T u in scaled unknowns
        gp, ggl = model.grad(x, y, a, w, glob, u_img.reshape(I.shape))
        return torch.cat([gp.reshape(-1), ggl]).double() * sig

    def jv(v):  # J v for v in scaled unknowns
        m = float(v.abs().max())
        if m == 0.0:
            return torch.zeros_like(If)
        e = pc.jvp_eps / m
        th = theta + e * sig * v
        return (model.render(*_unpack(th, n)).reshape(-1) - If) / e

    g = jt(r)
    # block-diagonal preconditioner in scaled unknowns
    A = particle_blocks(model, I, x, y, a, w, glob, win, pc.eps)
    sp = sig[:4 * n].reshape(4, n).T  # [n, 4]
    A = A * sp[:, :, None] * sp[:, None, :]
    Ag = global_block(model, I, x, y, a, w, glob, pc.eps_glob) * sig[4 * n:, None] * sig[None, 4 * n:]
    dA = torch.diagonal(A, dim1=-2, dim2=-1)
    dG = torch.diagonal(Ag)
    D = torch.cat([dA.T.reshape(-1), dG]).clamp_min(1e-30)
    Mp = A + torch.diag_embed(lam * dA + 1e-12 * (1.0 + dA))
    Mg = Ag + torch.diag(lam * dG + 1e-12 * (1.0 + dG))
    Mp_inv = torch.linalg.inv(Mp)
    Mg_inv = torch.linalg.inv(Mg)

    def precond(v):
        vp = v[:4 * n].reshape(4, n).T
        zp = (Mp_inv @ vp.unsqueeze(-1)).squeeze(-1).T.reshape(-1)
        zg = Mg_inv @ v[4 * n:]
        return torch.cat([zp, zg])

    def hv(v):
        return jt(jv(v)) + lam * D * v

    d = torch.zeros_like(g)
    res = -g
    z = precond(res)
    p = z.clone()
    rz = torch.dot(res, z)
    for _ in range(pc.cg_iters):
        q = hv(p)
        pq = torch.dot(p, q)
        if float(pq) <= 0.0:
            break
        alpha = rz / pq
        d = d + alpha * p
        res = res - alpha * q
        z = precond(res)
        rz_new = torch.dot(res, z)
        p = z + (rz_new / rz) * p
        rz = rz_new
    return d * sig


def polish(target: torch.Tensor, model: Model, x, y, a, w, glob, pc: PolishConfig = PolishConfig(),
           error_fn: Optional[Callable] = None, clock: Optional[Callable] = None):
    """Angle search, then Gauss-Newton steps (with the small prisms' angle search
    repeated every ``search_every`` steps) from (x, y, a, w, glob) (device tensors,
    returned updated), until the loss falls below ``loss_tol`` x mean(target^2) or
    after ``iters`` steps; then, above that floor, a closing fine search of the small
    prisms' angles and up to ``reseed_rounds`` times a re-seed (``reseed``) and the
    whole polish again.  error_fn(x, y, a, w, glob) -> e (float) is recorded after
    every stage when given (it only records; the loss alone decides when to stop);
    clock() -> seconds since the solve started.  Returns (x, y, a, w, glob, trace)."""
    N = target.numel()
    trace = []

    def record(tag):
        if error_fn is not None:
            trace.append((tag, clock() if clock else 0.0, error_fn(x, y, a, w, glob)))

    color, bounds = color_windows(x.detach().cpu().numpy(), y.detach().cpu().numpy(),
                                  w.detach().cpu().numpy(), model.H, model.W, pc.margin_px, pc.separation_px)
    win = Windows(color, bounds, model.H, model.W, x.device)
    span = pc.angle_span
    for r in range(1 + pc.angle_refine):
        a = angle_search(model, target, x, y, a, w, glob, win, span, pc.angle_steps)
        span /= 10.0
    record("angles")
    lam_p, lam_g = pc.lam0, pc.lam0
    I = model.render(x, y, a, w, glob)
    L = _loss(I, target)
    n = model.n
    for it in range(pc.iters):
        if pc.search_every and it > 0 and it % pc.search_every == 0:
            span = pc.research_span
            for r in range(1 + pc.research_refine):
                a = angle_search(model, target, x, y, a, w, glob, win, span, pc.angle_steps,
                                 only=w < pc.research_w_max)
                span /= 10.0
            I = model.render(x, y, a, w, glob)
            L = _loss(I, target)
        if pc.method == "cg":
            for _ in range(6):
                d = gn_cg_step(model, target, x, y, a, w, glob, I, win, pc, lam_p)
                xn, yn, an, wn, gn = _unpack(_pack(x, y, a, w, glob) + d, n)
                wn = torch.clamp(wn, min=1.0)
                In = model.render(xn, yn, an, wn, gn)
                Ln = _loss(In, target)
                if Ln < L:
                    x, y, a, w, glob, I, L = xn, yn, an, wn, gn, In, Ln
                    lam_p = max(lam_p / 3.0, 1e-9)
                    break
                lam_p *= 8.0
        else:
            # particle step (sum-of-squares scale: gradient of sum r^2 / 2 is N/2 dL/dtheta)
            gp, ggl = model.grad(x, y, a, w, glob, (2.0 / N) * (I - target))
            A = particle_blocks(model, I, x, y, a, w, glob, win, pc.eps)
            g = (gp.T.double() * (N / 2.0))
            for _ in range(6):
                d = _lm_solve(A, g, lam_p).float()
                xn, yn, an, wn = x + d[:, 0], y + d[:, 1], a + d[:, 2], torch.clamp(w + d[:, 3], min=1.0)
                In = model.render(xn, yn, an, wn, glob)
                Ln = _loss(In, target)
                if Ln < L:
                    x, y, a, w, I, L = xn, yn, an, wn, In, Ln
                    lam_p = max(lam_p / 3.0, 1e-7)
                    break
                lam_p *= 8.0
            # global step
            gp, ggl = model.grad(x, y, a, w, glob, (2.0 / N) * (I - target))
            Ag = global_block(model, I, x, y, a, w, glob, pc.eps_glob)
            gg = ggl.double() * (N / 2.0)
            for _ in range(6):
                dg = _lm_solve(Ag, gg, lam_g).float()
                gn = glob + dg
                In = model.render(x, y, a, w, gn)
                Ln = _loss(In, target)
                if Ln < L:
                    glob, I, L = gn, In, Ln
                    lam_g = max(lam_g / 3.0, 1e-7)
                    break
                lam_g *= 8.0
        record("lm%d loss %.3e" % (it, L))
        if L <= pc.loss_tol * float(torch.mean(target.double() ** 2)):
            break
    if pc.final_span > 0.0 and L > pc.loss_tol * float(torch.mean(target.double() ** 2)):
        # the repeated searches leave the small prisms' angles on a grid of
        # 2 research_span / ((angle_steps - 1) 10^research_refine), and the Gauss-Newton
        # steps barely move them; close with finer brackets
        span = pc.final_span
        for r in range(1 + pc.final_refine):
            a = angle_search(model, target, x, y, a, w, glob, win, span, pc.angle_steps,
                             only=w < pc.research_w_max)
            span /= 10.0
        I = model.render(x, y, a, w, glob)
        L = _loss(I, target)
        record("fine angles loss %.3e" % L)
    if pc.reseed_rounds > 0 and L > pc.loss_tol * float(torch.mean(target.double() ** 2)):
        x, y, a, w, moved = reseed(model, target, x, y, a, w, glob, pc)
        if moved:
            record("reseed %d" % moved)
            x, y, a, w, glob, more = polish(target, model, x, y, a, w, glob,
                                            replace(pc, reseed_rounds=pc.reseed_rounds - 1), error_fn, clock)
            trace += more
    return x, y, a, w, glob, trace
