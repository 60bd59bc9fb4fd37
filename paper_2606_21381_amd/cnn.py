"""Learned initializer for inverse rendering: a BF16 CNN on MFMA (libosog).

The network regresses the global optical parameters (dn, defocus, DIC shear,
DIC bias) of a DIC frame.  It is trained on crops the renderer itself produces
(one batch graph launch per training batch) with the library's own
forward, backward and Adam kernels; PyTorch only holds the buffers.

Target normalisation (zero-centred, about unit range over the training draw):
  dn: (dn - 0.03) / 0.02     dz: dz / 2     shear: (s - 1) / 0.2
  bias: (theta / (pi/2) - 1) / 0.2
"""
from __future__ import annotations

import ctypes
import math
import time
from typing import Optional

import numpy as np
import torch

from . import _lib, workloads
from .render import Batch, _ptr, _stream, context


# Network outputs per global: (g - centre) / scale.  Dn, shear and bias are scaled to
# their half-ranges; the defocus (dz ~ U[-2, 2] um) by 0.7 um instead of 2, which
# weights it (2 / 0.7)^2 ~ 8x in the squared loss: it is the global a single frame
# shows least (its depth of field is about its whole range), and with equal weights
# the trained network read it no better than the inverse problem's default start.
DZ_SCALE_UM = 0.7


def normalize(g: np.ndarray) -> np.ndarray:
    g = np.asarray(g, dtype=np.float64)
    return np.stack([(g[..., 0] - 0.03) / 0.02, g[..., 1] / DZ_SCALE_UM, (g[..., 2] - 1.0) / 0.2,
                     (g[..., 3] / (math.pi / 2) - 1.0) / 0.2], axis=-1)


def denormalize(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.float64)
    return np.stack([0.03 + 0.02 * z[..., 0], DZ_SCALE_UM * z[..., 1], 1.0 + 0.2 * z[..., 2],
                     (math.pi / 2) * (1.0 + 0.2 * z[..., 3])], axis=-1)


def param_count() -> int:
    c = ctypes.c_int64()
    _lib.check(_lib.load().osog_cnn_param_count(ctypes.byref(c)), "osog_cnn_param_count")
    return c.value


LAYERS = [(1, 32), (32, 32), (32, 64), (64, 64), (64, 128), (128, 128)]


def init_params(seed: int = 4) -> torch.Tensor:
    """He-normal convolutions, zero biases; Glorot-uniform dense layers (CPU, FP32)."""
    g = torch.Generator().manual_seed(seed)
    parts = []
    for ci, co in LAYERS:
        parts.append(torch.randn(9 * ci * co, generator=g) * math.sqrt(2.0 / (9 * ci)))
        parts.append(torch.zeros(co))
    for fi, fo in [(128, 64), (64, 4)]:
        lim = math.sqrt(6.0 / (fi + fo))
        parts.append((torch.rand(fi * fo, generator=g) * 2 - 1) * lim)
        parts.append(torch.zeros(fo))
    p = torch.cat(parts).float()
    assert p.numel() == param_count()
    return p


class LearnedInit:
    def __init__(self, device="cuda", seed: int = 4, batch: int = 256, crop: int = 256, n_max: int = 64):
        self.device = torch.device(device)
        self.lib = _lib.load()
        self.ctx = context(self.device)
        self.params = init_params(seed).to(self.device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.step_count = 0
        self.batch, self.crop, self.n_max = batch, crop, n_max
        self.seed = seed
        self._ws = {}

    # -- workspace --------------------------------------------------------------
    def _workspace(self, B, H, W):
        key = (B, H, W)
        if key not in self._ws:
            b = ctypes.c_size_t()
            _lib.check(self.lib.osog_cnn_workspace_size(B, H, W, ctypes.byref(b)), "osog_cnn_workspace_size")
            self._ws[key] = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        return self._ws[key]

    # -- network ------------------------------------------------------------------
    def forward(self, images: torch.Tensor) -> torch.Tensor:
        """Normalised predictions [B, 4] for images [B, H, W] (CUDA float32)."""
        images = images.contiguous()
        B, H, W = images.shape
        ws = self._workspace(B, H, W)
        pred = torch.empty((B, 4), dtype=torch.float32, device=self.device)
        _lib.check(self.lib.osog_cnn_forward(self.ctx, _stream(self.device), B, H, W, _ptr(images),
                                             _ptr(self.params), _ptr(pred), _ptr(ws), ws.numel()),
                   "osog_cnn_forward")
        return pred

    def train_step(self, images, targets, lr: float, grads_out: Optional[torch.Tensor] = None,
                   update: bool = True) -> torch.Tensor:
        images = images.contiguous()
        B, H, W = images.shape
        ws = self._workspace(B, H, W)
        loss = torch.empty(1, dtype=torch.float32, device=self.device)
        step = self.step_count + 1 if update else 0
        _lib.check(self.lib.osog_cnn_train_step(self.ctx, _stream(self.device), B, H, W, _ptr(images),
                                                _ptr(targets.contiguous()), _ptr(self.params), _ptr(self.m),
                                                _ptr(self.v), step, lr, _ptr(loss), _ptr(grads_out),
                                                _ptr(ws), ws.numel()), "osog_cnn_train_step")
        if update:
            self.step_count += 1
        return loss

    def predict(self, image: torch.Tensor) -> np.ndarray:
        """(dn, dz, shear, bias) for one frame [H, W] (fully convolutional + global pool)."""
        z = self.forward(image[None]).double().cpu().numpy()[0]
        return denormalize(z)

    # -- training data rendered by the engine -------------------------------------
    def _crop_source(self):
        """Fixed-shape batch of crops (padded particle tables) rendered by one batch graph launch."""
        B, S, N = self.batch, self.crop, self.n_max
        self.soa_dev = torch.zeros((B, 8, N), dtype=torch.float32, device=self.device)
        self.g_dev = torch.zeros((B, 4), dtype=torch.float32, device=self.device)
        self.images = torch.empty((B, S, S), dtype=torch.float32, device=self.device)
        opt = workloads.dic_optics(0.0)
        frames = [(self.soa_dev[b], S, S, opt, self.g_dev[b]) for b in range(B)]
        self.batch_renderer = Batch(frames, out=[self.images[b] for b in range(B)])

    def render_crops(self, rng: np.random.Generator):
        B, N = self.batch, self.n_max
        soa = np.zeros((B, 8, N), dtype=np.float32)
        g = np.zeros((B, 4), dtype=np.float32)
        tgt = np.zeros((B, 4), dtype=np.float64)
        for b in range(B):
            t, gl, truth = workloads.crop(rng, self.crop)
            n = min(N, t.shape[1])
            soa[b, :, :n] = t[:, :n]
            g[b] = gl
            tgt[b] = truth
        self.soa_dev.copy_(torch.from_numpy(soa))
        self.g_dev.copy_(torch.from_numpy(g))
        self.batch_renderer.run()
        return torch.from_numpy(normalize(tgt).astype(np.float32)).to(self.device)

    def train(self, samples: int = 200_000, lr: float = 1e-3, seed: Optional[int] = None, log=None):
        """Train on `samples` freshly rendered crops; returns (losses, seconds)."""
        if not hasattr(self, "batch_renderer"):
            self._crop_source()
        rng = np.random.Generator(np.random.PCG64(self.seed if seed is None else seed))
        steps = max(1, samples // self.batch)
        losses = []
        t0 = time.perf_counter()
        for k in range(steps):
            # cosine learning-rate schedule over the run
            lr_k = lr * 0.5 * (1 + math.cos(math.pi * k / steps))
            tgt = self.render_crops(rng)
            loss = self.train_step(self.images, tgt, lr_k)
            losses.append(loss)
            if log and (k % 50 == 0 or k == steps - 1):
                log(k, float(loss.item()))
        torch.cuda.synchronize(self.device)
        return torch.cat(losses).cpu().numpy(), time.perf_counter() - t0

    def evaluate(self, n: int = 1000, seed: int = 5):
        """Mean absolute error per global on n held-out crops (physical units)."""
        if not hasattr(self, "batch_renderer"):
            self._crop_source()
        rng = np.random.Generator(np.random.PCG64(seed))
        errs = []
        for _ in range(max(1, n // self.batch)):
            tgt = self.render_crops(rng)
            pred = self.forward(self.images)
            errs.append(np.abs(denormalize(pred.double().cpu().numpy()) - denormalize(tgt.double().cpu().numpy())))
        return np.concatenate(errs).mean(axis=0)


def _seed_globals(start, g):
    """Overwrite the four global parameters of an inverse-solve start in place."""
    with torch.no_grad():
        start.dn.fill_(float(g[0]))
        start.dz.fill_(float(g[1]))
        start.shear.fill_(float(g[2]))
        start.bias.fill_(float(g[3]))


def compare(device="cuda", samples: int = 200_000, n_targets: int = 10, target_seed0: int = 300,
            net: Optional["LearnedInit"] = None, cfg=None, pc=None, stall_loss: float = 1e-10, log=None) -> dict:
    """Learned-init against default-init inverse solves on 1024^2 DIC targets of 500 prisms.

    Both runs start every prism from the same perturbed position, angle and
    width and run the same solve (inverse.solve_hybrid: Adam, then the
    second-order polish); they differ only in the four globals: the default start
    perturbs them by x(1 + U[-0.2, 0.2]), the learned start takes the network's
    prediction on the full target frame.  Fallback to the plain solve from the
    default start: (a) when the image loss at the learned start exceeds the loss
    at the default start, before solving; (b) when the learned run stalls (its
    final mean squared image error stays above ``stall_loss`` x mean(target^2)
    while the default run's does not need to be known), after it -- its time then
    counts in full, plus the default solve's.  Returns training cost, held-out
    per-global error, per-target rows and the medians (over targets) of the time
    to e <= 1e-3 and to e_glob <= 1e-3 of each arm (inf when not reached).
    """
    from . import inverse
    from .render import render
    device = torch.device(device)
    if net is None:
        net = LearnedInit(device)
        losses, t_train = net.train(samples, log=log)
    else:
        losses, t_train = np.array([]), 0.0
    mae = net.evaluate()
    rows = []
    fallbacks_start, fallbacks_stall = 0, 0
    for k in range(n_targets):
        prob = workloads.config3(seed=target_seed0 + k)
        H, W, opt = prob.target.H, prob.target.W, prob.target.optics
        target, start_def, truth = inverse.problem_tensors(prob, device)
        _, start_cnn, _ = inverse.problem_tensors(prob, device)
        g_pred = net.predict(target)
        _seed_globals(start_cnn, g_pred)
        scale = float(torch.mean(target.double() ** 2))
        with torch.no_grad():
            l_def = float(torch.mean((render(start_def.soa(), H, W, opt, start_def.globals4()) - target) ** 2))
            l_cnn = float(torch.mean((render(start_cnn.soa(), H, W, opt, start_cnn.globals4()) - target) ** 2))
        r_def = inverse.solve_hybrid(target, start_def, truth, H, W, opt, cfg, pc)
        fb = "none"
        if l_cnn > l_def:
            fb = "start"
            fallbacks_start += 1
            r_cnn = r_def
            learned = _arm(r_def)
        else:
            r_cnn = inverse.solve_hybrid(target, start_cnn, truth, H, W, opt, cfg, pc)
            learned = _arm(r_cnn)
            if r_cnn.final_loss > stall_loss * scale:
                fb = "stall"
                fallbacks_stall += 1
                _, start_fb, _ = inverse.problem_tensors(prob, device)
                r_fb = inverse.solve_hybrid(target, start_fb, truth, H, W, opt, cfg, pc)
                learned = _arm(r_fb, offset=r_cnn.total_s)
        g_true = truth.globals4.double().cpu().numpy()
        rows.append({"seed": target_seed0 + k, "loss_start_default": l_def, "loss_start_learned": l_cnn,
                     "fallback": fb, "pred_abs_err": np.abs(g_pred - g_true).tolist(),
                     "default": _arm(r_def), "learned": learned})
        if log:
            log(k, rows[-1])

    def med(key):
        out = {}
        for arm in ("default", "learned"):
            v = [r[arm][key] if r[arm][key] is not None else math.inf for r in rows]
            out[arm] = float(np.median(v))
        return out

    rep = {"workload": "dic1024_n500 x %d targets (seeds %d..%d)" % (n_targets, target_seed0, target_seed0 + n_targets - 1),
           "train_samples": samples,
           "train_s": round(t_train, 2), "train_final_loss": float(losses[-20:].mean()) if len(losses) else None,
           "heldout_mae": dict(zip(("dn", "dz_um", "shear_px", "bias_rad"), map(float, mae))),
           "fallbacks_start": fallbacks_start, "fallbacks_stall": fallbacks_stall,
           "reached_1e-3": {arm: int(sum(r[arm]["time_to_1e-3_s"] is not None for r in rows)) for arm in ("default", "learned")},
           "targets": rows}
    for key in ("time_to_1e-3_s", "glob_time_to_1e-3_s", "final_e", "final_e_glob", "final_e_part", "total_s"):
        rep["median_" + key] = med(key)
    return rep


def _arm(r, offset: float = 0.0) -> dict:
    """Summary of one hybrid inverse solve (times shifted by `offset` seconds, the time
    a stalled learned run spent before its fallback)."""
    def sh(t):
        return None if t is None else t + offset
    return {"time_to_1e-3_s": sh(r.time_to_target_s), "glob_time_to_1e-3_s": sh(r.time_to_glob_target_s),
            "final_e": r.final_e, "final_e_glob": r.final_e_glob, "final_e_part": r.final_e_part,
            "final_loss": r.final_loss, "total_s": r.total_s + offset,
            "adam_e_glob_at_60": float(r.adam.error_glob[min(60, r.adam.steps)])}


STRIDES = (2, 1, 2, 1, 2, 2)  # stride of each layer of LAYERS


def conv_flops(crop: int) -> float:
    """Multiply-add FLOPs (2 per product) of one crop's training step in the
    convolutions: forward, input gradient (every layer but the first) and weight
    gradient, each one implicit GEMM of (pixels) x (9 Ci) x (Co)."""
    side, fwd, dgrad = crop, 0.0, 0.0
    for k, ((ci, co), s) in enumerate(zip(LAYERS, STRIDES)):
        side //= s
        f = 2.0 * side * side * 9 * ci * co
        fwd += f
        dgrad += f if k > 0 else 0.0
    return 2.0 * fwd + dgrad  # forward + weight gradient + input gradient


def main(argv=None) -> int:
    """Train the initializer on engine-rendered crops, or time its forward + backward."""
    import argparse
    import json
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--samples", type=int, default=200_000, help="crops to train on (0: skip training)")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--crop", type=int, default=256)
    ap.add_argument("--time-steps", type=int, default=0,
                    help="also time this many forward + backward passes of one rendered batch "
                         "(no rendering and no parameter update in the loop)")
    args = ap.parse_args(argv)
    dev = torch.device("cuda", 0)
    net = LearnedInit(dev, batch=args.batch, crop=args.crop)
    out = {"batch": args.batch, "crop": args.crop}
    if args.samples > 0:
        losses, secs = net.train(args.samples)
        out.update(samples=args.samples, train_s=round(secs, 2), final_loss=float(losses[-20:].mean()))
    if args.time_steps > 0:
        rng = np.random.Generator(np.random.PCG64(net.seed))
        if not hasattr(net, "batch_renderer"):
            net._crop_source()
        tgt = net.render_crops(rng)
        for _ in range(3):
            net.train_step(net.images, tgt, 0.0, update=False)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.time_steps):
            net.train_step(net.images, tgt, 0.0, update=False)
        e1.record()
        torch.cuda.synchronize(dev)
        ms = e0.elapsed_time(e1) / args.time_steps
        fl = conv_flops(args.crop) * args.batch
        out.update(fwd_bwd_ms=round(ms, 3), conv_gflop_per_batch=round(fl / 1e9, 1),
                   conv_tflops_over_fwd_bwd=round(fl / (ms * 1e-3) / 1e12, 1))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
