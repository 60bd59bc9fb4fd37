"""Python face of libosog: render(), render_backward(), RenderFn, bin_pairs(), batch_render().

PyTorch supplies device memory and the current stream; every computation runs
in libosog's HIP kernels through the C ABI.  There is no CPU fallback: if the
library or a GPU is missing these functions raise.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib

_contexts = {}


def context(device: Optional[torch.device] = None):
    """The library context of a CUDA (HIP) device, created on first use."""
    dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    ctx = _contexts.get(idx)
    if ctx is None:
        lib = _lib.load()
        p = ctypes.c_void_p()
        _lib.check(lib.osog_context_create(ctypes.byref(p), idx), "osog_context_create")
        ctx = p
        _contexts[idx] = ctx
    return ctx


def set_tiling(tile_h: int, tile_w: int, device=None):
    _lib.check(_lib.load().osog_set_tiling(context(device), tile_h, tile_w), "osog_set_tiling")


def get_tiling(device=None):
    h, w = ctypes.c_int32(), ctypes.c_int32()
    _lib.check(_lib.load().osog_get_tiling(context(device), ctypes.byref(h), ctypes.byref(w)),
               "osog_get_tiling")
    return h.value, w.value


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def soa_rows(optics) -> int:
    """Rows of the particle table these optics expect (9 with absorption)."""
    return 9 if getattr(optics, "absorption", 0) else 8


def _planes(optics) -> int:
    """Planes of the OPD output (OPD, and the absorbance with absorption)."""
    return 2 if getattr(optics, "absorption", 0) else 1


def _opd_tensor(optics, H: int, W: int, device) -> torch.Tensor:
    shape = (2, H, W) if _planes(optics) == 2 else (H, W)
    return torch.empty(shape, dtype=torch.float32, device=device)


def _check_soa(soa: torch.Tensor, rows: int = 8):
    if soa.dim() != 2 or soa.shape[0] != rows or soa.dtype != torch.float32 or not soa.is_cuda:
        raise ValueError("soa must be a CUDA float32 tensor of shape [%d, n]" % rows)
    if soa.shape[1] > 0 and soa.stride(1) != 1:
        raise ValueError("soa rows must be contiguous")
    n = soa.shape[1]
    ld = soa.stride(0) if n > 0 else 0
    return n, max(ld, n)


def _check_globals(g: torch.Tensor, device):
    if g.dtype != torch.float32 or g.numel() != 4 or not g.is_cuda or not g.is_contiguous():
        raise ValueError("globals must be a contiguous CUDA float32 tensor of 4 values")
    return g


def workspace_size(H: int, W: int, n: int, with_backward: bool = False, pairs_per_particle: int = 0,
                   device=None) -> int:
    b = ctypes.c_size_t()
    _lib.check(_lib.load().osog_workspace_size(context(device), H, W, n, pairs_per_particle,
                                               1 if with_backward else 0, ctypes.byref(b)),
               "osog_workspace_size")
    return b.value


_ws_cache = {}


def _workspace(nbytes: int, device) -> torch.Tensor:
    """A device byte buffer of at least nbytes, reused across calls on a stream."""
    key = (torch.device(device).index, torch.cuda.current_stream(device).cuda_stream)
    buf = _ws_cache.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(nbytes, dtype=torch.uint8, device=device)
        _ws_cache[key] = buf
    return buf


def render(soa: torch.Tensor, H: int, W: int, optics, globals4: torch.Tensor, want_opd: bool = False,
           out: Optional[torch.Tensor] = None, opd_out: Optional[torch.Tensor] = None,
           workspace: Optional[torch.Tensor] = None, pairs_per_particle: int = 0):
    """Render one frame.  Returns intensity [H, W] (and the OPD canvas if want_opd:
    [H, W], or [2, H, W] = OPD and absorbance with absorption)."""
    device = soa.device
    n, ld = _check_soa(soa, soa_rows(optics))
    _check_globals(globals4, device)
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=device)
    if want_opd and opd_out is None:
        opd_out = _opd_tensor(optics, H, W, device)
    if opd_out is not None and opd_out.numel() != _planes(optics) * H * W:
        raise ValueError("opd_out must hold %d plane(s) of H x W" % _planes(optics))
    # the incoherent DIC (mode 3) needs the larger workspace
    nb = workspace_size(H, W, n, int(optics.mode) == 3, pairs_per_particle, device)
    ws = workspace if workspace is not None else _workspace(nb, device)
    o = _lib.make_optics(optics)
    lib = _lib.load()
    _lib.check(lib.osog_render(context(device), _stream(device), H, W, _ptr(soa) if n else None, n, ld,
                               ctypes.byref(o), _ptr(globals4), _ptr(opd_out), _ptr(out), _ptr(ws),
                               ws.numel()), "osog_render")
    return (out, opd_out) if want_opd else out


def render_noalloc(soa: torch.Tensor, H: int, W: int, optics, globals4: torch.Tensor,
                   out: torch.Tensor, opd_out: Optional[torch.Tensor] = None):
    """osog_render_noalloc: the frame of render() in the library's fixed device scratch,
    with no workspace and no device allocation (out, and opd_out if given, are the
    caller's).  Calls on one GPU share that scratch: they must not overlap."""
    device = soa.device
    n, ld = _check_soa(soa, soa_rows(optics))
    _check_globals(globals4, device)
    if out.shape != (H, W) or out.dtype != torch.float32 or out.device != device or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 [H, W] tensor on the particle table's device")
    if opd_out is not None and opd_out.numel() != _planes(optics) * H * W:
        raise ValueError("opd_out must hold %d plane(s) of H x W" % _planes(optics))
    o = _lib.make_optics(optics)
    _lib.check(_lib.load().osog_render_noalloc(context(device), _stream(device), H, W, _ptr(soa) if n else None,
                                                n, ld, ctypes.byref(o), _ptr(globals4), _ptr(opd_out), _ptr(out)),
               "osog_render_noalloc")
    return out


def render_multi(soa: torch.Tensor, H: int, W: int, optics_list, globals_modes: torch.Tensor,
                 want_opd: bool = False, out=None, workspace: Optional[torch.Tensor] = None):
    """Several modalities of one particle table, pixel-aligned (one binning, raster
    and row FFT): list of intensities [H, W] (and the OPD if want_opd).
    ``globals_modes``: CUDA float32 [n_modes, 4]."""
    device = soa.device
    n, ld = _check_soa(soa, soa_rows(optics_list[0]))
    m = len(optics_list)
    g = globals_modes.contiguous()
    if g.shape != (m, 4) or g.dtype != torch.float32 or g.device != device:
        raise ValueError("globals_modes must be a float32 [n_modes, 4] tensor on the particle table's device")
    outs = out if out is not None else [torch.empty((H, W), dtype=torch.float32, device=device) for _ in range(m)]
    opd = _opd_tensor(optics_list[0], H, W, device) if want_opd else None
    nb = workspace_size(H, W, n, True, 0, device)
    ws = workspace if workspace is not None else _workspace(nb, device)
    opts = (_lib.Optics * m)(*[_lib.make_optics(o) for o in optics_list])
    ptrs = (ctypes.c_void_p * m)(*[o.data_ptr() for o in outs])
    _lib.check(_lib.load().osog_render_multi(context(device), _stream(device), H, W, _ptr(soa) if n else None,
                                              n, ld, m, opts, _ptr(g), ptrs, _ptr(opd), _ptr(ws), ws.numel()),
               "osog_render_multi")
    return (outs, opd) if want_opd else outs


def render_backward(soa: torch.Tensor, H: int, W: int, optics, globals4: torch.Tensor,
                    grad_intensity: torch.Tensor, grad_opd: Optional[torch.Tensor] = None,
                    need_soa: bool = True, need_globals: bool = True,
                    workspace: Optional[torch.Tensor] = None):
    """Adjoint of the noiseless render: (grad_soa [rows, n] or None, grad_globals [4] or None).
    With absorption the table and grad_soa have 9 rows and grad_opd (if given) is
    [2, H, W]: dL/dOPD and dL/dtau."""
    device = soa.device
    rows = soa_rows(optics)
    n, ld = _check_soa(soa, rows)
    _check_globals(globals4, device)
    gi = grad_intensity.contiguous()
    go = grad_opd.contiguous() if grad_opd is not None else None
    if go is not None and go.numel() != _planes(optics) * H * W:
        raise ValueError("grad_opd must hold %d plane(s) of H x W" % _planes(optics))
    gs = torch.empty((rows, ld), dtype=torch.float32, device=device) if (need_soa and n) else None
    gg = torch.empty(4, dtype=torch.float32, device=device) if need_globals else None
    nb = workspace_size(H, W, n, True, 0, device)
    ws = workspace if workspace is not None else _workspace(nb, device)
    o = _lib.make_optics(optics)
    _lib.check(_lib.load().osog_render_backward(context(device), _stream(device), H, W,
                                                 _ptr(soa) if n else None, n, ld, ctypes.byref(o),
                                                 _ptr(globals4), _ptr(gi), _ptr(go), _ptr(gs), _ptr(gg),
                                                 _ptr(ws), ws.numel()), "osog_render_backward")
    if gs is not None and ld != n:
        gs = gs[:, :n]
    return gs, gg


class RenderFn(torch.autograd.Function):
    """I = render(soa, globals) with the library's hand-written adjoint as backward.

    Only (soa, globals) are saved; the backward recomputes the forward
    intermediates inside the library.  Shot noise is treated as a constant.
    """

    @staticmethod
    def forward(ctx, soa, globals4, H, W, optics):
        I = render(soa.detach(), H, W, optics, globals4.detach())
        ctx.save_for_backward(soa, globals4)
        ctx.H, ctx.W, ctx.optics = H, W, optics
        return I

    @staticmethod
    def backward(ctx, grad_I):
        soa, globals4 = ctx.saved_tensors
        gs, gg = render_backward(soa.detach(), ctx.H, ctx.W, ctx.optics, globals4.detach(),
                                 grad_I, None, ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        return gs, gg, None, None, None


def render_diff(soa: torch.Tensor, globals4: torch.Tensor, H: int, W: int, optics) -> torch.Tensor:
    """Differentiable render (autograd through the HIP adjoint)."""
    return RenderFn.apply(soa, globals4, H, W, optics)


def bin_pairs(soa: torch.Tensor, H: int, W: int, capacity: Optional[int] = None):
    """Binning steps only: (keys, pids, tile_start, counts, pair_count) as CUDA int32 tensors.
    Binning reads the first 8 rows, so an absorbing table (9 rows) is accepted too."""
    device = soa.device
    n, ld = _check_soa(soa, 9 if soa.dim() == 2 and soa.shape[0] == 9 else 8)
    th, tw = get_tiling(device)
    n_tiles = (H // th) * (W // tw)
    if capacity is None:
        capacity = 32 * max(n, 1) + n_tiles
    keys = torch.empty(max(capacity, 1), dtype=torch.int32, device=device)
    pids = torch.empty_like(keys)
    ts = torch.empty(n_tiles + 1, dtype=torch.int32, device=device)
    counts = torch.empty(max(n, 1), dtype=torch.int32, device=device)
    pc = torch.empty(1, dtype=torch.int32, device=device)
    nb = workspace_size(H, W, n, False, max(1, (capacity + max(n, 1) - 1) // max(n, 1)), device)
    ws = _workspace(nb, device)
    _lib.check(_lib.load().osog_bin(context(device), _stream(device), H, W, _ptr(soa) if n else None, n, ld,
                                     _ptr(keys), _ptr(pids), capacity, _ptr(pc), _ptr(ts), _ptr(counts),
                                     _ptr(ws), ws.numel()), "osog_bin")
    P = int(pc.item())
    return keys[:P], pids[:P], ts, counts[:n], P


def band_columns(H: int, W: int, optics, device=None) -> int:
    """Number of in-band spectrum columns the chain carries for these optics."""
    lo, nn = ctypes.c_int32(), ctypes.c_int32()
    o = _lib.make_optics(optics)
    _lib.check(_lib.load().osog_band_info(context(device), H, W, ctypes.byref(o), ctypes.byref(lo),
                                           ctypes.byref(nn)), "osog_band_info")
    return nn.value


def philox(ctr: torch.Tensor, key0: int, key1: int) -> torch.Tensor:
    """Philox4x32-10 of a CUDA int32/uint32 counter tensor [m, 4] (device)."""
    c = ctr.contiguous()
    out = torch.empty_like(c)
    _lib.check(_lib.load().osog_philox4x32_10(_stream(c.device), _ptr(c), c.shape[0], key0 & 0xFFFFFFFF,
                                               key1 & 0xFFFFFFFF, _ptr(out)), "osog_philox4x32_10")
    return out


class Batch:
    """A batch of frames rendered by one HIP graph launch (one kernel chain per frame).

    ``frames``: list of (soa [8 or 9, n] CUDA float32, H, W, optics, globals [4] CUDA float32).
    Outputs are allocated once; ``run()`` re-renders into them (replaying the
    captured graph after the first call) and returns the outputs.
    """

    def __init__(self, frames, want_opd: bool = False, pairs_per_particle: int = 0, device=None, out=None):
        self.device = frames[0][0].device if device is None else torch.device(device)
        self.lib = _lib.load()
        self.ctx = context(self.device)
        self.inputs = frames
        self.out = out if out is not None else [torch.empty((H, W), dtype=torch.float32, device=self.device)
                                                for (_, H, W, _, _) in frames]
        self.opd = [_opd_tensor(o, H, W, self.device) if want_opd else None for (_, H, W, o, _) in frames]
        n = len(frames)
        self.c_frames = (_lib.Frame * n)()
        for f, (soa, H, W, optics, g) in enumerate(frames):
            nn, ld = _check_soa(soa, soa_rows(optics))
            _check_globals(g, self.device)
            fr = self.c_frames[f]
            fr.height, fr.width = H, W
            fr.soa = soa.data_ptr() if nn else None
            fr.n, fr.ld = nn, ld
            fr.optics = _lib.make_optics(optics)
            fr.globals = g.data_ptr()
            fr.opd_out = self.opd[f].data_ptr() if want_opd else None
            fr.intensity_out = self.out[f].data_ptr()
        b = ctypes.c_size_t()
        _lib.check(self.lib.osog_batch_workspace_size(self.ctx, self.c_frames, n, pairs_per_particle,
                                                      ctypes.byref(b)), "osog_batch_workspace_size")
        self.ws = torch.empty(b.value, dtype=torch.uint8, device=self.device)
        self.done_ns = torch.zeros(n + 1, dtype=torch.int64, device=self.device)

    def run(self):
        _lib.check(self.lib.osog_batch_render(self.ctx, _stream(self.device), self.c_frames, len(self.inputs),
                                              _ptr(self.ws), self.ws.numel(), _ptr(self.done_ns)),
                   "osog_batch_render")
        return self.out

    def error_flag(self) -> int:
        f = ctypes.c_int32()
        _lib.check(self.lib.osog_batch_error(self.ctx, _ptr(self.ws), ctypes.byref(f)), "osog_batch_error")
        return f.value

    def latencies_ms(self):
        """Per-frame completion time after the launch started, ms (after a sync)."""
        t = self.done_ns.cpu().numpy().astype("float64")
        return (t[:-1] - t[-1]) / 1e6


def set_batch_group(group: int, device=None):
    _lib.check(_lib.load().osog_set_batch_group(context(device), group), "osog_set_batch_group")


def set_size_tiling(H: int, W: int, tile_h: int, tile_w: int, device=None):
    _lib.check(_lib.load().osog_set_size_tiling(context(device), H, W, tile_h, tile_w), "osog_set_size_tiling")


# ---- spectral loss of Eq. 8 -------------------------------------------------------
def _spectral_ws(H: int, W: int, device, workspace=None) -> torch.Tensor:
    b = ctypes.c_size_t()
    _lib.check(_lib.load().osog_spectral_workspace_size(H, W, ctypes.byref(b)), "osog_spectral_workspace_size")
    return workspace if workspace is not None else _workspace(b.value, device)


def spectral_target(target: torch.Tensor, eps: float, workspace=None) -> torch.Tensor:
    """log(|DFT(target)| + eps) in the library's spectrum layout (float32 [H * W])."""
    t = target.contiguous()
    if t.dim() != 2 or t.dtype != torch.float32 or not t.is_cuda:
        raise ValueError("target must be a CUDA float32 [H, W] tensor")
    H, W = t.shape
    out = torch.empty(H * W, dtype=torch.float32, device=t.device)
    ws = _spectral_ws(H, W, t.device, workspace)
    _lib.check(_lib.load().osog_spectral_target(context(t.device), _stream(t.device), H, W, _ptr(t), float(eps),
                                                 _ptr(out), _ptr(ws), ws.numel()), "osog_spectral_target")
    return out


def spectral_loss(image: torch.Tensor, target_logamp: torch.Tensor, eps: float, want_grad: bool = True,
                  workspace=None):
    """(loss as a CUDA float32 [1] tensor, dL/dimage [H, W] or None) of Eq. 8's spectral loss."""
    im = image.contiguous()
    if im.dim() != 2 or im.dtype != torch.float32 or not im.is_cuda:
        raise ValueError("image must be a CUDA float32 [H, W] tensor")
    H, W = im.shape
    if target_logamp.numel() != H * W:
        raise ValueError("target_logamp must come from spectral_target of an H x W target")
    loss = torch.empty(1, dtype=torch.float32, device=im.device)
    grad = torch.empty((H, W), dtype=torch.float32, device=im.device) if want_grad else None
    ws = _spectral_ws(H, W, im.device, workspace)
    _lib.check(_lib.load().osog_spectral_loss(context(im.device), _stream(im.device), H, W, _ptr(im),
                                               _ptr(target_logamp), float(eps), _ptr(loss), _ptr(grad), _ptr(ws),
                                               ws.numel()), "osog_spectral_loss")
    return loss, grad


class SpectralLossFn(torch.autograd.Function):
    """L = spectral loss of Eq. 8 (image against a fixed target's log amplitudes),
    with the library's gradient image as backward."""

    @staticmethod
    def forward(ctx, image, target_logamp, eps):
        loss, grad = spectral_loss(image.detach(), target_logamp, eps, want_grad=image.requires_grad)
        ctx.save_for_backward(grad if grad is not None else loss)
        return loss[0]

    @staticmethod
    def backward(ctx, g):
        (grad,) = ctx.saved_tensors
        return grad * g, None, None


def spectral_loss_diff(image: torch.Tensor, target_logamp: torch.Tensor, eps: float) -> torch.Tensor:
    return SpectralLossFn.apply(image, target_logamp, eps)


# ---- polyhedral habits (Eq. 1) --------------------------------------------------
def set_habits(habits, topo_seed: int = 0, device=None):
    """Install the context's polyhedral habits: a list of objects with ``faces``
    ([M][4]: n_x, n_y, n_z, d), ``radius``, ``topo_amplitude_um`` and ``topo_cell_px``.
    Particles with table row 7 = 2 + k use habit k."""
    import numpy as np
    n = len(habits)
    counts = (ctypes.c_int32 * max(n, 1))(*[int(np.asarray(h.faces).shape[0]) for h in habits])
    flat = np.ascontiguousarray(np.concatenate([np.asarray(h.faces, dtype=np.float32).reshape(-1) for h in habits])
                                if n else np.zeros(4, np.float32))
    rad = (ctypes.c_float * max(n, 1))(*[float(h.radius) for h in habits])
    amp = (ctypes.c_float * max(n, 1))(*[float(h.topo_amplitude_um) for h in habits])
    cell = (ctypes.c_float * max(n, 1))(*[float(h.topo_cell_px) for h in habits])
    _lib.check(_lib.load().osog_set_habits(context(device), n, counts, flat.ctypes.data_as(ctypes.c_void_p), rad,
                                            amp, cell, int(topo_seed) & 0xFFFFFFFFFFFFFFFF), "osog_set_habits")
