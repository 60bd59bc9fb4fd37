"""FP64 CPU oracle of the learned initializer's network -- TEST INFRASTRUCTURE ONLY.

The network the GPU library trains (a small convolutional regressor of the four
global optical parameters), stated plainly in float64 PyTorch on the CPU with
its gradients from autograd.  It shares no code with the GPU path: the layer
list and the parameter layout below are the interface both sides implement.

Network: 3x3 convolutions with padding 1, each followed by bias and ReLU,
channels 1->32 (stride 2), 32->32, 32->64 (stride 2), 64->64, 64->128 (stride 2),
128->128 (stride 2); global average pooling; dense 128->64 with ReLU; dense
64->4.  The input image I enters as x = I / 4 - 1.

Parameter vector (float32 on the device, widened here), in order, for each
convolution: W[3][3][Ci][Co] then bias[Co]; then W7[128][64], b7[64], W8[64][4], b8[4].
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as Fn

LAYERS = ((1, 32, 2), (32, 32, 1), (32, 64, 2), (64, 64, 1), (64, 128, 2), (128, 128, 2))


def param_count() -> int:
    n = sum(9 * ci * co + co for ci, co, _ in LAYERS)
    return n + 128 * 64 + 64 + 64 * 4 + 4


def conv3x3(x: torch.Tensor, w: torch.Tensor, bias: torch.Tensor, stride: int) -> torch.Tensor:
    """out[b, co, oy, ox] = bias[co] + sum over (ky, kx, ci) of
    x[b, ci, oy*stride - 1 + ky, ox*stride - 1 + kx] * w[ky, kx, ci, co], zero outside.
    x is NCHW, w is [3][3][Ci][Co]; a library convolution is the step."""
    return Fn.conv2d(x, w.permute(3, 2, 0, 1), bias, stride=stride, padding=1)


def conv3x3_loops(x: np.ndarray, w: np.ndarray, bias: np.ndarray, stride: int) -> np.ndarray:
    """The same sum by explicit loops (tiny inputs only): an independent statement."""
    B, Ci, H, W = x.shape
    Co = w.shape[3]
    Ho, Wo = (H + 2 - 3) // stride + 1, (W + 2 - 3) // stride + 1
    out = np.zeros((B, Co, Ho, Wo))
    for b in range(B):
        for co in range(Co):
            for oy in range(Ho):
                for ox in range(Wo):
                    s = bias[co]
                    for ky in range(3):
                        for kx in range(3):
                            iy, ix = oy * stride - 1 + ky, ox * stride - 1 + kx
                            if 0 <= iy < H and 0 <= ix < W:
                                s += float(np.dot(x[b, :, iy, ix], w[ky, kx, :, co]))
                    out[b, co, oy, ox] = s
    return out


def unpack(params: torch.Tensor):
    """Split the parameter vector into (conv weights, conv biases, W7, b7, W8, b8)."""
    p = params.double()
    off = 0
    ws, bs = [], []
    for ci, co, _ in LAYERS:
        ws.append(p[off:off + 9 * ci * co].view(3, 3, ci, co))
        off += 9 * ci * co
        bs.append(p[off:off + co])
        off += co
    W7 = p[off:off + 128 * 64].view(128, 64); off += 128 * 64
    b7 = p[off:off + 64]; off += 64
    W8 = p[off:off + 64 * 4].view(64, 4); off += 64 * 4
    b8 = p[off:off + 4]; off += 4
    assert off == p.numel()
    return ws, bs, W7, b7, W8, b8


def network(params: torch.Tensor, images: torch.Tensor) -> torch.Tensor:
    """Predictions [B, 4] of the network for images [B, H, W] (float64, CPU)."""
    ws, bs, W7, b7, W8, b8 = unpack(params)
    x = (images.double() * 0.25 - 1.0)[:, None]
    for (ci, co, stride), w, b in zip(LAYERS, ws, bs):
        x = torch.relu(conv3x3(x, w, b, stride))
    pool = x.mean(dim=(2, 3))
    return torch.relu(pool @ W7 + b7) @ W8 + b8


def loss_and_grad(params: torch.Tensor, images: torch.Tensor, targets: torch.Tensor):
    """(mean squared error over the B x 4 outputs, its gradient wrt the parameters)."""
    p = params.detach().double().clone().requires_grad_(True)
    loss = ((network(p, images) - targets.double()) ** 2).mean()
    loss.backward()
    return float(loss), p.grad.detach()
