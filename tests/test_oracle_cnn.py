"""Pins of the CNN oracle: the convolution against explicit loops, the
parameter layout, and the autograd gradient against central finite differences."""
import numpy as np
import torch

import oracle.cnn as oc


def test_conv3x3_matches_explicit_loops():
    rng = np.random.default_rng(0)
    for stride, (B, Ci, H, W, Co) in ((1, (2, 3, 5, 4, 2)), (2, (1, 2, 6, 7, 3))):
        x = rng.standard_normal((B, Ci, H, W))
        w = rng.standard_normal((3, 3, Ci, Co))
        b = rng.standard_normal(Co)
        ref = oc.conv3x3_loops(x, w, b, stride)
        got = oc.conv3x3(torch.from_numpy(x), torch.from_numpy(w), torch.from_numpy(b), stride).numpy()
        assert got.shape == ref.shape
        assert np.abs(got - ref).max() < 1e-12


def test_param_count_and_layout():
    n = oc.param_count()
    assert n == 294948
    p = torch.arange(n, dtype=torch.float64)
    ws, bs, W7, b7, W8, b8 = oc.unpack(p)
    assert ws[0].shape == (3, 3, 1, 32) and float(ws[0][0, 0, 0, 1]) == 1.0   # W[ky][kx][ci][co], co fastest
    assert float(bs[0][0]) == 9 * 32 and float(ws[1][0, 0, 0, 0]) == 9 * 32 + 32
    assert float(b8[-1]) == n - 1 and W7.shape == (128, 64)


def test_gradient_matches_central_differences():
    g = torch.Generator().manual_seed(1)
    n = oc.param_count()
    params = torch.randn(n, generator=g, dtype=torch.float64) * 0.1
    images = 4.0 + torch.randn(2, 32, 32, generator=g, dtype=torch.float64)
    targets = torch.randn(2, 4, generator=g, dtype=torch.float64)
    L, grad = oc.loss_and_grad(params, images, targets)
    idx = [0, 5, 300, 9300, n - 1, n - 300, n - 8300]
    for i in idx:
        h = 1e-6
        pp, pm = params.clone(), params.clone()
        pp[i] += h
        pm[i] -= h
        lp = float(((oc.network(pp, images) - targets) ** 2).mean())
        lm = float(((oc.network(pm, images) - targets) ** 2).mean())
        fd = (lp - lm) / (2 * h)
        assert abs(fd - float(grad[i])) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (i, fd, float(grad[i]))
