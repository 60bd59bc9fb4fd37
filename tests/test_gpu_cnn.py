"""The learned initializer's MFMA convolutions against float64 PyTorch on the CPU,
full-network predictions and gradients against the CPU oracle (oracle/cnn.py),
a short training run on crops the renderer produces, and what the trained
network gains over the default start of the inverse problem."""
import ctypes
import math

import numpy as np
import pytest
import torch
import torch.nn.functional as Fn

from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def bf16_bits(t):
    return t.to(torch.bfloat16).view(torch.int16)


def bits_to_f64(b):
    return b.view(torch.bfloat16).double()


def conv_call(mode, B, H, W, Ci, Co, s, x=None, y=None, gy=None, w=None, bias=None):
    from paper_2606_21381_amd import _lib, render
    lib = _lib.load()
    ctx = render.context()
    Ho, Wo = (H // 2, W // 2) if s == 2 else (H, W)
    nb = ctypes.c_size_t()
    _lib.check(lib.osog_conv3x3_workspace_size(mode, B, H, W, Ci, Co, s, ctypes.byref(nb)), "ws")
    ws = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr()) if t is not None else None
    if mode == 0:
        out = torch.empty((B, Ho, Wo, Co), dtype=torch.int16, device="cuda")
        _lib.check(lib.osog_conv3x3(ctx, None, 0, B, H, W, Ci, Co, s, p(x), None, None, p(w), p(bias), p(out), None,
                                    p(ws), ws.numel()), "conv fwd")
    elif mode == 1:
        out = torch.empty((B, H, W, Ci), dtype=torch.int16, device="cuda")
        _lib.check(lib.osog_conv3x3(ctx, None, 1, B, H, W, Ci, Co, s, None, p(y), p(gy), p(w), None, p(out), None,
                                    p(ws), ws.numel()), "conv dgrad")
    else:
        out = torch.empty((3, 3, Ci, Co), dtype=torch.float32, device="cuda")
        _lib.check(lib.osog_conv3x3(ctx, None, 2, B, H, W, Ci, Co, s, p(x), p(y), p(gy), None, None, None, p(out),
                                    p(ws), ws.numel()), "conv wgrad")
    torch.cuda.synchronize()
    return out


def rel(a, b):
    return float((a - b).norm() / b.norm())


@pytest.mark.parametrize("B,H,W,Ci,Co,s", [(2, 16, 16, 1, 32, 2), (3, 20, 12, 32, 32, 1), (2, 16, 16, 32, 64, 2),
                                           (1, 8, 8, 128, 128, 2), (2, 12, 16, 64, 64, 1)])
def test_conv_modes_vs_float64(B, H, W, Ci, Co, s):
    need_gpu()
    g = torch.Generator().manual_seed(B * 100 + Ci)
    x = torch.randn(B, H, W, Ci, generator=g)
    w = torch.randn(3, 3, Ci, Co, generator=g) / math.sqrt(9 * Ci)
    bias = torch.randn(Co, generator=g) * 0.1
    xb, wb = bf16_bits(x), bf16_bits(w)
    X = bits_to_f64(xb).permute(0, 3, 1, 2)
    Wt = bits_to_f64(wb).permute(3, 2, 0, 1).contiguous()
    ref = torch.relu(Fn.conv2d(X, Wt, bias.double(), stride=s, padding=1))
    y = conv_call(0, B, H, W, Ci, Co, s, x=xb.cuda(), w=wb.cuda(), bias=bias.cuda())
    Y = bits_to_f64(y.cpu()).permute(0, 3, 1, 2)
    e_f = rel(Y, ref)
    # gradients through the ReLU of this layer's output
    gy = torch.randn(Y.shape[0], Y.shape[2], Y.shape[3], Co, generator=g)
    gyb = bf16_bits(gy)
    gz = bits_to_f64(gyb).permute(0, 3, 1, 2) * (Y > 0)
    ref_dx = torch.nn.grad.conv2d_input(X.shape, Wt, gz, stride=s, padding=1)
    ref_dw = torch.nn.grad.conv2d_weight(X, Wt.shape, gz, stride=s, padding=1)
    dx = conv_call(1, B, H, W, Ci, Co, s, y=y, gy=gyb.cuda(), w=wb.cuda())
    dw = conv_call(2, B, H, W, Ci, Co, s, x=xb.cuda(), y=y, gy=gyb.cuda())
    e_dx = rel(bits_to_f64(dx.cpu()).permute(0, 3, 1, 2), ref_dx)
    e_dw = rel(dw.cpu().double().permute(3, 2, 0, 1), ref_dw)
    say("conv B%d %dx%d %d->%d s%d: fwd %.2e dgrad %.2e wgrad %.2e" % (B, H, W, Ci, Co, s, e_f, e_dx, e_dw))
    assert e_f < 1e-2 and e_dx < 1e-2 and e_dw < 1e-2


@pytest.mark.parametrize("crop", [64, 256])
def test_network_gradients_vs_float64_autograd(crop):
    """Loss, prediction and every gradient against float64 autograd of the oracle's
    network.  At 256^2 the first layer's weight gradient is split over 256 pixel
    ranges and summed in two levels."""
    need_gpu()
    from paper_2606_21381_amd import cnn
    net = cnn.LearnedInit(batch=4, crop=crop)
    g = torch.Generator().manual_seed(3)
    images = (4.0 + torch.randn(4, crop, crop, generator=g)).float()
    targets = torch.randn(4, 4, generator=g).float()
    grads = torch.empty_like(net.params)
    loss = net.train_step(images.cuda(), targets.cuda(), 0.0, grads_out=grads, update=False)
    pred = net.forward(images.cuda())
    torch.cuda.synchronize()
    import oracle.cnn as oc
    P = net.params.cpu().double()
    ref_pred = oc.network(P, images)
    ref_loss, ref_grad = oc.loss_and_grad(P, images, targets)
    e_pred = rel(pred.cpu().double(), ref_pred)
    gg = grads.cpu().double()
    cos = float(torch.dot(gg, ref_grad) / (gg.norm() * ref_grad.norm()))
    say("cnn: pred rel %.2e, loss %.6f vs %.6f, grad cosine %.6f" % (e_pred, float(loss.item()), float(ref_loss), cos))
    assert e_pred < 3e-2 and abs(float(loss.item()) - float(ref_loss)) < 3e-2 * float(ref_loss) and cos > 0.995
    # each convolution's bias gradient on its own (the weight-gradient GEMM's row of ones)
    off = 0
    for ci, co in cnn.LAYERS:
        off += 9 * ci * co
        gb, rb = gg[off:off + co], ref_grad[off:off + co]
        off += co
        if float(rb.norm()) < 1e-6 * float(ref_grad.norm()):
            continue
        cb = float(torch.dot(gb, rb) / (gb.norm() * rb.norm()))
        say("cnn: bias gradient %d->%d cosine %.5f" % (ci, co, cb))
        assert cb > 0.99


def test_training_on_engine_crops_reduces_loss():
    need_gpu()
    from paper_2606_21381_amd import cnn
    net = cnn.LearnedInit(batch=64, crop=128, n_max=16)
    losses, secs = net.train(samples=64 * 200, lr=2e-3)
    say("cnn training smoke: loss %.4f -> %.4f in %.2f s" % (losses[:10].mean(), losses[-20:].mean(), secs))
    assert np.isfinite(losses).all() and losses[-20:].mean() < 0.8 * losses[:10].mean()


def test_trained_network_beats_the_default_start():
    """Trained on 600,000 engine-rendered 256^2 crops, the network predicts the four
    globals of held-out 1024^2 frames (500 prisms each, globals drawn from the training
    distribution; the network runs fully convolutionally with a global pool, as the
    inverse solve uses it) with a smaller mean absolute error than the inverse
    problem's default start, which multiplies each true global by 1 + U[-0.2, 0.2]:
    0.1 E|g| over that distribution (dn ~ U[0.01, 0.05], dz ~ U[-2, 2] um, shear ~
    U[0.8, 1.2] px, bias ~ pi/2 U[0.8, 1.2]) -- on every global."""
    need_gpu()
    from paper_2606_21381_amd import cnn, render, workloads
    net = cnn.LearnedInit()
    losses, secs = net.train(samples=600_000, lr=1e-3)
    crop_mae = net.evaluate(1024, seed=5)
    rng = np.random.Generator(np.random.PCG64(6))
    errs = []
    for _ in range(16):
        dn, dz, sh, th = workloads.crop_globals(rng)
        t = workloads.prisms(rng, 500, 1024, 1024)
        t[6] = dn
        g = torch.tensor([dz, sh, th, 0.0], dtype=torch.float32, device="cuda")
        I = render.render(torch.from_numpy(workloads.f32(t)).cuda(), 1024, 1024, workloads.dic_optics(0.0), g)
        errs.append(np.abs(net.predict(I) - np.array([dn, dz, sh, th])))
    mae = np.mean(errs, axis=0)
    default = np.array([0.1 * 0.03, 0.1 * 1.0, 0.1 * 1.0, 0.1 * math.pi / 2])
    say("trained 600k crops in %.1f s (loss %.4f); held-out 256^2 crop MAE %s; 1024^2 frame MAE dn %.4f dz %.3f um "
        "shear %.3f px bias %.4f rad; default start %s" % (secs, losses[-50:].mean(), np.array2string(crop_mae, precision=4),
                                                          *mae, np.array2string(default, precision=4)))
    assert np.isfinite(losses).all()
    assert np.all(mae < default)
