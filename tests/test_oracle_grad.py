"""Pins of the oracle's finite-difference gradients against closed forms."""
import math

import numpy as np

from oracle import grad, optics as O


def test_fd_of_patch_integral_matches_closed_form():
    # With unit weights on the OPD (not the image): d/da sum OPD = dn h 4 b, d/dh = dn 4ab.
    from oracle import raster
    s = np.zeros((8, 1))
    s[:, 0] = (30.3, 31.7, 0.6, 6.0, 4.0, 1.5, 0.03, 0)

    def tot(v, r):
        t = s.copy()
        t[r, 0] = v
        return raster.opd(t, 64, 64).sum()
    d = 1e-5
    ga = (tot(6.0 + d, 3) - tot(6.0 - d, 3)) / (2 * d)
    gh = (tot(1.5 + d, 5) - tot(1.5 - d, 5)) / (2 * d)
    gx = (tot(30.3 + d, 0) - tot(30.3 - d, 0)) / (2 * d)
    assert abs(ga - 0.03 * 1.5 * 4 * 4.0) < 1e-7
    assert abs(gh - 0.03 * 4 * 24.0) < 1e-7
    assert abs(gx) < 1e-7


def test_fd_of_empty_dic_bias_closed_form():
    # Empty canvas, DIC: I = 4 sin^2 theta everywhere -> d(sum I)/d theta = HW 4 sin 2 theta.
    opt = O.Optics(mode=O.DIC, na=0.5, shear_angle_rad=math.pi / 4)
    soa = np.zeros((8, 0))
    w = np.ones((32, 32))
    th = 1.1
    _, gg, _, fg = grad.fd_gradients(soa, 32, 32, opt, (0.3, 1.0, th, 0), w, rows=())
    assert abs(gg[2] - 32 * 32 * 4 * math.sin(2 * th)) < 1e-6 * 32 * 32
    assert abs(gg[0]) < 1e-6 and abs(gg[1]) < 1e-6 and not fg.any()


def test_loss_zero_at_truth():
    from paper_2606_21381_amd import workloads
    fr = workloads.config0()
    I = grad.image64(fr.soa, 64, 64, O.Optics(mode=O.BRIGHTFIELD, na=0.4), fr.globals4)
    assert grad.mse(I, I) == 0.0
