"""The inverse solve of the 1024^2 DIC target from 500 prisms (seed 3) through the
library's forward render and adjoint: Adam from the perturbed start, then the
second-order polish, to a parameter error e <= 1e-3 (every prism's centre, width
within 3e-3 px, angle within 2e-4 rad modulo pi/2; every global within 1e-3
relative)."""
import math

import pytest
import torch

from gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def test_hybrid_solve_reaches_1e3_on_seed_3():
    need_gpu()
    from paper_2606_21381_amd import inverse, workloads
    prob = workloads.config3(seed=3)
    target, start, truth = inverse.problem_tensors(prob, torch.device("cuda", 0))
    r = inverse.solve_hybrid(target, start, truth, prob.target.H, prob.target.W, prob.target.optics)
    say("hybrid solve seed 3: time to 1e-3 %s s, final e %.3e (glob %.3e, part %.3e), loss %.3e, %.2f s" % (
        r.time_to_target_s, r.final_e, r.final_e_glob, r.final_e_part, r.final_loss, r.total_s))
    assert r.time_to_target_s is not None and r.final_e <= 1e-3
    # the start is 0.2 rad / 3 px / 20 % away, so the solve did move everything
    assert float(r.adam.error[0]) > 0.5
    # the solved parameters reproduce the target to FP32 rounding
    assert r.final_loss < 1e-10 * float(torch.mean(target.double() ** 2))
