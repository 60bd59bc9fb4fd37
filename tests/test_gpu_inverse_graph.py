"""The inverse solver's captured-graph steps against its eager steps: the same
trajectory bit for bit (losses, parameter errors, final parameters) over runs
that replay each curriculum stage's graph many times, with eager copies and
rate updates between the replays -- for the pixel MSE with the globals-first
stage and the cosine decay, and for the spectral loss of Eq. 8."""
import numpy as np
import pytest

from paper_2606_21381_amd import inverse, workloads
from tests.gpu_util import need_gpu, say

pytestmark = pytest.mark.gpu


def run(graph, loss="mse", steps=90, curriculum=None):
    prob = workloads.config3(seed=11, n=40, size=256)
    target, start, truth = inverse.problem_tensors(prob, "cuda")
    cfg = inverse.SolverConfig(steps=steps, globals_first=25, decay_after=0.5, graph=graph, loss=loss,
                               curriculum=curriculum)
    r = inverse.solve(target, start, truth, prob.target.H, prob.target.W, prob.target.optics, cfg)
    return r, [q.detach().cpu().numpy() for q in start.parameters()]


@pytest.mark.parametrize("loss,steps,curriculum", [("mse", 90, None),
                                                   ("spectral", 40, ((15, ("dz", "bias")), (25, ("dz", "bias", "dn"))))])
def test_graph_steps_equal_eager_steps(loss, steps, curriculum):
    need_gpu()
    a, pa = run(True, loss, steps, curriculum)
    b, pb = run(False, loss, steps, curriculum)
    say("%s: graph %s, %.0f steps/s replayed vs %.0f eager; loss %.4g -> %.4g" % (
        loss, a.graphed, steps / a.time_s[-1], steps / b.time_s[-1], a.loss[0], a.loss[-1]))
    assert a.graphed and not b.graphed
    assert np.array_equal(a.loss, b.loss)
    assert np.array_equal(a.error, b.error)
    for x, y in zip(pa, pb):
        assert np.array_equal(x, y)
    assert a.loss[-1] < a.loss[0]
