"""Measured prices (fz_plan_measure) on the GPU.

Timings vary from run to run, so the checks are the ones that hold for any
measurement: every group that the analytic model allows gets a positive
finite time; the chosen partition is the exhaustive optimum over the measured
table; the plan's cost is the sum of its groups' measured times; and the
re-planned chain computes the same bits as before (fusion does not change
the arithmetic).
"""
import math

import numpy as np
import pytest

from oracle import partition as P
from paper_1509_04394_amd import fz, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _check_measured(plan, analytic_costs, x, before):
    n = len(plan.stages)
    c = [[plan.group_cost(a, b) if b >= a else None for b in range(n)] for a in range(n)]
    for a in range(n):
        for b in range(a, n):
            if math.isfinite(analytic_costs[a][b]):
                assert math.isfinite(c[a][b]) and c[a][b] > 0, (a, b)
    want, groups = P.best(c, n)
    assert plan.cost == pytest.approx(want, rel=1e-12)
    assert plan.segments == [b for (_, b) in groups]
    assert plan.cost == pytest.approx(sum(s.cost for s in plan.segment_info()), rel=1e-12)
    out, _, _ = plan.run(x)
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), before
    assert np.array_equal(a.view(np.uint8), b.view(np.uint8))


def test_measured_plan_harris_rgb(dev):
    W, H, T = 320, 240, 24
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T)
    n = len(plan.stages)
    ana = [[plan.group_cost(a, b) if b >= a else None for b in range(n)] for a in range(n)]
    x = torch.from_numpy(synth.video(W, H, T, seed=3, rgb=True)).to(dev)
    before, _, _ = plan.run(x)
    torch.cuda.synchronize()
    before = before.cpu().numpy()
    plan.measure(x, reps=3)
    print("[gpu-measure] harris rgb: measured partition", plan.segments, f"{plan.cost:.0f} us", flush=True)
    _check_measured(plan, ana, x, before)


def test_measured_plan_generic(dev):
    spec = synth.random_chain(5003)
    W, H, T = 192, 432, 16
    plan = fz.Plan(spec, W, H, T)
    n = len(spec)
    ana = [[plan.group_cost(a, b) if b >= a else None for b in range(n)] for a in range(n)]
    x = torch.from_numpy(synth.video(W, H, T, seed=9)).to(dev)
    before, _, _ = plan.run(x)
    torch.cuda.synchronize()
    before = before.cpu().numpy()
    plan.measure(x, reps=3)
    print("[gpu-measure] generic: analytic", [len(spec) - 1], "measured", plan.segments, f"{plan.cost:.0f} us",
          flush=True)
    _check_measured(plan, ana, x, before)
