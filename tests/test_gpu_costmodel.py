"""The learned price against the analytic one, measured.

Held-out workloads -- fixed chains at (chain, W, H, T) tuples no training
case contains, and random generic chains of unseen seeds -- have every group
timed in every configuration; the best partition under measured prices
(exact DP over the table) is the reference.  The partition the planner
chooses with the trained network must be within 5% of it (geometric mean),
separately on the fixed chains and on the random chains, and no worse than
the analytic (bytes) prices."""
import math
import os

import numpy as np
import pytest

from paper_1509_04394_amd import costmodel

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def weights():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(costmodel.WEIGHTS_PATH):
        pytest.skip("no trained cost weights")
    return costmodel.load_weights()


def evaluate(cases, params, tag):
    rows = []
    for name, W, H, T in cases:
        ops = costmodel.case_ops(name)
        table = costmodel.measure_table(ops, W, H, T, seed=77, reps=7)
        r = costmodel.evaluate_case(ops, W, H, T, params, table)
        rows.append(r)
        print(f"[costmodel] {tag} {name} {W}x{H}x{T}: best {r['best_us']:.0f} us {r['best_partition']}, "
              f"learned {r['learned_ratio']:.3f} {r['learned_partition']}, "
              f"analytic {r['analytic_ratio']:.3f} {r['analytic_partition']}", flush=True)
    geo = lambda k: math.exp(np.mean([math.log(r[k]) for r in rows]))
    print(f"[costmodel] {tag} geomean over best: learned {geo('learned_ratio'):.4f}, "
          f"analytic {geo('analytic_ratio'):.4f}", flush=True)
    return geo("learned_ratio"), geo("analytic_ratio")


def test_learned_partitions_near_best_measured(weights):
    params, meta = weights
    fixed_l, fixed_a = evaluate(costmodel.FIXED_HELD_OUT[:6], params, "fixed")
    rand_l, rand_a = evaluate(costmodel.random_cases(9500, 3), params, "random")
    assert fixed_l <= 1.05
    assert rand_l <= 1.05
    assert fixed_l <= fixed_a * 1.02 and rand_l <= rand_a * 1.02
