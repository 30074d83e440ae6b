"""Learned pricing on the host: the planner's network evaluation agrees with
the FP64 oracle network, and hand-built weights move the partition as the
prices they encode say they should."""
import math

import numpy as np
import pytest

from oracle import mlp
from paper_1509_04394_amd import costmodel, fz

F = fz.fz_cost_n_features()


def linear_in_feature(feature, alpha, beta):
    """Network computing alpha * x[feature] + beta (feature values >= 0)."""
    p = np.zeros(mlp.n_params(F))
    o_b1 = 64 * F
    o_w2 = o_b1 + 64
    o_b2 = o_w2 + 64 * 64
    o_w3 = o_b2 + 64
    o_b3 = o_w3 + 64
    p[feature] = 1.0          # W1[0][feature]
    p[o_w2] = 1.0             # W2[0][0]
    p[o_w3] = alpha           # W3[0]
    p[o_b3] = beta
    return p


def test_host_prediction_matches_oracle_network():
    w = mlp.init(F, seed=3) * 0.5
    for ops in [fz.RGB_HARRIS_CHAIN, fz.GRAD_CHAIN, fz.HARRIS_CHAIN[2:6]]:
        for tile in [(64, 16), (32, 32)]:
            plan = fz.Plan(ops, 640, 480, 64, partition=[], engine="tile", tile=tile, cost_weights=w)
            x = np.array(fz.fz_plan_segment_features(plan.handle, 0))
            want = math.exp(mlp.forward(w, x[None], F)[0])
            assert abs(plan.cost - want) <= 1e-5 * want


def test_features_describe_the_group():
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, 800, 600, 1000)
    x = fz.fz_plan_segment_features(plan.handle, 0)
    assert len(x) == F
    assert x[0] == pytest.approx(1.0)          # all 9 stages
    assert x[2] == pytest.approx(1.0)          # halo 6 of 6
    assert x[3] == 1.0                         # one frame of temporal halo
    assert x[8] == 1.0 and x[7] == 0.0         # row-marching engine
    with pytest.raises(fz.FzError):
        fz.fz_plan_segment_features(plan.handle, 1)


def test_prices_steer_the_partition():
    ops = fz.HARRIS_CHAIN
    # price grows 10x per stage in a group: singletons win
    steep = linear_in_feature(0, alpha=9 * math.log(10.0), beta=0.0)
    p = fz.Plan(ops, 320, 240, 16, cost_weights=steep)
    assert p.segments == list(range(len(ops)))
    # price falls with group length: one group wins
    falling = linear_in_feature(0, alpha=-5.0, beta=2.0)
    p = fz.Plan(ops, 320, 240, 16, cost_weights=falling)
    assert p.segments == [len(ops) - 1]


def test_learned_requires_weights():
    o = fz.make_opts(64, 48, 2, cost_model="learned")
    stages = [fz.fz_stage_describe(op) for op in fz.GRAD_CHAIN]
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_chain(stages, o)
    assert e.value.code == fz.FZ_E_INVALID


def test_committed_weights_plan_random_chains_optimally():
    """The trained weights shipped with the package load, match this build's
    feature set, and give finite prices from which the DP picks the exhaustive
    optimum (on random generic chains of the learned-cost workload)."""
    import os
    from oracle import partition as P
    from paper_1509_04394_amd import costmodel, synth
    if not os.path.exists(costmodel.WEIGHTS_PATH):
        pytest.skip("no trained weights in the package")
    params, meta = costmodel.load_weights()
    assert len(params) == fz.fz_mlp_param_count(F)
    assert np.all(np.isfinite(params))
    assert meta["train_chains"] >= 1000 and meta["test_chains"] >= 100
    for seed in (9600, 9601, 9602):
        spec = synth.random_chain(seed)[:10]
        plan = fz.Plan(spec, 640, 480, 64, cost_weights=params)
        n = len(spec)
        c = [[plan.group_cost(a, b) if b >= a else None for b in range(n)] for a in range(n)]
        assert all(math.isfinite(c[a][b]) and c[a][b] > 0 for a in range(n) for b in range(a, n))
        want, groups = P.best(c, n)
        assert plan.cost == pytest.approx(want, rel=1e-12)
        assert plan.segments == [b for (_, b) in groups]


def test_fixed_held_out_cases_are_not_training_cases():
    """The held-out fixed-chain workloads of the cost-model test are neither in
    the fine-tuning grid nor in the original campaign's training split."""
    held = set(costmodel.FIXED_HELD_OUT)
    assert len(held) >= 6
    assert not held & set(costmodel.fixed_campaign()["train"])
    assert not held & set(costmodel.campaign()["train"])
