"""Host-side tests of the planner on generic chains (no GPU needed).

Random chains of generic stages (point, weighted stencil, window sum) are
planned under several on-chip budgets; the DP's partition is compared with
the exhaustive enumeration of every partition on the planner's own price
table; the prices are checked against the compulsory-traffic closed form and
the LDS footprint against the box size the kernel stages; and every malformed
descriptor is rejected before anything runs.
"""
import math

import numpy as np
import pytest

from oracle import partition as P
from paper_1509_04394_amd import fz, synth

TILES = [(64, 16), (32, 32), (64, 32)]


def _halo(spec, a, b):
    hx = sum(s[1] for s in spec[a:b + 1] if s[0] != "point")
    hy = sum(s[2] for s in spec[a:b + 1] if s[0] != "point")
    nwin = sum(1 for s in spec[a:b + 1] if s[0] != "point")
    return hx, hy, nwin


def _lds(tw, th, hx, hy, nwin):
    # input box as f32, twice when one window step feeds another, and 4 floats of slack
    return 0 if nwin == 0 else ((2 if nwin >= 2 else 1) * (tw + 2 * hx) * (th + 2 * hy) + 4) * 4


@pytest.mark.parametrize("seed", range(12))
@pytest.mark.parametrize("budget", [0, 60000, 20000])
def test_generic_optimum_equals_exhaustive(seed, budget):
    spec = synth.random_chain(5000 + seed)[:10]
    W, H, T = 192, 432, 64
    try:
        plan = fz.Plan(spec, W, H, T, lds_budget=budget)
    except fz.FzError as e:
        assert e.code == fz.FZ_E_LDS
        # some single stage must be too large for the budget on every tile
        assert any(min(_lds(tw, th, *_halo(spec, i, i)) for tw, th in TILES) > budget for i in range(len(spec)))
        return
    n = len(spec)
    c = [[plan.group_cost(a, b) if b >= a else None for b in range(n)] for a in range(n)]
    want, groups = P.best(c, n)
    assert plan.cost == want
    assert plan.segments == [b for (_, b) in groups]


@pytest.mark.parametrize("seed", range(6))
def test_generic_prices_and_footprint(seed):
    spec = synth.random_chain(6000 + seed)[:9]
    W, H, T = 320, 240, 10
    budget = 163840
    plan = fz.Plan(spec, W, H, T, in_dtype="u8")
    n = len(spec)
    for a in range(n):
        for b in range(a, n):
            hx, hy, nwin = _halo(spec, a, b)
            fits = [(tw, th) for tw, th in TILES if _lds(tw, th, hx, hy, nwin) <= budget]
            cost = plan.group_cost(a, b)
            if nwin and not fits:
                assert math.isinf(cost)
                continue
            # compulsory traffic: the group's input once (u8 only into stage 0) and f32 out once
            assert cost == ((1 if a == 0 else 4) + 4) * W * H * T
    for s in plan.segment_info():
        hx, hy, nwin = _halo(spec, s.first, s.last)
        assert s.halo == hx and s.halo_t == 0
        if nwin == 0:
            assert s.engine == fz.FZ_ENGINE_STREAM and s.lds_bytes == 0
        else:
            assert s.engine == fz.FZ_ENGINE_TILE
            assert s.lds_bytes == _lds(s.tile_w, s.tile_h, hx, hy, nwin) <= budget
            # the tile of best data utilisation (Eq. 3) among those that fit
            du = lambda t: t[0] * t[1] / ((t[0] + 2 * hx) * (t[1] + 2 * hy))
            fits = [t for t in TILES if _lds(t[0], t[1], hx, hy, nwin) <= budget]
            assert du((s.tile_w, s.tile_h)) == max(du(t) for t in fits)


def test_generic_fully_fused_when_it_fits():
    w = np.full((3, 3), 1.0 / 9.0, np.float32)
    spec = [("stencil", 1, 1, w), ("point", "abs", 0, 0), ("box", 2, 2), ("point", "sqrtabs", 0, 0)]
    plan = fz.Plan(spec, 640, 480, 8)
    assert plan.segments == [3]
    assert plan.cost == (1 + 4) * 640 * 480 * 8
    plan = fz.Plan(spec, 640, 480, 8, partition="unfused")
    assert plan.cost == (1 + 4 + 4 * 3 + 4 * 3) * 640 * 480 * 8


def test_generic_kernel_to_kernel_forces_a_cut():
    w = np.ones((3, 3), np.float32)
    spec = [("stencil", 1, 1, w), ("box", 1, 1), ("point", "abs", 0, 0)]
    plan = fz.Plan(spec, 100, 80, 4, deps={1: fz.FZ_DEP_KK})
    assert plan.segments == [0, 2]


def test_generic_point_only_chain_streams():
    spec = [("point", "affine", 2.0, 1.0), ("point", "clamp", 0.0, 100.0)]
    plan = fz.Plan(spec, 100, 80, 4, in_dtype="f32")
    info = plan.segment_info()
    assert len(info) == 1 and info[0].streaming == 1 and info[0].engine == fz.FZ_ENGINE_STREAM
    assert plan.input_shape() == (1, 4, 80, 100) and plan.output_shape() == (1, 4, 80, 100)


def _bad(spec, code, **kw):
    with pytest.raises(fz.FzError) as e:
        fz.Plan(spec, 64, 64, 2, **kw)
    assert e.value.code == code, str(e.value)


def test_generic_descriptor_errors():
    w3 = np.ones((3, 3), np.float32)
    _bad([("stencil", 4, 4, np.ones((9, 9), np.float32))], fz.FZ_E_INVALID)  # radius above 3
    _bad([("box", 1, -1)], fz.FZ_E_INVALID)
    _bad([("point", "clamp", 5.0, 1.0)], fz.FZ_E_INVALID)  # a > b
    bad_w = w3.copy()
    bad_w[1, 1] = np.nan
    _bad([("stencil", 1, 1, bad_w)], fz.FZ_E_INVALID)
    _bad([("point", "affine", float("inf"), 0.0)], fz.FZ_E_INVALID)
    _bad([("box", 1, 1)], fz.FZ_E_INVALID, deps={0: fz.FZ_DEP_TT})  # a window cannot be thread-to-thread
    # stencil without weights, unknown point kind, u8 into a later stage
    stages, keep = fz.generic_stages([("stencil", 1, 1, w3)])
    stages[0].weights = None
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_chain(stages, fz.make_opts(64, 64, 2))
    assert e.value.code == fz.FZ_E_INVALID
    stages, keep = fz.generic_stages([("point", "abs", 0, 0)])
    stages[0].param[0] = 7.0
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_chain(stages, fz.make_opts(64, 64, 2))
    assert e.value.code == fz.FZ_E_INVALID
    stages, keep = fz.generic_stages([("point", "abs", 0, 0), ("box", 1, 1)])
    stages[1].in_dtype = fz.FZ_U8
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_chain(stages, fz.make_opts(64, 64, 2))
    assert e.value.code == fz.FZ_E_INVALID
    # generic and fixed stages do not mix
    g = fz.generic_stages([("box", 1, 1)], in_dtype="f32")[0][0]
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_chain([fz.fz_stage_describe("gauss5"), g], fz.make_opts(64, 64, 2))
    assert e.value.code == fz.FZ_E_UNSUPPORTED


def test_generic_learned_features_are_finite():
    spec = synth.random_chain(5003)
    plan = fz.Plan(spec, 192, 432, 64)
    for i in range(len(plan.segments)):
        f = fz.fz_plan_segment_features(plan.handle, i)
        assert len(f) == fz.fz_cost_n_features() and all(math.isfinite(v) for v in f)
        assert f[-1] == 1.0  # the generic-kernel flag
