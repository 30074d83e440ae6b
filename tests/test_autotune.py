"""Box sizing for the row kernel and the autotuner's candidate set (host
only): the one-axis form of Eq. 6 against a grid search, the seed's use of
it, and that every candidate configuration is one the planner accepts."""
import numpy as np
import pytest

from paper_1509_04394_amd import autotune, fz


@pytest.mark.parametrize("beta,dy,dt", [(800, 6, 1), (93750 / 116, 6, 1), (5000, 3, 2), (64, 1, 1)])
def test_eq6_row_is_the_grid_minimum(beta, dy, dt):
    y, t = autotune.eq6_row(beta, dy, dt)
    assert y * t == pytest.approx(beta, rel=1e-12)
    ys = np.exp(np.linspace(np.log(0.2), np.log(beta * 5), 400001))
    V = (ys + 2 * dy) * (beta / ys + dt)
    assert y == pytest.approx(ys[int(np.argmin(V))], rel=1e-3)
    assert (y + 2 * dy) * (t + dt) <= V.min() * (1 + 1e-9)


def test_eq6_row_degenerate_halos():
    assert autotune.eq6_row(100, 6, 0) == (100, 1.0)
    assert autotune.eq6_row(100, 0, 1) == (1.0, 100)


def test_row_seed_for_the_benchmark_video():
    # 800 wide: 7 strips of 116 new columns; one round of 5120 wavefronts over
    # 600 rows x 1000 frames x 7 strips: beta = 820.3 rows x frames
    y, t = autotune.row_seed(800, 600, 1000, 1)
    yy, tt = autotune.eq6_row(600 * 1000 * 7 / 5120, 6, 1)
    assert (y, t) == (round(yy), round(tt))
    assert 8 <= y <= 600 and 1 <= t <= 1000


def test_every_candidate_is_accepted_by_the_planner():
    W, H, T = 800, 600, 64
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T)
    (info,) = plan.segment_info()
    assert info.engine == fz.FZ_ENGINE_ROW
    cands = autotune.candidates(info, W, H, T)
    y, t = autotune.row_seed(W, H, T, info.halo_t)
    assert dict(engine="row", tile_h=y, frames_per_block=t) in cands
    ok = 0
    for cfg in cands:
        trial = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T, partition=[])
        fz.fz_plan_set_segment_config(trial.handle, 0, **cfg)
        s = trial.segment_info()[0]
        if cfg["engine"] == "row":
            assert (s.tile_h, s.frames_per_block) == (cfg["tile_h"], min(cfg["frames_per_block"], T))
        else:
            assert (s.tile_w, s.tile_h) == (cfg["tile_w"], cfg["tile_h"])
        ok += 1
    assert ok == len(cands)
