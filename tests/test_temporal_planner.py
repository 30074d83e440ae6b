"""Host-side planning of the temporal generic stages (no GPU): the Eq. 6 box
sizing against a grid search, descriptor validation of the IIR and of
stencils that look back, and the planner's engine, frame-run and group
choices for them."""
import numpy as np
import pytest

from paper_1509_04394_amd import fz


def eq6(beta, dx, dt):
    return fz.fz_box_eq6(beta, dx, dt)


@pytest.mark.parametrize("beta,dx,dt", [(4096, 2, 1), (30000, 3, 2), (1e6, 6, 1), (500, 1, 3), (8e4, 2.5, 0.5)])
def test_eq6_is_the_grid_minimum(beta, dx, dt):
    """Sec. VI-E: Eq. 6 minimises the input box (x + 2dx)^2 (t + dt) over boxes
    of volume x^2 t = beta.  A fine grid over x (t = beta / x^2) finds the
    same minimiser and the closed form's volume is the grid's minimum."""
    x, t = eq6(beta, dx, dt)
    assert x * x * t == pytest.approx(beta, rel=1e-12)
    xs = np.exp(np.linspace(np.log(0.5), np.log(beta ** 0.5 * 4), 400001))
    V = (xs + 2 * dx) ** 2 * (beta / xs ** 2 + dt)
    j = int(np.argmin(V))
    assert x == pytest.approx(xs[j], rel=1e-3)
    Vx = (x + 2 * dx) ** 2 * (t + dt)
    assert Vx <= V.min() * (1 + 1e-9)
    # the printed closed form: x = cbrt(2 beta dx / dt), t = beta^(1/3) (dt/dx)^(2/3) / 2^(2/3)
    assert x == pytest.approx((2 * beta * dx / dt) ** (1 / 3), rel=1e-12)
    assert t == pytest.approx(beta ** (1 / 3) * (dt / dx) ** (2 / 3) / 2 ** (2 / 3), rel=1e-12)


def test_eq6_worked_value_and_degenerate_halos():
    # beta = 4096, one pixel of halo per side per frame of temporal halo:
    # x = cbrt(8192) = 20.158..., t = 4096 / x^2
    x, t = eq6(4096, 1, 1)
    assert x == pytest.approx(8192 ** (1 / 3))
    assert t == pytest.approx(4096 / x ** 2)
    assert eq6(100, 2, 0) == pytest.approx((10.0, 1.0))   # no temporal halo: the flattest box
    assert eq6(100, 0, 2) == pytest.approx((1.0, 100.0))  # no spatial halo: the thinnest
    for bad in [(0, 1, 1), (-5, 1, 1), (10, -1, 1), (10, 1, -1), (float("nan"), 1, 1)]:
        with pytest.raises(fz.FzError):
            eq6(*bad)


W3T = np.full((3, 3, 3), 1.0 / 27.0, np.float32)


def test_iir_descriptor_validation():
    s = fz.fz_stage_describe("iir")
    assert (s.rx, s.ry, s.rt, s.dep) == (0, 0, -1, fz.FZ_DEP_TT)
    assert s.param[0] == pytest.approx(0.5)
    for a in (0.0, -0.5, 1.5, float("nan")):
        with pytest.raises(fz.FzError) as e:
            fz.Plan([("iir", a)], 64, 32, 5)
        assert e.value.code == fz.FZ_E_INVALID
    fz.Plan([("iir", 1.0)], 64, 32, 5)  # a = 1 passes the input through


def test_temporal_stencil_validation():
    fz.Plan([("stencil", 1, 1, W3T)], 64, 32, 5)
    with pytest.raises(fz.FzError):  # more than 3 frames back
        fz.Plan([("stencil", 1, 1, np.full((5, 3, 3), 0.1, np.float32))], 64, 32, 5)
    with pytest.raises(ValueError):  # weights of the wrong shape (the binding checks; the C ABI cannot)
        fz.Plan([("stencil", 1, 1, np.full((2, 3, 5), 0.1, np.float32))], 64, 32, 5)


def test_learned_prices_refuse_temporal_chains():
    import json
    import os
    w = json.load(open(os.path.join(os.path.dirname(fz.__file__), "cost_weights.json")))["params"]
    fz.Plan([("stencil", 1, 1, np.full((3, 3), 0.1, np.float32))], 64, 32, 5, cost_weights=w)
    with pytest.raises(fz.FzError) as e:
        fz.Plan([("iir", 0.5), ("box", 1, 1)], 64, 32, 5, cost_weights=w)
    assert e.value.code == fz.FZ_E_UNSUPPORTED


def test_engines_and_frame_runs():
    T = 50
    p = fz.Plan([("iir", 0.25), ("point", "abs", 0.0, 0.0)], 800, 600, T)
    (s,) = p.segment_info()
    assert s.engine == fz.FZ_ENGINE_STREAM and s.frames_per_block == T
    # an IIR before the window stage is checkpointed: 8-frame runs here (64x32 tiles: 247 x 7 runs
    # already leave fewer than two fills of work items at 16), the checkpoints priced per run
    p = fz.Plan([("iir", 0.25), ("box", 1, 1)], 800, 600, T, partition=[])
    (s,) = p.segment_info()
    assert s.engine == fz.FZ_ENGINE_TILE and s.frames_per_block == 8 and s.halo_t == 0
    assert s.bytes_per_px == pytest.approx(1 + 4 + 1 + 16.0 / 8)
    # an IIR after a window stage cannot resume from a checkpoint: whole-clip runs
    p = fz.Plan([("box", 1, 1), ("iir", 0.25)], 800, 600, T, partition=[])
    (s,) = p.segment_info()
    assert s.engine == fz.FZ_ENGINE_TILE and s.frames_per_block == T
    # a stencil two frames back: the frame run follows Eq. 6 with beta = W H T / 1024
    p = fz.Plan([("stencil", 1, 1, W3T), ("box", 1, 1)], 800, 600, 1000, partition=[])
    (s,) = p.segment_info()
    x, t = fz.fz_box_eq6(800 * 600 * 1000 / 1024, 2.0, 2.0)
    assert s.engine == fz.FZ_ENGINE_TILE and s.halo_t == 2
    assert s.frames_per_block == int(np.floor(t + 0.5))
    # the compulsory bytes count the temporal halo re-read once per frame run
    assert s.bytes_per_px == pytest.approx(1 + 4 + 2.0 / s.frames_per_block)


def test_iir_frame_run_requests():
    """A frame run shorter than the clip is refused for a group whose IIR
    follows a window stage (its state cannot be checkpointed), and kept for
    one whose IIRs lead (checkpointed)."""
    with pytest.raises(fz.FzError) as e:
        fz.Plan([("box", 1, 1), ("iir", 0.5)], 128, 64, 20, frames_per_block=4)
    assert e.value.code == fz.FZ_E_UNSUPPORTED
    p = fz.Plan([("box", 1, 1), ("iir", 0.5)], 128, 64, 20, partition=[])
    with pytest.raises(fz.FzError) as e:
        p.set_segment_config(0, engine="tile", tile=(32, 32), frames_per_block=4)
    assert e.value.code == fz.FZ_E_UNSUPPORTED
    p.set_segment_config(0, engine="tile", tile=(32, 32), frames_per_block=20)
    assert p.segment_info()[0].frames_per_block == 20
    p = fz.Plan([("iir", 0.5), ("box", 1, 1)], 128, 64, 20, frames_per_block=4)
    assert p.segment_info()[0].frames_per_block == 4
    # the checkpoints live in the workspace: (20 / 4 - 1) runs x 128 x 64 states of 8 bytes
    assert p.workspace_bytes >= 4 * 128 * 64 * 8


def test_weight_store_limits_group_size():
    """A group's stencils share a 784-float argument store: five 7x7
    stencils reading four frames each (980 weights) cannot be one group (nor
    would their rings fit the LDS), but every stage alone can."""
    w = np.full((4, 7, 7), 1.0 / 196.0, np.float32)
    spec = [("stencil", 3, 3, w)] * 5
    with pytest.raises(fz.FzError):
        fz.Plan(spec, 256, 128, 8, partition=[])
    p = fz.Plan(spec, 256, 128, 8)
    assert len(p.segments) >= 2
    assert np.isinf(p.group_cost(0, 4)) and np.isfinite(p.group_cost(2, 2))


def test_under_filled_marching_groups_cost_more():
    """An IIR group marches whole clips, one work item per tile: on small
    frames it cannot fill the device, and its price grows by the idle share."""
    spec = [("iir", 0.5), ("box", 1, 1)]
    big = fz.Plan(spec, 800, 600, 100, partition=[])
    small = fz.Plan(spec, 192, 96, 100, partition=[])
    per_px = lambda p: p.cost / (p.W * p.H * p.T)
    assert per_px(small) > per_px(big) >= 5.0
