"""Host-side tests of the planner and the C ABI (no GPU needed).

The DP optimum is compared with the exhaustive enumeration of every partition
(oracle/partition.py) on the planner's own price tables and on random tables
with ties and forbidden groups, for every chain length up to 10.
"""
import ctypes
import math
import re

import numpy as np
import pytest

from oracle import partition as P
from paper_1509_04394_amd import fz


def test_library_exports_every_declared_symbol():
    header = open(fz.os.path.join(fz.os.path.dirname(fz.HERE), "include", "fz.h")).read()
    declared = set(re.findall(r"\b(fz_[a-z0-9_]+)\s*\(", header))
    declared -= {"fz_plan"}  # type name, not a function
    L = ctypes.CDLL(fz.LIB_PATH)
    for name in declared:
        assert hasattr(L, name), name
    assert declared == {n for n, _, _ in fz.SIGNATURES}


def test_static_workspace_refuses_oversized_plans_on_the_host():
    """fz_run_chain_static checks the plan's workspace against its fixed
    array before touching any device: an unfused 800x600x40 plan needs more
    than 64 MiB and is refused (the buffer addresses are never used)."""
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, 800, 600, 40, partition="unfused")
    assert plan.workspace_bytes > fz.FZ_STATIC_WORKSPACE_BYTES
    rc = fz.lib().fz_run_chain_static(plan.handle, 1, 1, None, None, 0, None)
    assert rc == fz.FZ_E_WORKSPACE
    assert "static" in fz.fz_last_error()
    rc = fz.lib().fz_run_chain_static(plan.handle, None, 1, None, None, 0, None)
    assert rc == fz.FZ_E_INVALID


@pytest.mark.parametrize("n", range(1, 11))
def test_dp_equals_exhaustive_random_tables(n):
    rng = np.random.default_rng(100 + n)
    for trial in range(30):
        c = [[None] * n for _ in range(n)]
        for a in range(n):
            for b in range(a, n):
                r = rng.random()
                # small integer prices give many exact ties; some groups forbidden
                c[a][b] = math.inf if (r < 0.15 and b > a) else float(rng.integers(1, 6))
        total, sl = fz.fz_partition_min(c)
        want_total, groups = P.best(c, n)
        assert total == want_total
        assert sl == [b for (_, b) in groups]


def test_dp_infeasible():
    c = [[math.inf, math.inf], [None, math.inf]]
    total, sl = fz.fz_partition_min(c)
    assert math.isinf(total) and sl == []


CHAINS = [fz.RGB_HARRIS_CHAIN, fz.HARRIS_CHAIN, fz.GRAD_CHAIN, fz.HARRIS_CHAIN[2:7]]


@pytest.mark.parametrize("ops", CHAINS, ids=lambda o: "-".join(o))
@pytest.mark.parametrize("budget", [0, 40000, 24000])
def test_planner_optimum_equals_exhaustive(ops, budget):
    try:
        plan = fz.Plan(ops, 800, 600, 1000, lds_budget=budget)
    except fz.FzError as e:
        assert e.code == fz.FZ_E_LDS
        return
    n = len(ops)
    c = [[plan.group_cost(a, b) if b >= a else None for b in range(n)] for a in range(n)]
    want, groups = P.best(c, n)
    assert plan.cost == want
    assert plan.segments == [b for (_, b) in groups]


def test_analytic_costs_are_compulsory_traffic():
    # per-pixel bytes in/out of every stage of the Harris chain (u8 RGB input)
    ops = fz.RGB_HARRIS_CHAIN
    bi = [3, 1, 4, 8, 12, 12, 4, 4, 1]
    bo = [1, 4, 8, 12, 12, 4, 4, 1, 1]
    W, H, T = 800, 600, 1000
    npx = W * H * T
    plan = fz.Plan(ops, W, H, T, partition="unfused")
    info = plan.segment_info()
    for i, s in enumerate(info):
        extra = bi[i] if ops[i] == "framediff" else 0.0  # the previous frame is re-read
        assert s.bytes_per_px == P.compulsory_bytes(bi, bo, i, i) + extra
    assert plan.cost == npx * (P.unfused_bytes(bi, bo) + 1)
    full = fz.Plan(ops, W, H, T)
    assert full.segments == [8]
    s = full.segment_info()[0]
    assert s.halo == 6 and s.halo_t == 1
    # the fused group runs on the row kernel, whose items take the frame
    # before their run from the previous run's item: input and output once
    assert s.engine == fz.FZ_ENGINE_ROW
    assert s.bytes_per_px == 3 + 1
    assert s.lds_bytes <= 163840
    # the same group on the tile engine re-reads the frame before each run
    tile = fz.Plan(ops, W, H, T, engine="tile").segment_info()[0]
    assert tile.bytes_per_px == 3 + 1 + 3 / tile.frames_per_block


def test_halo_is_sum_of_radii_not_max():
    # gauss (r=2) then sobel (r=1) needs a 3-pixel halo; taking the larger
    # radius (2) would leave the sobel of the outermost output pixels reading
    # gauss values that were never computed
    plan = fz.Plan(["gauss5", "sobel3"], 64, 48, 2)
    assert plan.segment_info()[0].halo == 3
    plan = fz.Plan(fz.HARRIS_CHAIN[:7], 64, 48, 2)
    assert plan.segment_info()[0].halo == 2 + 1 + 2 + 1


def test_kk_dependence_forces_a_cut():
    plan = fz.Plan(fz.HARRIS_CHAIN, 192, 432, 600, deps={4: fz.FZ_DEP_KK})
    segs = plan.segments
    assert 3 in segs  # group boundary right before stage 4
    assert math.isinf(plan.group_cost(0, 4)) and math.isinf(plan.group_cost(3, 5))


def test_budget_limits_fusion():
    loose = fz.Plan(fz.HARRIS_CHAIN, 192, 432, 600)
    tight = fz.Plan(fz.HARRIS_CHAIN, 192, 432, 600, lds_budget=40000)
    assert len(loose.segments) == 1
    assert len(tight.segments) >= 1
    for s in tight.segment_info():
        assert s.lds_bytes <= 40000
    assert tight.cost >= loose.cost


def test_explicit_and_unfused_partitions():
    p = fz.Plan(fz.HARRIS_CHAIN, 64, 48, 4, partition=[0, 2, 5])
    assert p.segments == [0, 2, 5, 7]
    u = fz.Plan(fz.HARRIS_CHAIN, 64, 48, 4, partition="unfused")
    assert u.segments == list(range(8))
    assert u.workspace_bytes >= 64 * 48 * 4 * 12


@pytest.mark.parametrize("bad", [
    dict(ops=["sobel3", "gauss5"]),                       # not a compiled sequence / type mismatch
    dict(ops=["gauss5"], W=0),
    dict(ops=["gauss5"], T=-1),
    dict(ops=fz.HARRIS_CHAIN, partition=[3, 3]),
    dict(ops=fz.HARRIS_CHAIN, partition=[7]),
    dict(ops=["gauss5"], tile=(48, 48)),
])
def test_plan_errors(bad):
    kw = dict(W=64, H=48, T=2)
    kw.update(bad)
    ops = kw.pop("ops")
    with pytest.raises(fz.FzError) as e:
        fz.Plan(ops, kw.pop("W"), kw.pop("H"), kw.pop("T"), **kw)
    assert e.value.code in (fz.FZ_E_INVALID, fz.FZ_E_UNSUPPORTED)
    assert fz.fz_last_error()


def test_descriptor_mismatch_rejected():
    s = fz.fz_stage_describe("gauss5")
    s.rx = 3
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_chain([s], fz.make_opts(10, 10, 1))
    assert e.value.code == fz.FZ_E_INVALID


def test_run_argument_errors_without_launch():
    p = fz.Plan(fz.HARRIS_CHAIN, 64, 48, 2, partition="unfused")
    with pytest.raises(fz.FzError) as e:
        fz.fz_run_chain(p.handle, 1, 1, None, None, 0, None, 0, None)
    assert e.value.code == fz.FZ_E_WORKSPACE
    with pytest.raises(fz.FzError) as e:
        fz.fz_run_chain(p.handle, None, 1, None, None, 0, None, 0, None)
    assert e.value.code == fz.FZ_E_INVALID
    with pytest.raises(fz.FzError) as e:
        fz.fz_run_chain(p.handle, 1, 1, None, None, 5, 1, 1 << 40, None)
    assert e.value.code == fz.FZ_E_INVALID


def test_stage_describe_access_patterns():
    # Table I classes: point ops read one pixel, window ops a square, the frame
    # difference one frame back
    for name in ["rgb2gray", "gradmag", "products", "harris", "threshold"]:
        s = fz.fz_stage_describe(name)
        assert (s.rx, s.ry, s.rt) == (0, 0, 0)
    assert (fz.fz_stage_describe("gauss5").rx, fz.fz_stage_describe("boxsum5").rx) == (2, 2)
    assert (fz.fz_stage_describe("sobel3").rx, fz.fz_stage_describe("nms3").rx) == (1, 1)
    assert fz.fz_stage_describe("framediff").rt == 1
    with pytest.raises(fz.FzError):
        fz.fz_stage_describe(99)


def test_batch_argument_errors_without_launch():
    plan = fz.Plan(fz.HARRIS_CHAIN, 320, 240, 10)
    c = fz.fz_clip()
    c.d_in, c.d_out, c.width, c.height, c.frames = 1, 1, 320, 240, 10
    assert fz.fz_batch_workspace_bytes(plan.handle, [c]) > 0
    with pytest.raises(fz.FzError) as e:
        fz.fz_run_batch(plan.handle, [c], None, 0, None)
    assert e.value.code == fz.FZ_E_WORKSPACE
    bad = fz.fz_clip()
    bad.d_in, bad.d_out, bad.width, bad.height, bad.frames = 1, None, 320, 240, 10
    with pytest.raises(fz.FzError) as e:
        fz.fz_run_batch(plan.handle, [c, bad], 1, 1 << 20, None)
    assert e.value.code == fz.FZ_E_INVALID and "clip 1" in fz.fz_last_error()
    bad.d_out, bad.frames = 1, 0
    with pytest.raises(fz.FzError):
        fz.fz_run_batch(plan.handle, [bad], 1, 1 << 20, None)
    bad.frames, bad.point_capacity = 3, 10
    with pytest.raises(fz.FzError):
        fz.fz_run_batch(plan.handle, [bad], 1, 1 << 20, None)
    with pytest.raises(fz.FzError):
        fz.fz_run_batch(plan.handle, [], 1, 1 << 20, None)


def test_segment_config_override():
    p = fz.Plan(fz.RGB_HARRIS_CHAIN, 800, 600, 100, partition=[0, 7])
    info = p.segment_info()
    assert [s.engine for s in info] == [fz.FZ_ENGINE_STREAM, fz.FZ_ENGINE_ROW, fz.FZ_ENGINE_STREAM]
    fz.fz_plan_set_segment_config(p.handle, 1, "tile", 32, 32)
    s = p.segment_info()[1]
    assert (s.engine, s.tile_w, s.tile_h) == (fz.FZ_ENGINE_TILE, 32, 32)
    fz.fz_plan_set_segment_config(p.handle, 1, "row", 0, 50, 0)
    s = p.segment_info()[1]
    assert (s.engine, s.tile_h) == (fz.FZ_ENGINE_ROW, 50)
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_set_segment_config(p.handle, 1, "tile", 48, 48)
    assert e.value.code == fz.FZ_E_UNSUPPORTED
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_set_segment_config(p.handle, 0, "row", 0, 50, 0)
    assert e.value.code == fz.FZ_E_UNSUPPORTED
    with pytest.raises(fz.FzError):
        fz.fz_plan_set_segment_config(p.handle, 3, "auto")
    # the plan's total follows the group prices
    assert p.cost == sum(s.cost for s in p.segment_info())


def test_measure_workspace_and_errors_before_any_launch():
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, 800, 600, 10)
    # three buffers of the largest stage output (3 x f32 = 12 B/px) and a counter
    slot = (800 * 600 * 10 * 12 + 255) // 256 * 256
    # ... and the largest single-group workspace of a timed group: here the
    # frame-boundary exchange of a fused frame-difference row group
    extra = fz.fz_measure_workspace_bytes(plan.handle) - (3 * slot + 256)
    assert extra >= plan.workspace_bytes > 0 and extra % 256 == 0
    fake = 0x1000  # never dereferenced: the checks come first
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_measure(plan.handle, fake, fake, 100, 3, None)
    assert e.value.code == fz.FZ_E_WORKSPACE
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_measure(plan.handle, fake, fake, 1 << 40, 0, None)
    assert e.value.code == fz.FZ_E_INVALID
    with pytest.raises(fz.FzError) as e:
        fz.fz_plan_measure(plan.handle, None, fake, 1 << 40, 3, None)
    assert e.value.code == fz.FZ_E_INVALID
    # the measured model plans with bytes until measured
    p2 = fz.fz_plan_chain(plan.stages, fz.make_opts(800, 600, 10, cost_model="measured"))
    assert fz.fz_plan_cost(p2) == plan.cost
    fz.fz_plan_destroy(p2)


def test_band_and_frame_run_requests_are_kept_or_refused():
    """A requested band height or frame run is either kept as given or refused
    with FZ_E_UNSUPPORTED, never replaced by another shape."""
    W, H, T = 800, 600, 1000
    # a band of 300 rows on a group ending in the frame difference is over what
    # the kernel's previous-frame LDS rows allow: refused, through fz_plan_chain
    with pytest.raises(fz.FzError) as e:
        fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T, engine="row", band_h=300, frames_per_block=8)
    assert e.value.code == fz.FZ_E_UNSUPPORTED and "256" in str(e.value)
    # kept: band and frame run exactly as requested
    for band, run in [(256, 8), (55, 16), (8, 1), (100, 3)]:
        s = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T, engine="row", band_h=band, frames_per_block=run).segment_info()
        assert len(s) == 1 and s[0].engine == fz.FZ_ENGINE_ROW
        assert (s[0].tile_h, s[0].frames_per_block) == (band, run)
        assert s[0].lds_bytes == 4 * 64 * band <= 65536
    # a frame run longer than the video is the whole video; a band taller
    # than the frame is the whole frame
    s = fz.Plan(fz.HARRIS_CHAIN, 192, 200, 5, engine="row", band_h=250, frames_per_block=24).segment_info()[0]
    assert (s.tile_h, s.frames_per_block) == (200, 5)
    # groups without the frame difference take tall bands
    s = fz.Plan(fz.RGB_HARRIS_CHAIN[:8], W, H, T, engine="row", band_h=300).segment_info()[0]
    assert s.engine == fz.FZ_ENGINE_ROW and s.tile_h == 300 and s.lds_bytes == 0
    # through fz_plan_set_segment_config: refused, and the plan is unchanged
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T)
    before = (plan.segment_info()[0].tile_h, plan.segment_info()[0].frames_per_block, plan.cost)
    with pytest.raises(fz.FzError) as e:
        plan.set_segment_config(0, "row", (0, 300), 8)
    assert e.value.code == fz.FZ_E_UNSUPPORTED
    assert (plan.segment_info()[0].tile_h, plan.segment_info()[0].frames_per_block, plan.cost) == before
    plan.set_segment_config(0, "row", (0, 120), 40)
    s = plan.segment_info()[0]
    assert (s.tile_h, s.frames_per_block) == (120, 40)


def test_row_sizing_model_prefers_short_runs_and_full_rounds():
    """The row kernel's band x run model (total work x (1 + 1/rounds)): with the
    frame-boundary exchange the 800x600x1000 RGB chain gets 2-frame runs and a
    band of 55-100 rows (the measured sweep's best region), at least four
    rounds of wavefronts, and a workspace holding the exchange words."""
    W, H, T = 800, 600, 1000
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T)
    (s,) = plan.segment_info()
    assert s.engine == fz.FZ_ENGINE_ROW and s.frames_per_block == 2 and 55 <= s.tile_h <= 100
    strips = -(-(W - 128) // 116) + 1
    items = strips * -(-H // s.tile_h) * -(-T // s.frames_per_block)
    assert items >= 4 * 5120
    bounds = strips * -(-H // s.tile_h) * (-(-T // s.frames_per_block) - 1)
    assert plan.workspace_bytes >= bounds * (2 * s.tile_h * 2 * 8 + 4)
    # one run covering the clip: no boundaries, no workspace
    one = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T, engine="row", band_h=75, frames_per_block=T)
    assert one.workspace_bytes == 0
