"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Sizes span several tiles with ragged right/bottom tails; the full-size cases
use the launch configuration the benchmark times and compare sampled frames.
Fused and unfused runs share the per-pixel arithmetic, so their outputs must
be identical bit for bit whatever the partition.
"""
import itertools

import numpy as np
import pytest

import oracle
from paper_1509_04394_amd import fz, synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-parity]", *a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def run_gpu(ops, vol, dev, partition="optimal", **kw):
    """Run ops over numpy volume `vol` on the GPU; returns (out numpy, points numpy|None, plan)."""
    v = np.ascontiguousarray(vol)
    if ops[0] == "rgb2gray":
        T, H, W, _ = v.shape
    elif v.ndim == 3:
        T, H, W = v.shape
    else:
        _, T, H, W = v.shape
    plan = fz.Plan(ops, W, H, T, partition=partition, **kw)
    x = torch.from_numpy(v).to(dev)
    out, pts, cnt = plan.run(x)
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    p = fz.points_to_numpy(pts, cnt) if pts is not None else None
    return o, p, plan


def oracle_run(ops, vol):
    return oracle.chain(ops, vol)


def as_planes(o):
    return o[None] if o.ndim == 3 else o


# ---------------------------------------------------------------- point stages, exact
def test_rgb2gray_every_triple(dev):
    say("rgb2gray over all 2^24 RGB triples")
    v = np.arange(1 << 24, dtype=np.uint32)
    rgb = np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], -1).astype(np.uint8).reshape(1, 4096, 4096, 3)
    g, _, _ = run_gpu(["rgb2gray"], rgb, dev)
    c = rgb.astype(np.int64)
    ref = (299 * c[..., 0] + 587 * c[..., 1] + 114 * c[..., 2] + 500) // 1000
    o, _ = oracle_run(["rgb2gray"], rgb[:, :64])  # the oracle on a slice pins ref's formula
    assert np.array_equal(o[0], ref[:, :64])
    assert np.array_equal(g, ref.astype(np.uint8))


def test_decisions_bit_exact(dev):
    """Threshold, suppression and frame difference on the same FP32 responses:
    no floating-point arithmetic is involved, so everything is exact."""
    ops = ["threshold", "nms3", "framediff"]
    for shape in [(5, 37, 70), (3, 1, 9), (2, 66, 1), (4, 130, 90)]:
        say("decisions", shape)
        R = synth.response_field(shape, seed=sum(shape), thr=parity.THR)
        for part in ["unfused", "optimal", [0], [1]]:
            g, gp, _ = run_gpu(ops, R[None], dev, partition=part)
            o, op_ = oracle_run(ops, R[None])
            assert np.array_equal(g, o[0].astype(np.uint8)), part
            m, mp, _ = run_gpu(ops[:2], R[None], dev, partition=part if part != [1] else "optimal")
            mo, _ = oracle_run(ops[:2], R[None])
            assert np.array_equal(m, mo[0].astype(np.uint8))
            key = lambda p: sorted(map(tuple, p.tolist()))
            assert key(gp) == key(op_), part
            assert key(mp) == key(op_)


# ---------------------------------------------------------------- FP32 stages vs oracle
PREFIXES = [fz.RGB_HARRIS_CHAIN[:k] for k in range(2, 8)]


@pytest.mark.parametrize("partition", ["unfused", "optimal"])
def test_stage_prefixes_within_tolerance(dev, partition):
    rgb = synth.video(150, 70, 5, seed=21, rgb=True)
    for ops in PREFIXES:
        say("prefix", ops[-1], partition)
        g, _, _ = run_gpu(ops, rgb, dev, partition=partition)
        o, _ = oracle_run(ops, rgb)
        err = np.abs(g.astype(np.float64) - o).max()
        assert err <= parity.fp_tol(ops[-1]), (ops[-1], err, parity.fp_tol(ops[-1]))


def test_isolated_float_stages(dev):
    cases = [
        (["sobel3"], synth.field_f32((1, 3, 45, 77), 31, 0, 255)),
        (["gradmag"], synth.field_f32((2, 3, 20, 33), 32, -1020, 1020)),
        (["products"], synth.field_f32((2, 3, 20, 33), 33, -1020, 1020)),
        (["boxsum5"], synth.field_f32((3, 2, 40, 70), 34, -1.0e6, 1.0e6)),
        (["harris"], synth.field_f32((3, 2, 20, 33), 35, 0, 2.6e7)),
        (["sobel3", "products", "boxsum5", "harris"], synth.field_f32((1, 2, 50, 90), 36, 0, 255)),
    ]
    for ops, f in cases:
        for part in ["unfused", "optimal"]:
            say("isolated", ops, part)
            g, _, _ = run_gpu(ops, f, dev, partition=part)
            o, _ = oracle_run(ops, f)
            err = np.abs(as_planes(g).astype(np.float64) - o).max()
            assert err <= parity.fp_tol(ops[-1]), (ops, err)


def check_full_chain(ops, vol, g, gp, o=None, op_=None, skip=0):
    """Mask / frame difference / points against the oracle.  A difference is
    only ever allowed inside both exemption sets (the literal 1e-5-of-threshold
    rule and the FP32 error model); on these seeded workloads no pixel and no
    point differs at all, so no exemption is used: asserted.  The sizes of the
    two sets (pixels whose decision FP32 rounding could flip) are reported."""
    st = parity.check_chain(oracle, ops, vol, g, gp, skip)
    say("stats", st)
    assert st["px_differ"] == 0 and st["points_differ"] == 0, st
    return st


PARTITIONS = ["unfused", "optimal", [1], [2, 5], [0, 3, 6], [4], [7], [0, 1, 2, 3, 4, 5, 6]]


@pytest.mark.parametrize("partition", PARTITIONS, ids=str)
def test_full_rgb_chain_vs_oracle(dev, partition):
    ops = fz.RGB_HARRIS_CHAIN
    rgb = synth.video(150, 70, 6, seed=22, rgb=True)
    say("full chain", partition)
    g, gp, _ = run_gpu(ops, rgb, dev, partition=partition)
    st = check_full_chain(ops, rgb, g, gp)
    assert st["points_oracle"] > 0


def test_every_partition_bitwise_equal(dev):
    """All 2^8 partitions of the 9-stage chain give the same bytes and points."""
    ops = fz.RGB_HARRIS_CHAIN
    rgb = synth.video(70, 45, 4, seed=23, rgb=True)
    ref, refp, _ = run_gpu(ops, rgb, dev, partition="unfused")
    key = lambda p: sorted(map(tuple, p.tolist()))
    n = len(ops)
    for bits in itertools.product((0, 1), repeat=n - 1):
        cuts = [i for i, b in enumerate(bits) if b]
        g, gp, _ = run_gpu(ops, rgb, dev, partition=cuts)
        assert np.array_equal(g, ref), cuts
        assert key(gp) == key(refp), cuts
    # float-output groups too: every partition of the prefix ending at harris
    pre = ops[:6]
    fref, _, _ = run_gpu(pre, rgb, dev, partition="unfused")
    for bits in itertools.product((0, 1), repeat=len(pre) - 1):
        cuts = [i for i, b in enumerate(bits) if b]
        g, _, _ = run_gpu(pre, rgb, dev, partition=cuts)
        assert np.array_equal(g, fref), cuts


def test_grad_chain_all_partitions(dev):
    v = synth.video(192, 432, 8, seed=1)
    o, _ = oracle_run(fz.GRAD_CHAIN, v)
    ref = None
    for cuts in [[], [0], [1], [0, 1]]:
        say("grad chain", cuts)
        g, _, _ = run_gpu(fz.GRAD_CHAIN, v, dev, partition=cuts)
        err = np.abs(g.astype(np.float64) - o).max()
        assert err <= parity.fp_tol("gradmag"), err
        if ref is None:
            ref = g
        assert np.array_equal(g, ref)


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (9, 1), (7, 9), (2, 3), (64, 16), (65, 33)])
def test_tiny_and_ragged_frames(dev, shape):
    W, H = shape
    ops = fz.HARRIS_CHAIN
    rng = np.random.default_rng(W * 100 + H)
    v = synth.video(W, H, 3, seed=24) if min(W, H) >= 8 else rng.integers(0, 256, (3, H, W), dtype=np.uint8)
    say("tiny", shape)
    for part in ["unfused", "optimal", [3]]:
        g, gp, _ = run_gpu(ops, v, dev, partition=part)
        check_full_chain(ops, v, g, gp)
    g, _, _ = run_gpu(ops[:3], v, dev)
    o3, _ = oracle_run(ops[:3], v)
    assert np.abs(g.astype(np.float64) - o3).max() <= parity.fp_tol("products")


def test_tiles_and_frames_per_block_do_not_change_results(dev):
    ops = fz.RGB_HARRIS_CHAIN
    rgb = synth.video(150, 70, 7, seed=25, rgb=True)
    ref, refp, _ = run_gpu(ops, rgb, dev, partition="unfused")
    key = lambda p: sorted(map(tuple, p.tolist()))
    for tile in [(64, 16), (32, 32), (64, 32)]:
        for tpb in [1, 2, 3, 7, 12]:
            say("tile", tile, "tpb", tpb)
            g, gp, plan = run_gpu(ops, rgb, dev, tile=tile, frames_per_block=tpb)
            assert plan.segment_info()[0].tile_w == tile[0]
            assert np.array_equal(g, ref) and key(gp) == key(refp), (tile, tpb)


def test_point_capacity_overflow_counts(dev):
    ops = fz.HARRIS_CHAIN
    v = synth.video(192, 432, 4, seed=26)
    plan = fz.Plan(ops, 192, 432, 4)
    x = torch.from_numpy(v).to(dev)
    out, pts, cnt, ws = plan.alloc(dev, point_capacity=5)
    plan.run(x, out, pts, cnt, ws)
    torch.cuda.synchronize()
    full_out, full_p, _ = run_gpu(ops, v, dev)
    assert int(cnt.item()) == len(full_p) > 5
    raw = pts.cpu().numpy()
    got = {tuple(r) for r in raw[:, :3].view(np.uint32).tolist()}
    assert got <= {tuple(r) for r in full_p[:, :3].astype(np.uint32).tolist()}
    assert np.array_equal(out.cpu().numpy(), full_out)


# ---------------------------------------------------------------- workload sizes
def test_gradient_config_full(dev):
    """192x432x64 gray, Gaussian -> Sobel -> magnitude, whole volume vs oracle."""
    v = synth.video(192, 432, 64, seed=1)
    g, _, _ = run_gpu(fz.GRAD_CHAIN, v, dev)
    o, _ = oracle_run(fz.GRAD_CHAIN, v)
    assert np.abs(g.astype(np.float64) - o).max() <= parity.fp_tol("gradmag")


def test_harris_config_full(dev):
    """192x432x600 gray, 8-stage chain, planner's partition, whole volume vs oracle."""
    v = synth.video(192, 432, 600, seed=2)
    g, gp, plan = run_gpu(fz.HARRIS_CHAIN, v, dev)
    say("segments", plan.segments)
    check_full_chain(fz.HARRIS_CHAIN, v, g, gp)
    u, up, _ = run_gpu(fz.HARRIS_CHAIN, v, dev, partition="unfused")
    assert np.array_equal(u, g)


def test_rgb_config_full_size_vs_oracle(dev):
    """800x600x1000 RGB, the benchmark's plan: fused == unfused over the whole
    volume, and every one of the 1000 frames against the oracle, in chunks of
    100 frames (each chunk starts one frame early: the frame difference's
    temporal halo)."""
    W, H, T = 800, 600, 1000
    ops = fz.RGB_HARRIS_CHAIN
    say("generating 800x600x1000 RGB")
    rgb = synth.video(W, H, T, seed=3, rgb=True)
    x = torch.from_numpy(rgb).to(dev)
    fused = fz.Plan(ops, W, H, T)
    out, pts, cnt = fused.run(x)
    torch.cuda.synchronize()
    g = out.cpu().numpy()
    gp = fz.points_to_numpy(pts, cnt)
    say("fused points", len(gp))
    del out, pts
    unf = fz.Plan(ops, W, H, T, partition="unfused")
    uo, upts, ucnt = unf.run(x)
    torch.cuda.synchronize()
    assert np.array_equal(uo.cpu().numpy(), g)
    up = fz.points_to_numpy(upts, ucnt)
    key = lambda p: sorted(map(tuple, p.tolist()))
    assert key(up) == key(gp)
    del uo, upts, x
    torch.cuda.empty_cache()
    total = {}
    for c0 in range(0, T, 100):
        s, e = max(c0 - 1, 0), min(c0 + 100, T)
        sel = (gp[:, 0] >= s) & (gp[:, 0] < e)
        gps = gp[sel].copy()
        gps[:, 0] -= s
        st = parity.check_chain(oracle, ops, rgb[s:e], g[s:e], gps, skip=c0 - s)
        parity.add_stats(total, st)
        say("frames", c0, e - 1, st)
    say("all frames", total)
    assert total["points_gpu"] == len(gp) > 0
    # no decision differs at all on this seeded video
    assert total["px_differ"] == 0 and total["points_differ"] == 0, total


# ---------------------------------------------------------------- row-marching engine
ROW_SHAPES = [(128, 9, 3), (150, 70, 5), (192, 100, 4), (257, 33, 6), (300, 40, 3), (800, 64, 3)]


@pytest.mark.parametrize("shape", ROW_SHAPES, ids=lambda s: "x".join(map(str, s)))
def test_row_engine_equals_tile_engine(dev, shape):
    """The row-marching kernel computes the same bytes and points as the LDS
    tile engine for every group it implements, whatever the band height and
    frames per work item."""
    W, H, T = shape
    rgb = synth.video(W, H, T, seed=W + H, rgb=True)
    gray = synth.video(W, H, T, seed=W + H + 1)
    key = lambda p: sorted(map(tuple, p.tolist()))
    for ops, vol in [(fz.RGB_HARRIS_CHAIN, rgb), (fz.RGB_HARRIS_CHAIN[:8], rgb),
                     (fz.HARRIS_CHAIN, gray), (fz.HARRIS_CHAIN[:7], gray)]:
        ref, refp, _ = run_gpu(ops, vol, dev, engine="tile")
        for band_h, tpb in [(0, 0), (8, 1), (17, 2), (H, T), (H // 2 + 1, 3)]:
            say("row engine", shape, len(ops), band_h, tpb)
            g, gp, plan = run_gpu(ops, vol, dev, engine="row", band_h=band_h, frames_per_block=tpb)
            assert plan.segment_info()[0].engine == fz.FZ_ENGINE_ROW
            assert np.array_equal(g, ref), (ops[-1], band_h, tpb)
            assert key(gp) == key(refp), (ops[-1], band_h, tpb)


def test_row_frame_boundary_exchange(dev):
    """Frame-difference row groups: the item of a run takes the mask of the
    frame before it from the previous run's item (whichever of the two ends
    second writes that frame's difference).  Runs of 1 .. T frames, a run
    length that does not divide T, and repeated runs on one workspace (the
    arrival counters are cleared by each launch) give the tile engine's
    bytes and points."""
    W, H, T = 300, 40, 23
    rgb = synth.video(W, H, T, seed=91, rgb=True)
    key = lambda p: sorted(map(tuple, p.tolist()))
    ref, refp, _ = run_gpu(fz.RGB_HARRIS_CHAIN, rgb, dev, engine="tile")
    x = torch.from_numpy(rgb).to(dev)
    for band_h, tpb in [(8, 1), (13, 2), (40, 5), (21, 22), (40, 23)]:
        plan = fz.Plan(fz.RGB_HARRIS_CHAIN, W, H, T, partition=[], engine="row", band_h=band_h,
                       frames_per_block=tpb)
        s = plan.segment_info()[0]
        assert s.engine == fz.FZ_ENGINE_ROW and s.frames_per_block == tpb
        out, pts, cnt, ws = plan.alloc(dev, point_capacity=1 << 16)
        if tpb < T:
            assert plan.workspace_bytes > 0
        for rep in range(2):
            say("row exchange", band_h, tpb, rep)
            out.zero_()
            plan.run(x, out, pts, cnt, ws)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), ref), (band_h, tpb, rep)
            assert key(fz.points_to_numpy(pts, cnt)) == key(refp), (band_h, tpb, rep)


def test_row_engine_vs_oracle(dev):
    ops = fz.RGB_HARRIS_CHAIN
    rgb = synth.video(300, 120, 7, seed=40, rgb=True)
    g, gp, plan = run_gpu(ops, rgb, dev, engine="row")
    assert plan.segment_info()[0].engine == fz.FZ_ENGINE_ROW
    st = check_full_chain(ops, rgb, g, gp)
    assert st["points_oracle"] > 0


GEN_SHAPES = [(128, 8, 3), (150, 70, 5), (257, 40, 4)]


@pytest.mark.parametrize("shape", GEN_SHAPES, ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("chain", ["rgb", "grad"])
def test_generic_row_groups_equal_tile_engine(dev, shape, chain):
    """Every contiguous group with a window stage: the generic row kernel gives
    the tile engine's bytes and points on real intermediate inputs."""
    W, H, T = shape
    ops = fz.RGB_HARRIS_CHAIN if chain == "rgb" else fz.GRAD_CHAIN
    vid = torch.from_numpy(synth.video(W, H, T, seed=W * 7 + H, rgb=chain == "rgb")).to(dev)
    ins = [vid]
    for a in range(1, len(ops)):
        out, _, _ = fz.Plan(ops[:a], W, H, T, engine="tile").run(vid)
        ins.append(out)
    torch.cuda.synchronize()
    windows = {"gauss5", "sobel3", "boxsum5", "nms3"}
    key = lambda p: sorted(map(tuple, p.tolist()))
    n = 0
    for a in range(len(ops)):
        for b in range(a, len(ops)):
            if not windows & set(ops[a:b + 1]):
                continue
            sub = ops[a:b + 1]
            pr = fz.Plan(sub, W, H, T, partition=[], engine="row")
            pt = fz.Plan(sub, W, H, T, partition=[], engine="tile")
            assert pr.segment_info()[0].engine == fz.FZ_ENGINE_ROW
            assert pt.segment_info()[0].engine == fz.FZ_ENGINE_TILE
            ro, rp, rc = pr.run(ins[a])
            to, tp, tc = pt.run(ins[a])
            torch.cuda.synchronize()
            assert torch.equal(ro, to), (sub, shape)
            if rp is not None:
                assert key(fz.points_to_numpy(rp, rc)) == key(fz.points_to_numpy(tp, tc)), (sub, shape)
            n += 1
    say("generic row groups", chain, shape, n)


def test_every_partition_bitwise_equal_row_width(dev):
    """All 2^8 partitions at a width where every group runs row-marching."""
    ops = fz.RGB_HARRIS_CHAIN
    rgb = synth.video(150, 40, 4, seed=31, rgb=True)
    ref, refp, _ = run_gpu(ops, rgb, dev, partition="unfused", engine="tile")
    key = lambda p: sorted(map(tuple, p.tolist()))
    for bits in itertools.product((0, 1), repeat=len(ops) - 1):
        cuts = [i for i, b in enumerate(bits) if b]
        g, gp, plan = run_gpu(ops, rgb, dev, partition=cuts)
        assert np.array_equal(g, ref), cuts
        assert key(gp) == key(refp), cuts
