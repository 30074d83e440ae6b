"""GPU parity of generic chains (point, weighted stencil, window sum) through
the C ABI, against the FP64 oracle.

Every output pixel must lie within the FP32 forward-error bound that
tests/parity.py propagates from the oracle's exact intermediates; every
partition and every tile shape must give the same bits (each stage's result
is rounded to FP32 once, in a fixed order, whichever kernel holds it).  Sizes
span several tiles with ragged right and bottom tails; the edge cases are
frames smaller than the window, one-pixel frames, point-only chains, a group
whose LDS box exceeds 64 KB, weights changed after planning, and a batch
of generic clips (graph replay included).
"""
import itertools

import numpy as np
import pytest

from paper_1509_04394_amd import fz, synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-generic]", *a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def run_gpu(spec, vol, dev, partition="optimal", in_dtype="u8", configs=None, **kw):
    T, H, W = vol.shape
    plan = fz.Plan(spec, W, H, T, partition=partition, in_dtype=in_dtype, **kw)
    for i, cfg in (configs or {}).items():
        plan.set_segment_config(i, **cfg)
    x = torch.from_numpy(np.ascontiguousarray(vol if in_dtype == "u8" else vol[None].astype(np.float32))).to(dev)
    out, _, _ = plan.run(x)
    torch.cuda.synchronize()
    return out.cpu().numpy()[0], plan


W3 = (np.arange(9, dtype=np.float32).reshape(3, 3) - 4.0) / 20.0  # asymmetric, signed
WELL = [  # well-conditioned: positive weights, no cancellation
    ("point", "affine", 0.5, 3.0),
    ("stencil", 2, 1, np.full((3, 5), 1.0 / 15.0, np.float32)),
    ("box", 1, 2),
    ("point", "sqrtabs", 0.0, 0.0),
    ("stencil", 1, 1, np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]], np.float32) / 16.0),
    ("point", "clamp", 2.0, 40.0),
]


@pytest.mark.parametrize("seed", [5000, 5001, 5002, 5004, 5007, 5011])
def test_random_chain_within_fp32_bound(dev, oracle_lib, seed):
    spec = synth.random_chain(seed)
    vol = synth.video(150, 70, 3, seed=seed)
    say("random chain", seed, "stages", len(spec), "size 150x70x3")
    ref, bound = parity.generic_reference(oracle_lib, spec, vol)
    if not np.isfinite(ref).all() or np.abs(ref).max() > 1e30:
        pytest.skip("chain leaves the FP32 range on this input")
    out, plan = run_gpu(spec, vol, dev)
    ratio = parity.assert_within_bound(out, ref, bound, f"seed {seed} {plan.segments}")
    err = float(np.abs(out.astype(np.float64) - ref).max())
    say("segments", plan.segments, "worst err/bound", ratio,
        "err over the 1e-4-on-0..255 tolerance", err / parity.north_star_tol(spec))
    un, _ = run_gpu(spec, vol, dev, partition="unfused")
    assert np.array_equal(un.view(np.uint32), out.view(np.uint32))


def test_well_conditioned_chain_is_tight(dev, oracle_lib):
    vol = synth.video(203, 77, 4, seed=21)
    ref, bound = parity.generic_reference(oracle_lib, WELL, vol)
    assert (bound <= 1e-5 * np.abs(ref).max()).all()  # the bound itself is small here
    out, plan = run_gpu(WELL, vol, dev)
    parity.assert_within_bound(out, ref, bound, "well-conditioned")
    err = float(np.abs(out - ref).max())
    tol = parity.north_star_tol(WELL)
    say("well-conditioned: max abs err", err, "= %.3g of the 1e-4-on-0..255 tolerance" % (err / tol),
        "segments", plan.segments)
    assert err <= tol, (err, tol)


def test_generic_workload_full_size_within_tolerance(dev, oracle_lib):
    """The benchmark's generic chain (3x3 binomial stencil -> |x| -> 3x3
    window sum, one fused tile kernel) over the whole 800x600x64 video, against
    the oracle, within 1e-4 on a 0..255 scale and within the FP32 bound."""
    spec = [("stencil", 1, 1, (np.outer([1, 2, 1], [1, 2, 1]) / 16.0).astype(np.float32)),
            ("point", "abs", 0.0, 0.0), ("box", 1, 1)]
    vol = synth.video(800, 600, 64, seed=6)
    ref, bound = parity.generic_reference(oracle_lib, spec, vol)
    out, plan = run_gpu(spec, vol, dev)
    assert plan.segments == [2]
    parity.assert_within_bound(out, ref, bound, "generic 800x600x64")
    err = float(np.abs(out - ref).max())
    tol = parity.north_star_tol(spec)
    say("generic 800x600x64: max abs err", err, "tolerance", tol, "ratio", err / tol)
    assert err <= tol, (err, tol)


@pytest.mark.parametrize("size", [(70, 45, 2), (131, 40, 1)])
def test_every_partition_same_bits(dev, oracle_lib, size):
    spec = WELL[:5] + [("stencil", 1, 1, W3)]
    n = len(spec)
    W, H, T = size
    vol = synth.video(W, H, T, seed=31)
    ref, bound = parity.generic_reference(oracle_lib, spec, vol)
    first = None
    for bits in itertools.product((0, 1), repeat=n - 1):
        cuts = [i for i, b in enumerate(bits) if b]
        out, _ = run_gpu(spec, vol, dev, partition=cuts)
        if first is None:
            first = out
            parity.assert_within_bound(out, ref, bound, "partition")
        else:
            assert np.array_equal(out.view(np.uint32), first.view(np.uint32)), cuts
    say("all", 2 ** (n - 1), "partitions identical at", size)


@pytest.mark.parametrize("tile", [(64, 16), (32, 32), (64, 32)])
def test_every_tile_same_bits(dev, tile):
    spec = WELL
    vol = synth.video(150, 70, 2, seed=41)
    base, _ = run_gpu(spec, vol, dev)
    out, plan = run_gpu(spec, vol, dev, configs={0: {"engine": "tile", "tile": tile}})
    assert plan.segment_info()[0].tile_w == tile[0]
    assert np.array_equal(out.view(np.uint32), base.view(np.uint32))


@pytest.mark.parametrize("size", [(3, 2, 2), (1, 1, 3), (7, 1, 1), (1, 9, 2)])
def test_frames_smaller_than_the_window(dev, oracle_lib, size):
    W, H, T = size
    spec = [("stencil", 3, 2, np.random.default_rng(1).standard_normal((5, 7)).astype(np.float32)),
            ("box", 3, 3), ("point", "abs", 0, 0)]
    vol = synth.video(max(W, 8), max(H, 8), T, seed=51)[:, :H, :W].copy()
    ref, bound = parity.generic_reference(oracle_lib, spec, vol)
    out, _ = run_gpu(spec, vol, dev)
    parity.assert_within_bound(out, ref, bound, f"size {size}")


def test_point_only_chain_f32_input(dev, oracle_lib):
    spec = [("point", "affine", -1.5, 7.25), ("point", "square", 0, 0), ("point", "sqrtabs", 0, 0),
            ("point", "clamp", -3.0, 90.0), ("point", "abs", 0, 0)]
    vol = np.random.default_rng(61).uniform(-100, 100, (3, 33, 129)).astype(np.float32)
    ref, bound = parity.generic_reference(oracle_lib, spec, vol.astype(np.float64))
    out, plan = run_gpu(spec, vol, dev, in_dtype="f32")
    assert plan.segment_info()[0].engine == fz.FZ_ENGINE_STREAM
    parity.assert_within_bound(out, ref, bound, "point-only")


def test_lds_box_above_64k(dev, oracle_lib):
    # eight 7x7 stencils: halo 24 per side; the 64x32 tile's two f32 boxes take 70 KB
    rng = np.random.default_rng(71)
    spec = []
    for _ in range(8):
        w = rng.uniform(0.1, 1.0, (7, 7))
        spec.append(("stencil", 3, 3, (w / w.sum()).astype(np.float32)))
    vol = synth.video(140, 90, 2, seed=72)
    out, plan = run_gpu(spec, vol, dev)
    info = plan.segment_info()
    assert len(info) == 1 and info[0].lds_bytes > 65536
    ref, bound = parity.generic_reference(oracle_lib, spec, vol)
    parity.assert_within_bound(out, ref, bound, "64 KB+ LDS")
    say("lds", info[0].lds_bytes, "tile", info[0].tile_w, info[0].tile_h)


def test_weights_are_copied_at_plan_time(dev, oracle_lib):
    w = np.array([[0.0, 1.0, 0.0], [1.0, -4.0, 1.0], [0.0, 1.0, 0.0]], np.float32)
    spec = [("stencil", 1, 1, w)]
    vol = synth.video(64, 48, 2, seed=81)
    T, H, W = vol.shape
    stages, keep = fz.generic_stages(spec)
    plan = fz.fz_plan_chain(stages, fz.make_opts(W, H, T))
    keep[0][4] = 100.0  # change the caller's array after planning
    x = torch.from_numpy(vol).to(dev)
    out = torch.empty((1, T, H, W), dtype=torch.float32, device=dev)
    fz.fz_run_chain(plan, x.data_ptr(), out.data_ptr(), None, None, 0, None, 0,
                    torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    fz.fz_plan_destroy(plan)
    ref, bound = parity.generic_reference(oracle_lib, spec, vol)
    parity.assert_within_bound(out.cpu().numpy()[0], ref, bound, "copied weights")


def test_random_chain_full_size_config(dev, oracle_lib):
    # the cost-model workload shape: a 192 x 432 frame, 64 frames
    spec = synth.random_chain(5005)
    vol = synth.video(192, 432, 64, seed=5005)
    say("full-size random chain, stages", len(spec))
    ref, bound = parity.generic_reference(oracle_lib, spec, vol)
    if not np.isfinite(ref).all() or np.abs(ref).max() > 1e30:
        pytest.skip("chain leaves the FP32 range on this input")
    out, plan = run_gpu(spec, vol, dev)
    ratio = parity.assert_within_bound(out, ref, bound, "full size")
    say("segments", plan.segments, "worst err/bound", ratio)


def test_batch_of_generic_clips_equals_single_runs(dev):
    """fz_run_batch on a generic plan (clips run one after another inside the
    captured graph): every clip equals a single run bit for bit, on the first
    launch and on a graph replay."""
    spec = WELL[:4] + [("box", 2, 1)]
    sizes = [(150, 70, 3), (64, 48, 5), (203, 77, 2)]
    xs, outs, refs = [], [], []
    for i, (W, H, T) in enumerate(sizes):
        x = torch.from_numpy(synth.video(W, H, T, seed=90 + i)).to(dev)
        ref, _ = run_gpu(spec, synth.video(W, H, T, seed=90 + i), dev)
        xs.append(x)
        outs.append(torch.full((1, T, H, W), float("nan"), dtype=torch.float32, device=dev))
        refs.append(ref)
    plan = fz.Plan(spec, 800, 600, 100)
    clips = [fz.make_clip(x, o) for x, o in zip(xs, outs)]
    for rep in range(2):
        for o in outs:
            o.fill_(float("nan"))
        ws = fz.run_batch(plan, clips) if rep == 0 else fz.run_batch(plan, clips, workspace=ws)
        torch.cuda.synchronize()
        for i, (o, ref) in enumerate(zip(outs, refs)):
            assert np.array_equal(o.cpu().numpy()[0].view(np.uint32), ref.view(np.uint32)), f"clip {i}, run {rep}"
