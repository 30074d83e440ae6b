"""GPU parity of the temporal generic stages through the C ABI, against the
FP64 oracle: Table II's IIR filter (a point operation over every earlier
frame) and stencils that also read the frames before t (Table I's
spatio-temporal class).

Every output pixel lies within the FP32 forward-error bound tests/parity.py
propagates (the IIR's own rule included); every partition, tile and frame run
gives the same bits, since each stage rounds the same operations in the same
order whichever kernel holds it (the streaming IIR kernel, the frame-marching
tile kernel, the plain tile kernel).  Sizes span several tiles with ragged
tails, frame counts that are not multiples of the frame run or of the
streaming kernel's eight-frame loads, and frames whose pixel count is not a
multiple of four (the streaming kernel's one-pixel path)."""
import itertools

import numpy as np
import pytest

import oracle
from paper_1509_04394_amd import fz, synth
from tests import parity

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-temporal]", *a, flush=True)


@pytest.fixture(scope="module")
def dev(oracle_lib):
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


A = float(np.float32(0.3))  # an FP32-exact coefficient, given to both sides
G5 = np.exp(-np.arange(-2, 3) ** 2 / 2.0)
G5 = (np.outer(G5, G5) / np.outer(G5, G5).sum()).astype(np.float32)
SOBEL_X = np.array([[-1, 0, 1], [-2, 0, 2], [-1, 0, 1]], np.float32)
# stencils that look back: rt = 2 (3x3) and rt = 1 (5x3, signed)
ST_T2 = (np.arange(27, dtype=np.float32).reshape(3, 3, 3) % 5 + 1.0) / 60.0
ST_T1 = ((np.arange(30, dtype=np.float32).reshape(2, 3, 5) % 7) - 3.0) / 40.0

# the paper's five-kernel chain with generic stages (gray input): IIR ->
# Gaussian -> gradient -> magnitude-like point op -> clamp
PAPER5 = [("iir", A), ("stencil", 2, 2, G5), ("stencil", 1, 1, SOBEL_X), ("point", "abs", 0.0, 0.0),
          ("point", "clamp", 0.0, 200.0)]
SPATIO = [("point", "affine", 0.5, 1.0), ("stencil", 1, 1, ST_T2), ("box", 1, 1), ("stencil", 2, 1, ST_T1),
          ("point", "sqrtabs", 0.0, 0.0)]
MIXED = [("stencil", 1, 1, ST_T2), ("iir", A), ("box", 2, 1), ("point", "abs", 0.0, 0.0), ("iir", float(np.float32(0.75)))]


def scale_spec(spec):
    """The stages whose full scale sets the 1e-4-of-full-scale tolerance: a
    trailing clamp narrows the output's range but not an absolute error that
    comes through it (it is 1-Lipschitz), so the scale is that of the chain
    before it."""
    return spec[:-1] if spec[-1][0] == "point" and spec[-1][1] == "clamp" else spec


def check(spec, vol, g, what):
    ref, bound = parity.generic_reference(oracle, spec, vol)
    worst = parity.assert_within_bound(g, ref, bound, what)
    err = float(np.abs(g.astype(np.float64) - ref).max())
    tol = parity.north_star_tol(scale_spec(spec))
    say(what, f"worst err/bound {worst:.3f}, max err {err:.3g} (1e-4 of full scale / 255: {tol:.3g})")
    return err, tol


@pytest.mark.parametrize("size", [(150, 70, 21), (37, 23, 11), (64, 32, 9)], ids=str)
def test_iir_alone_streaming(dev, size):
    W, H, T = size
    vol = synth.video(W, H, T, seed=61)
    for a in (A, 1.0, float(np.float32(0.05))):
        spec = [("iir", a)]
        g, plan = run_gpu(spec, vol, dev)
        assert plan.segment_info()[0].engine == fz.FZ_ENGINE_STREAM
        assert plan.segment_info()[0].frames_per_block == T
        err, tol = check(spec, vol, g, f"iir a={a} {size}")
        assert err <= tol
    # f32 input, point stages around the IIR
    f = synth.field_f32((1, T, H, W), 62, -100, 100)[0]
    spec = [("point", "square", 0.0, 0.0), ("iir", A), ("point", "sqrtabs", 0.0, 0.0)]
    g, _ = run_gpu(spec, f, dev, in_dtype="f32")
    check(spec, f, g, f"point-iir-point f32 {size}")


@pytest.mark.parametrize("spec_name", ["PAPER5", "SPATIO", "MIXED"])
def test_temporal_chain_vs_oracle(dev, spec_name):
    spec = globals()[spec_name]
    vol = synth.video(150, 70, 13, seed=63)
    for part in ["optimal", "unfused"]:
        g, plan = run_gpu(spec, vol, dev, partition=part)
        say(spec_name, part, plan.segments, [(s.engine, s.tile_w, s.tile_h, s.frames_per_block)
                                             for s in plan.segment_info()])
        err, tol = check(spec, vol, g, f"{spec_name} {part}")
        if spec_name == "PAPER5":
            assert err <= tol  # well conditioned: spec units hold too


@pytest.mark.parametrize("spec_name", ["PAPER5", "SPATIO", "MIXED"])
def test_every_partition_same_bits(dev, spec_name):
    spec = globals()[spec_name]
    vol = synth.video(90, 41, 7, seed=64)
    ref, _ = run_gpu(spec, vol, dev, partition="unfused")
    n = len(spec)
    for bits in itertools.product((0, 1), repeat=n - 1):
        cuts = [i for i, b in enumerate(bits) if b]
        g, _ = run_gpu(spec, vol, dev, partition=cuts)
        assert np.array_equal(g, ref), (spec_name, cuts)
    check(spec, vol, ref, f"{spec_name} all partitions")


@pytest.mark.parametrize("tile", [(64, 16), (32, 32), (64, 32)], ids=str)
def test_tiles_and_frame_runs_same_bits(dev, tile):
    vol = synth.video(133, 77, 17, seed=65)
    ref, _ = run_gpu(SPATIO, vol, dev, partition=[])
    for tpb in (1, 2, 5, 16, 17, 40):
        g, plan = run_gpu(SPATIO, vol, dev, partition=[], configs={0: dict(engine="tile", tile=tile,
                                                                            frames_per_block=tpb)})
        assert plan.segment_info()[0].frames_per_block == min(tpb, 17)
        assert np.array_equal(g, ref), (tile, tpb)
    # IIRs that lead the group resume from checkpoints: every frame run gives the same bits
    ref, _ = run_gpu(PAPER5, vol, dev, partition=[], configs={0: dict(engine="tile", tile=tile,
                                                                      frames_per_block=17)})
    for tpb in (1, 2, 5, 8, 16):
        g, plan = run_gpu(PAPER5, vol, dev, partition=[], configs={0: dict(engine="tile", tile=tile,
                                                                          frames_per_block=tpb)})
        assert plan.segment_info()[0].frames_per_block == tpb
        assert np.array_equal(g, ref), (tile, tpb)
    # an IIR after a window stage keeps whole-clip work items
    g, plan = run_gpu(MIXED, vol, dev, partition=[], configs={0: dict(engine="tile", tile=tile)})
    assert plan.segment_info()[0].frames_per_block == 17


@pytest.mark.parametrize("size", [(1, 1, 5), (3, 2, 4), (7, 5, 9), (200, 3, 6)], ids=str)
def test_tiny_and_thin_frames(dev, size):
    W, H, T = size
    vol = synth.video(max(W, 8), max(H, 8), T, seed=66)[:, :H, :W].copy()
    for spec in (PAPER5, SPATIO, MIXED):
        g, _ = run_gpu(spec, vol, dev)
        check(spec, vol, g, f"tiny {size}")


def test_single_frame_clip(dev):
    vol = synth.video(70, 45, 1, seed=67)
    for spec in (PAPER5, SPATIO, MIXED):
        g, _ = run_gpu(spec, vol, dev)
        check(spec, vol, g, "one frame")


def test_full_size_paper_chain_sampled(dev):
    """The paper's five-kernel chain (generic stages) at 800x600 over 300
    frames, as the benchmark runs it: frames 0-9 and 290-299 against the
    oracle (the oracle needs every earlier frame for the IIR, so it runs the
    first 300 frames and is compared on both ends)."""
    vol = synth.video(800, 600, 300, seed=68)
    g, plan = run_gpu(PAPER5, vol, dev)
    say("paper5 800x600x300", plan.segments, [(s.engine, s.tile_w, s.tile_h, s.frames_per_block)
                                             for s in plan.segment_info()])
    ref, bound = parity.generic_reference(oracle, PAPER5, vol)
    for sl in (slice(0, 10), slice(290, 300)):
        parity.assert_within_bound(g[sl], ref[sl], bound[sl], f"paper5 frames {sl}")
        assert float(np.abs(g[sl].astype(np.float64) - ref[sl]).max()) <= parity.north_star_tol(scale_spec(PAPER5))
