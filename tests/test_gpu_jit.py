"""Generated kernels (FZ_ENGINE_JIT: each generic group's kernel written out
with its stage list, radii, box sizes and weights as constants and compiled
with hipRTC) against the generic tile kernel and the oracle.

The generated kernel evaluates the same operations in the same order as the
tile kernel, so the outputs must be equal (in value) for every chain, tile,
partition and frame size; against the FP64 oracle they lie within the FP32
error bound of tests/parity.py."""
import numpy as np
import pytest

import oracle
from paper_1509_04394_amd import fz, synth
from tests import parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-jit]", *a, flush=True)


@pytest.fixture(scope="module")
def dev(oracle_lib):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def run(spec, vol, dev, **kw):
    T, H, W = vol.shape
    plan = fz.Plan(spec, W, H, T, **kw)
    out, _, _ = plan.run(torch.from_numpy(vol).to(dev))
    torch.cuda.synchronize()
    return out.cpu().numpy()[0], plan


W3 = (np.arange(9, dtype=np.float32).reshape(3, 3) - 4.0) / 20.0
CHAINS = {
    "well": [("point", "affine", 0.5, 3.0), ("stencil", 2, 1, np.full((3, 5), 1.0 / 15.0, np.float32)),
             ("box", 1, 2), ("point", "sqrtabs", 0.0, 0.0),
             ("stencil", 1, 1, np.array([[1, 2, 1], [2, 4, 2], [1, 2, 1]], np.float32) / 16.0),
             ("point", "clamp", 2.0, 40.0)],
    "signed": [("stencil", 1, 1, W3), ("point", "square", 0.0, 0.0), ("box", 3, 0), ("point", "abs", 0.0, 0.0),
               ("stencil", 0, 3, np.linspace(-1, 1, 7, dtype=np.float32).reshape(7, 1) / 4.0)],
    "random": synth.random_chain(5003),
}


@pytest.mark.parametrize("width", [203, 204], ids=["w203", "w204"])
@pytest.mark.parametrize("name", sorted(CHAINS))
def test_generated_equals_tile_kernel_and_oracle(dev, name, width):
    """Width 203: every tile loads its box cell by cell; width 204 (a
    multiple of four): tiles inside the frame across load four cells at a
    time, u8 in the first group and f32 in the later groups of the unfused
    partition."""
    spec = CHAINS[name]
    vol = synth.video(width, 117, 5, seed=71)
    for part in ("optimal", "unfused"):
        ref, _ = run(spec, vol, dev, partition=part)
        g, plan = run(spec, vol, dev, partition=part, engine="jit")
        say(name, part, [(s.engine, s.tile_w, s.tile_h) for s in plan.segment_info()])
        assert any(s.engine == fz.FZ_ENGINE_JIT for s in plan.segment_info())
        assert np.array_equal(g, ref), (name, part)
    ref_o, bound = parity.generic_reference(oracle, spec, vol)
    parity.assert_within_bound(g, ref_o, bound, f"jit {name}")


@pytest.mark.parametrize("tile", fz.JIT_TILES, ids=str)
def test_every_generated_tile_same_bits(dev, tile):
    spec = CHAINS["well"]
    vol = synth.video(150, 70, 3, seed=72)
    ref, _ = run(spec, vol, dev, partition=[])
    T, H, W = vol.shape
    plan = fz.Plan(spec, W, H, T, partition=[])
    plan.set_segment_config(0, engine="jit", tile=tile)
    assert plan.segment_info()[0].engine == fz.FZ_ENGINE_JIT
    out, _, _ = plan.run(torch.from_numpy(vol).to(dev))
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy()[0], ref), tile


def test_frames_per_work_item(dev):
    """A group without temporal stages marching several frames per work item
    (the input box of the next frame loaded while the current one is
    computed): any run length, including one that does not divide the clip
    and one longer than it, gives the tile kernel's values."""
    spec = CHAINS["well"]
    vol = synth.video(204, 70, 7, seed=77)
    ref, _ = run(spec, vol, dev, partition=[])
    T, H, W = vol.shape
    plan = fz.Plan(spec, W, H, T, partition=[], engine="jit")
    assert plan.segment_info()[0].frames_per_block >= 1
    for tpb in (1, 2, 3, 4, 7, 9):
        plan = fz.Plan(spec, W, H, T, partition=[])
        plan.set_segment_config(0, engine="jit", tile=(64, 32), frames_per_block=tpb)
        assert plan.segment_info()[0].frames_per_block == min(tpb, T)
        out, _, _ = plan.run(torch.from_numpy(vol).to(dev))
        torch.cuda.synchronize()
        assert np.array_equal(out.cpu().numpy()[0], ref), tpb


@pytest.mark.parametrize("size", [(1, 1, 2), (7, 5, 3), (200, 3, 2), (65, 33, 2)], ids=str)
def test_tiny_and_ragged_frames(dev, size):
    W, H, T = size
    vol = synth.video(max(W, 8), max(H, 8), T, seed=73)[:, :H, :W].copy()
    for spec in CHAINS.values():
        ref, _ = run(spec, vol, dev)
        g, _ = run(spec, vol, dev, engine="jit")
        assert np.array_equal(g, ref), size


def test_unaligned_input_pointer(dev):
    """An input tensor whose data starts one byte past an aligned address
    (a view into a larger buffer): the four-cell loads are not used for it,
    and the output equals that of an aligned copy."""
    spec = CHAINS["well"]
    vol = synth.video(208, 64, 3, seed=76)
    ref, _ = run(spec, vol, dev)
    T, H, W = vol.shape
    big = torch.zeros(T * H * W + 16, dtype=torch.uint8, device=dev)
    x = big[1:1 + T * H * W].view(T, H, W)
    x.copy_(torch.from_numpy(vol).to(dev))
    assert x.data_ptr() % 4 == 1
    plan = fz.Plan(spec, W, H, T, engine="jit")
    out, _, _ = plan.run(x)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy()[0], ref)


def test_large_box_and_batch(dev):
    """A group whose LDS box exceeds 64 KB (static LDS of the generated
    kernel), and a batch of clips of different sizes through a JIT plan
    (modules loaded before the graph capture) equal to single runs."""
    spec = [("stencil", 3, 3, np.full((7, 7), 1.0 / 49.0, np.float32)), ("box", 3, 3), ("box", 3, 3),
            ("stencil", 3, 3, np.full((7, 7), 1.0 / 49.0, np.float32))]
    vol = synth.video(300, 200, 2, seed=74)
    ref, _ = run(spec, vol, dev, partition=[])
    g, plan = run(spec, vol, dev, partition=[], engine="jit")
    say("large box lds", plan.segment_info()[0].lds_bytes)
    assert np.array_equal(g, ref)
    sizes = [(192, 432, 3), (320, 240, 4), (97, 61, 5)]
    bplan = fz.Plan(CHAINS["well"], 800, 600, 8, engine="jit")
    xs, outs, clips = [], [], []
    for i, (W, H, T) in enumerate(sizes):
        v = synth.video(W, H, T, seed=80 + i)
        x = torch.from_numpy(v).to(dev)
        o = torch.empty((1, T, H, W), dtype=torch.float32, device=dev)
        xs.append((v, x))
        outs.append(o)
        clips.append(fz.make_clip(x, o, plan=bplan))
    ws = torch.empty((max(fz.fz_batch_workspace_bytes(bplan.handle, clips), 1),), dtype=torch.uint8, device=dev)
    for rep in range(3):
        fz.fz_run_batch(bplan.handle, clips, ws.data_ptr(), ws.numel(), torch.cuda.current_stream(dev).cuda_stream)
        torch.cuda.synchronize()
        for (v, _), o in zip(xs, outs):
            ref, _ = run(CHAINS["well"], v, dev)
            assert np.array_equal(o.cpu().numpy()[0], ref), rep


def test_generated_marching_kernels_equal_interpreted(dev):
    """Groups with temporal stages (an IIR, stencils over several frames, an
    IIR after a window stage) as generated frame-marching kernels: the same
    bits as the interpreted marching kernel, for checkpointed and whole-clip
    IIR groups and several frame runs, and within the oracle's bound."""
    from tests.test_gpu_temporal import MIXED, PAPER5, SPATIO
    for width in (133, 136):
        marching_case(dev, MIXED, PAPER5, SPATIO, synth.video(width, 77, 17, seed=75))


def marching_case(dev, MIXED, PAPER5, SPATIO, vol):
    for name, spec in (("paper5", PAPER5), ("spatio", SPATIO), ("mixed", MIXED)):
        ref, _ = run(spec, vol, dev, partition=[])
        g, plan = run(spec, vol, dev, partition=[], engine="jit")
        (s,) = plan.segment_info()
        say("marching", name, s.engine, s.tile_w, s.tile_h, s.frames_per_block)
        assert s.engine == fz.FZ_ENGINE_JIT
        assert np.array_equal(g, ref), name
        if name != "mixed":  # runs shorter than the clip (checkpointed IIR, look-back rings)
            T, H, W = vol.shape
            for tpb in (1, 4, 16):
                plan = fz.Plan(spec, W, H, T, partition=[])
                plan.set_segment_config(0, engine="jit", tile=(32, 16), frames_per_block=tpb)
                out, _, _ = plan.run(torch.from_numpy(vol).to(dev))
                torch.cuda.synchronize()
                assert np.array_equal(out.cpu().numpy()[0], ref), (name, tpb)
        ref_o, bound = parity.generic_reference(oracle, spec, vol)
        parity.assert_within_bound(g, ref_o, bound, f"jit marching {name}")
