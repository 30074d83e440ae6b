"""Batched runs: many clips of uneven size and length in one persistent
launch captured into a HIP graph.  Every clip's output and point set must equal
those of a single-clip run bit for bit, and match the FP64 oracle (all frames
of short clips; sampled frames, each with the frame before it, of long ones)."""
import numpy as np
import pytest

import oracle
from paper_1509_04394_amd import fz, synth
from tests import parity

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def say(*a):
    print("[gpu-batch]", *a, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


SIZES = [(192, 432, 7), (320, 240, 20), (640, 480, 3), (800, 600, 17), (192, 432, 1), (320, 240, 33)]
key = lambda p: sorted(map(tuple, p.tolist()))


def make_clips(ops, sizes, dev, rgb, seed0=4000, cap=1 << 16):
    items = []
    for i, (W, H, T) in enumerate(sizes):
        v = synth.video(W, H, T, seed=seed0 + i, rgb=rgb)
        x = torch.from_numpy(v).to(dev)
        plan = fz.Plan(ops, W, H, T)
        out, pts, cnt, ws = plan.alloc(dev, point_capacity=cap)
        items.append(dict(x=x, out=out, pts=pts, cnt=cnt, plan=plan, ws=ws, seed=seed0 + i, size=(W, H, T), rgb=rgb))
    return items


def single_runs(items):
    refs = []
    for it in items:
        o, p, c = it["plan"].run(it["x"], torch.empty_like(it["out"]), torch.empty_like(it["pts"]),
                                 torch.empty_like(it["cnt"]), it["ws"])
        torch.cuda.synchronize()
        refs.append((o.cpu().numpy(), fz.points_to_numpy(p, c)))
    return refs


def check(items, refs):
    """Batch results == single-clip runs, bit for bit."""
    for i, (it, (ro, rp)) in enumerate(zip(items, refs)):
        assert np.array_equal(it["out"].cpu().numpy(), ro), f"clip {i} output"
        assert key(fz.points_to_numpy(it["pts"], it["cnt"])) == key(rp), f"clip {i} points"


def check_oracle(ops, items, all_frames_upto=200, samples=3):
    """Batch results against the oracle: every frame of clips up to
    `all_frames_upto` frames, else `samples` frames spread over the clip, each
    with the frame before it (the frame difference's temporal halo)."""
    total = {}
    for i, it in enumerate(items):
        W, H, T = it["size"]
        g = it["out"].cpu().numpy()
        gp = fz.points_to_numpy(it["pts"], it["cnt"])
        if T <= all_frames_upto:
            ranges = [(0, T, 0)]
        else:
            ts = sorted({int(round(q)) for q in np.linspace(0, T - 1, samples)})
            ranges = [(max(t - 1, 0), t + 1, t - max(t - 1, 0)) for t in ts]
        for s, e, skip in ranges:
            vol = synth.video(W, H, e - s, seed=it["seed"], rgb=it["rgb"], t0=s)
            sel = (gp[:, 0] >= s) & (gp[:, 0] < e)
            gps = gp[sel].copy()
            gps[:, 0] -= s
            st = parity.check_chain(oracle, ops, vol, g[s:e], gps, skip=skip)
            parity.add_stats(total, st)
    say("oracle", total)
    assert total["px_differ"] == 0 and total["points_differ"] == 0, total
    return total


@pytest.mark.parametrize("rgb", [False, True])
def test_batch_equals_single_clip_runs(dev, rgb):
    ops = fz.RGB_HARRIS_CHAIN if rgb else fz.HARRIS_CHAIN
    items = make_clips(ops, SIZES, dev, rgb)
    refs = single_runs(items)
    plan = fz.Plan(ops, 800, 600, 100)
    assert len(plan.segments) == 1
    clips = [fz.make_clip(it["x"], it["out"], it["pts"], it["cnt"], plan=plan) for it in items]
    ws = None
    for rep in range(3):  # first call captures the graph, later calls replay it
        for it in items:
            it["out"].fill_(7)
            it["cnt"].fill_(12345)
        torch.cuda.synchronize()
        ws = fz.run_batch(plan, clips, ws)
        torch.cuda.synchronize()
        say("rgb" if rgb else "gray", "replay", rep)
        check(items, refs)
    st = check_oracle(ops, items)
    assert st["points_oracle"] > 0
    # a different output buffer for one clip: re-captured, still exact
    items[2]["out"] = torch.empty_like(items[2]["out"])
    clips[2] = fz.make_clip(items[2]["x"], items[2]["out"], items[2]["pts"], items[2]["cnt"], plan=plan)
    ws = fz.run_batch(plan, clips, ws)
    torch.cuda.synchronize()
    check(items, refs)


def test_batch_more_clips_than_one_launch(dev):
    ops = fz.HARRIS_CHAIN
    sizes = [(128 + 8 * (i % 5), 16 + i % 7, 2 + i % 4) for i in range(37)]
    items = make_clips(ops, sizes, dev, False, seed0=500)
    refs = single_runs(items)
    plan = fz.Plan(ops, 128, 16, 4)
    clips = [fz.make_clip(it["x"], it["out"], it["pts"], it["cnt"], plan=plan) for it in items]
    fz.run_batch(plan, clips)
    torch.cuda.synchronize()
    check(items, refs)
    check_oracle(ops, items)


def test_batch_clip_by_clip_with_run_exchange(dev):
    """A fused plan with one clip too narrow for the row kernel runs clip by
    clip inside the graph: the wide clips' fused row groups meet at their
    frame-run boundaries through the exchange words in the batch workspace,
    whose counters a kernel node clears on every replay."""
    ops = fz.HARRIS_CHAIN
    sizes = [(200, 48, 9), (96, 40, 5), (160, 33, 12)]
    items = make_clips(ops, sizes, dev, False, seed0=950)
    refs = single_runs(items)
    plan = fz.Plan(ops, 200, 48, 9)
    assert len(plan.segments) == 1
    clips = [fz.make_clip(it["x"], it["out"], it["pts"], it["cnt"], plan=plan) for it in items]
    ws = None
    for rep in range(3):
        for it in items:
            it["out"].fill_(7)
            it["cnt"].fill_(12345)
        torch.cuda.synchronize()
        ws = fz.run_batch(plan, clips, ws)
        torch.cuda.synchronize()
        say("clip by clip, exchange, replay", rep)
        check(items, refs)


@pytest.mark.parametrize("partition", ["unfused", [3]])
def test_batch_clip_by_clip_path(dev, partition):
    """Plans the persistent kernel does not cover run clip after clip in the graph."""
    ops = fz.HARRIS_CHAIN
    items = make_clips(ops, SIZES[:4], dev, False, seed0=900)
    refs = single_runs(items)
    plan = fz.Plan(ops, 320, 240, 20, partition=partition)
    clips = [fz.make_clip(it["x"], it["out"], it["pts"], it["cnt"], plan=plan) for it in items]
    ws = fz.run_batch(plan, clips)
    torch.cuda.synchronize()
    check(items, refs)
    fz.run_batch(plan, clips, ws)  # replay
    torch.cuda.synchronize()
    check(items, refs)
    check_oracle(ops, items)


def test_batch_workload_32_clips(dev):
    """The 32-clip batch of the benchmark: frame sizes drawn from 192x432,
    320x240, 640x480, 800x600, 50-1000 frames each (about 4 Gpx of gray
    video), one persistent launch replayed from a graph.  Every clip equals its
    single-clip run over all frames; three frames per clip (first, middle,
    last, each with its predecessor) are checked against the oracle."""
    ops = fz.HARRIS_CHAIN
    shapes = synth.batch_shapes(4, 32)
    say("32 clips", sum(W * H * T for W, H, T in shapes) / 1e9, "Gpx")
    items = make_clips(ops, shapes, dev, False, seed0=4000, cap=1 << 18)
    refs = single_runs(items)
    plan = fz.Plan(ops, 800, 600, 1000)
    clips = [fz.make_clip(it["x"], it["out"], it["pts"], it["cnt"], plan=plan) for it in items]
    ws = None
    for rep in range(2):
        for it in items:
            it["out"].fill_(3)
        torch.cuda.synchronize()
        ws = fz.run_batch(plan, clips, ws)
        torch.cuda.synchronize()
        check(items, refs)
        say("replay", rep, "equals single-clip runs")
    del refs
    st = check_oracle(ops, items, all_frames_upto=0)
    assert st["points_oracle"] > 0
