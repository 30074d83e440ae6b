"""Batched runs: many clips of uneven size and length in one persistent
launch captured into a HIP graph.  Every clip's output and point set must equal
those of a single-clip run bit for bit."""
import numpy as np
import pytest

from paper_1509_04394_amd import fz, synth

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


def make_clips(ops, sizes, dev, rgb, seed0=4000):
    items = []
    for i, (W, H, T) in enumerate(sizes):
        v = synth.video(W, H, T, seed=seed0 + i, rgb=rgb)
        x = torch.from_numpy(v).to(dev)
        plan = fz.Plan(ops, W, H, T)
        out, pts, cnt, ws = plan.alloc(dev, point_capacity=1 << 16)
        items.append(dict(x=x, out=out, pts=pts, cnt=cnt, plan=plan, ws=ws))
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
    for i, (it, (ro, rp)) in enumerate(zip(items, refs)):
        assert np.array_equal(it["out"].cpu().numpy(), ro), f"clip {i} output"
        assert key(fz.points_to_numpy(it["pts"], it["cnt"])) == key(rp), f"clip {i} points"


@pytest.mark.parametrize("rgb", [False, True])
def test_batch_equals_single_clip_runs(dev, rgb):
    ops = fz.RGB_HARRIS_CHAIN if rgb else fz.HARRIS_CHAIN
    items = make_clips(ops, SIZES, dev, rgb)
    refs = single_runs(items)
    plan = fz.Plan(ops, 800, 600, 100)
    assert len(plan.segments) == 1
    clips = [fz.make_clip(it["x"], it["out"], it["pts"], it["cnt"]) for it in items]
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
    # a different output buffer for one clip: re-captured, still exact
    items[2]["out"] = torch.empty_like(items[2]["out"])
    clips[2] = fz.make_clip(items[2]["x"], items[2]["out"], items[2]["pts"], items[2]["cnt"])
    ws = fz.run_batch(plan, clips, ws)
    torch.cuda.synchronize()
    check(items, refs)


def test_batch_more_clips_than_one_launch(dev):
    ops = fz.HARRIS_CHAIN
    sizes = [(128 + 8 * (i % 5), 16 + i % 7, 2 + i % 4) for i in range(37)]
    items = make_clips(ops, sizes, dev, False, seed0=500)
    refs = single_runs(items)
    plan = fz.Plan(ops, 128, 16, 4)
    clips = [fz.make_clip(it["x"], it["out"], it["pts"], it["cnt"]) for it in items]
    fz.run_batch(plan, clips)
    torch.cuda.synchronize()
    check(items, refs)


@pytest.mark.parametrize("partition", ["unfused", [3]])
def test_batch_clip_by_clip_path(dev, partition):
    """Plans the persistent kernel does not cover run clip after clip in the graph."""
    ops = fz.HARRIS_CHAIN
    items = make_clips(ops, SIZES[:4], dev, False, seed0=900)
    refs = single_runs(items)
    plan = fz.Plan(ops, 320, 240, 20, partition=partition)
    clips = [fz.make_clip(it["x"], it["out"], it["pts"], it["cnt"]) for it in items]
    ws = fz.run_batch(plan, clips)
    torch.cuda.synchronize()
    check(items, refs)
    fz.run_batch(plan, clips, ws)  # replay
    torch.cuda.synchronize()
    check(items, refs)
