"""fz_run_chain_static (the entry point that allocates nothing, for callers
that cannot call hipMalloc) against fz_run_chain on the same plans and inputs.

Two calls in a row share the library's static workspace; the second uses a
smaller video, so stale contents of the first call must not leak into it."""
import numpy as np
import pytest
import torch

from paper_1509_04394_amd import fz, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def say(*a):
    print("[no-alloc]", *a, flush=True)


def run_both(ops, vol, partition, dev, **kw):
    W, H, T = vol.shape[2], vol.shape[1], vol.shape[0]
    plan = fz.Plan(ops, W, H, T, partition=partition, **kw)
    assert 0 < plan.workspace_bytes <= fz.FZ_STATIC_WORKSPACE_BYTES
    x = torch.from_numpy(vol).to(dev)
    ref, rp, rc = plan.run(x)
    cap = 1 << 16
    pts = torch.zeros((cap, 4), dtype=torch.int32, device=dev)
    cnt = torch.zeros((1,), dtype=torch.int32, device=dev)
    out, pts, cnt = plan.run_static(x, points=pts if plan.has_points() else None,
                                    count=cnt if plan.has_points() else None)
    torch.cuda.synchronize()
    assert torch.equal(out, ref), "static-workspace output differs from fz_run_chain"
    if plan.has_points():
        key = lambda p, c: sorted(map(tuple, p[:int(c.item())].cpu().numpy().tolist()))
        assert int(cnt.item()) == int(rc.item())
        assert key(pts, cnt) == key(rp, rc)
    return plan


def test_static_workspace_matches_caller_workspace_two_calls(dev):
    ops = fz.RGB_HARRIS_CHAIN
    big = synth.video(160, 96, 6, seed=41, rgb=True)
    small = synth.video(100, 64, 4, seed=42, rgb=True)
    say("unfused 160x96x6 then 100x64x4")
    p1 = run_both(ops, big, "unfused", dev)
    p2 = run_both(ops, small, "unfused", dev)
    assert p2.workspace_bytes < p1.workspace_bytes
    # a partial fusion (three groups: both slots in use), again big then small
    say("cuts [1, 4] 160x96x6 then 100x64x4")
    run_both(ops, big, [1, 4], dev)
    run_both(ops, small, [1, 4], dev)


def test_static_workspace_generic_chain(dev):
    w3 = np.full((3, 3), 1.0 / 9.0, np.float32)
    spec = [("stencil", 1, 1, w3), ("point", "abs", 0.0, 0.0), ("box", 2, 1), ("point", "sqrtabs", 0.0, 0.0)]
    for W, H, T in [(200, 120, 5), (90, 70, 3)]:
        say("generic unfused", W, H, T)
        run_both(spec, synth.video(W, H, T, seed=43), "unfused", dev)


def test_static_workspace_fused_row_exchange(dev):
    """The fused Harris chain on the row kernel with 2-frame runs: its work
    items meet at run boundaries through the exchange words and counters in
    the workspace (here the library's static array), big clip then small."""
    for W, H, T, band in [(300, 40, 23, 13), (200, 24, 9, 8)]:
        say("fused row exchange", W, H, T)
        plan = run_both(fz.RGB_HARRIS_CHAIN, synth.video(W, H, T, seed=44 + W, rgb=True), [], dev,
                        engine="row", band_h=band, frames_per_block=2)
        assert plan.segment_info()[0].engine == fz.FZ_ENGINE_ROW


def test_static_workspace_refuses_oversized_plans(dev):
    plan = fz.Plan(fz.RGB_HARRIS_CHAIN, 800, 600, 40, partition="unfused")
    assert plan.workspace_bytes > fz.FZ_STATIC_WORKSPACE_BYTES
    x = torch.zeros(plan.input_shape(), dtype=torch.uint8, device=dev)
    with pytest.raises(fz.FzError) as e:
        plan.run_static(x)
    assert e.value.code == fz.FZ_E_WORKSPACE
