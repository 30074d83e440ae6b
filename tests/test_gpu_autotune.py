"""The autotuner on the device: the configuration it keeps is no slower than
the planner's (it only replaces it when measured faster), and the output does
not change (every configuration gives the same bits)."""
import numpy as np
import pytest

from paper_1509_04394_amd import autotune, fz, synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.mark.parametrize("ops,W,H,T,rgb", [(fz.RGB_HARRIS_CHAIN, 800, 600, 48, True),
                                           (fz.HARRIS_CHAIN, 192, 432, 64, False)], ids=["rgb800", "harris192"])
def test_autotuned_plan_is_not_slower_and_same_bits(dev, ops, W, H, T, rgb):
    x = torch.from_numpy(synth.video(W, H, T, seed=91, rgb=rgb)).to(dev)
    plan = fz.Plan(ops, W, H, T)
    ref, rp, rc = plan.run(x)
    torch.cuda.synchronize()
    ref = ref.cpu().numpy()
    key = lambda p, c: sorted(map(tuple, p[:int(c.item())].cpu().numpy()[:, :3].tolist()))
    ref_pts = key(rp, rc)
    before = autotune._time(fz.Plan(ops, W, H, T), x, 7)
    report = autotune.autotune(plan, x, reps=5)
    after = autotune._time(plan, x, 7)
    print(f"[gpu-autotune] {W}x{H}x{T}: planner {before:.3f} ms, autotuned {after:.3f} ms, {report}", flush=True)
    for (_, cfg, best_ms, default_ms) in report:
        assert best_ms <= default_ms
    assert after <= before * 1.08  # timing noise between the two measurements
    out, p, c = plan.run(x)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref)
    assert key(p, c) == ref_pts
