"""The cost network's HIP kernels against the FP64 oracle (oracle/mlp.py)."""
import numpy as np
import pytest

from oracle import mlp
from paper_1509_04394_amd import fz

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

F = 18


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def t32(a, dev):
    return torch.tensor(np.asarray(a, np.float32), device=dev)


def data(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(n, F)).astype(np.float32)
    t = (np.sin(x[:, 0]) + 0.5 * x[:, 1] * x[:, 2] - 0.3 * np.abs(x[:, 3])).astype(np.float32)
    return x, t


@pytest.mark.parametrize("n", [1, 63, 300, 4096])
def test_forward_matches_oracle(dev, n):
    p = mlp.init(F, seed=n).astype(np.float32)
    x, _ = data(n, n)
    y = torch.empty(n, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    dp, dx = t32(p, dev), t32(x, dev)  # keep the buffers alive until the kernel has run
    fz.fz_mlp_forward(dp.data_ptr(), F, dx.data_ptr(), n, y.data_ptr(), s)
    torch.cuda.synchronize()
    ref = mlp.forward(p.astype(np.float64), x.astype(np.float64), F)
    got = y.cpu().numpy().astype(np.float64)
    assert np.max(np.abs(got - ref)) <= 1e-5 * (1 + np.max(np.abs(ref)))


@pytest.mark.parametrize("n", [5, 200, 2048])
def test_loss_and_gradient_match_oracle(dev, n):
    p = mlp.init(F, seed=7 + n).astype(np.float32)
    x, t = data(n, 100 + n)
    P = fz.fz_mlp_param_count(F)
    assert P == mlp.n_params(F)
    g = torch.empty(P, device=dev)
    L = torch.empty(1, device=dev)
    ws = torch.empty(fz.fz_mlp_workspace_bytes(F, n), dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    dp, dx, dt = t32(p, dev), t32(x, dev), t32(t, dev)
    fz.fz_mlp_loss_grad(dp.data_ptr(), F, dx.data_ptr(), dt.data_ptr(), n, g.data_ptr(), L.data_ptr(),
                        ws.data_ptr(), ws.numel(), s)
    Lr, gr = mlp.loss_grad(p.astype(np.float64), x.astype(np.float64), t.astype(np.float64), F)
    gg = g.cpu().numpy().astype(np.float64)
    assert abs(L.item() - Lr) <= 1e-5 * max(1.0, Lr)
    rel = np.linalg.norm(gg - gr) / np.linalg.norm(gr)
    assert rel <= 1e-4, rel
    assert np.max(np.abs(gg - gr)) <= 1e-4 * np.max(np.abs(gr))
    # deterministic: the same call twice gives the same bits
    g2 = torch.empty_like(g)
    fz.fz_mlp_loss_grad(dp.data_ptr(), F, dx.data_ptr(), dt.data_ptr(), n, g2.data_ptr(), L.data_ptr(),
                        ws.data_ptr(), ws.numel(), s)
    assert torch.equal(g, g2)


def test_adam_step_matches_oracle(dev):
    P = fz.fz_mlp_param_count(F)
    rng = np.random.default_rng(3)
    p = rng.normal(size=P).astype(np.float32)
    m = rng.normal(size=P).astype(np.float32) * 0.01
    v = np.abs(rng.normal(size=P)).astype(np.float32) * 0.001
    g = rng.normal(size=P).astype(np.float32)
    dp, dg, dm, dv = t32(p, dev), t32(g, dev), t32(m, dev), t32(v, dev)
    fz.fz_mlp_adam_step(dp.data_ptr(), dg.data_ptr(), dm.data_ptr(), dv.data_ptr(), P, 4, 1e-3, 0.9, 0.999, 1e-8,
                        torch.cuda.current_stream().cuda_stream)
    rp, rm, rv = mlp.adam(p.astype(np.float64), g.astype(np.float64), m.astype(np.float64), v.astype(np.float64),
                          4, 1e-3)
    np.testing.assert_allclose(dp.cpu().numpy(), rp, rtol=0, atol=2e-6)
    # FP32 holds 1 - 0.9 and 1 - 0.999 with relative errors up to 4.7e-5, so the
    # moment updates agree with the FP64 definition to about 1e-4 relative
    np.testing.assert_allclose(dm.cpu().numpy(), rm, rtol=1e-4, atol=1e-8)
    np.testing.assert_allclose(dv.cpu().numpy(), rv, rtol=1e-4, atol=1e-10)


def test_training_on_gpu_follows_oracle_and_learns(dev):
    n = 1024
    x, t = data(n, 11)
    p0 = mlp.init(F, seed=5)
    P = p0.size
    dp = t32(p0, dev)
    dx, dt = t32(x, dev), t32(t, dev)
    g = torch.empty(P, device=dev)
    L = torch.empty(1, device=dev)
    m = torch.zeros(P, device=dev)
    v = torch.zeros(P, device=dev)
    ws = torch.empty(fz.fz_mlp_workspace_bytes(F, n), dtype=torch.uint8, device=dev)
    s = torch.cuda.current_stream().cuda_stream
    rp, rm, rv = p0.astype(np.float64), np.zeros(P), np.zeros(P)
    losses = []
    for step in range(1, 301):
        fz.fz_mlp_loss_grad(dp.data_ptr(), F, dx.data_ptr(), dt.data_ptr(), n, g.data_ptr(), L.data_ptr(),
                            ws.data_ptr(), ws.numel(), s)
        fz.fz_mlp_adam_step(dp.data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), P, step, 3e-3, 0.9, 0.999,
                            1e-8, s)
        if step <= 3:  # the first steps track the FP64 trajectory closely
            Lr, gr = mlp.loss_grad(rp, x.astype(np.float64), t.astype(np.float64), F)
            rp, rm, rv = mlp.adam(rp, gr, rm, rv, step, 3e-3)
            assert abs(L.item() - Lr) <= 1e-4 * max(1.0, Lr)
            assert np.max(np.abs(dp.cpu().numpy() - rp)) <= 1e-4
        losses.append(L.item())
    assert losses[-1] < 0.2 * losses[0], (losses[0], losses[-1])
