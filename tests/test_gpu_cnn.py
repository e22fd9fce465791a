"""Warm-start network kernels against the CPU FP64 oracle (through the C-ABI)."""
import numpy as np
import pytest

from oracle import cnn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2206_11009_amd as otip
    c = otip.Context(0)
    yield c
    c.close()


def params(seed, noise=0.02):
    rng = np.random.default_rng(seed)
    th = cnn.init_params(seed) + noise * rng.standard_normal(cnn.param_count())
    return th


def test_param_count_matches_oracle():
    import paper_2206_11009_amd as otip
    assert otip.otip_ws_param_count() == cnn.param_count()


@pytest.mark.parametrize("N,H,W", [(3, 32, 32), (2, 13, 9), (1, 40, 33)])
def test_forward_matches_oracle(ctx, N, H, W):
    import torch
    import paper_2206_11009_amd as otip
    th = params(N + H)
    rng = np.random.default_rng(H)
    x = rng.uniform(0, 3, (N, 2, H, W))
    wt = torch.as_tensor(th, dtype=torch.float32, device="cuda:0")
    out = otip.otip_ws_forward(ctx, wt, torch.as_tensor(x, dtype=torch.float32, device="cuda:0"))
    # the oracle sees the same FP32-rounded weights and inputs
    ref = cnn.forward(th.astype(np.float32).astype(np.float64),
                      x.astype(np.float32).astype(np.float64))[-1]
    err = np.abs(out.cpu().numpy() - ref).max()
    assert err <= 1e-5 * max(1.0, np.abs(ref).max()), err


@pytest.mark.parametrize("N,H,W", [(4, 16, 16), (2, 32, 32), (3, 11, 17)])
def test_gradient_matches_oracle(ctx, N, H, W):
    import torch
    import paper_2206_11009_amd as otip
    th = params(7 + N).astype(np.float32).astype(np.float64)
    rng = np.random.default_rng(N * H)
    x = rng.uniform(0, 3, (N, 2, H, W)).astype(np.float32).astype(np.float64)
    t = rng.standard_normal((N, 2, H, W)).astype(np.float32).astype(np.float64)
    f32 = lambda a: torch.as_tensor(a, dtype=torch.float32, device="cuda:0")
    loss, g = otip.otip_ws_grad(ctx, f32(th), f32(x), f32(t))
    rloss, rg = cnn.grad(th, x, t)
    assert loss == pytest.approx(rloss, rel=1e-5)
    g = g.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(g - rg) <= 1e-4 * np.linalg.norm(rg)
    # per layer, so that a small layer's error is not hidden by a large one
    off = 0
    for ci, co, _, _ in cnn.LAYERS:
        sl = slice(off, off + co * ci * 9 + co)
        assert np.linalg.norm(g[sl] - rg[sl]) <= 1e-4 * np.linalg.norm(rg[sl]) + 1e-12
        off = sl.stop


def test_adam_matches_oracle(ctx):
    import torch
    import paper_2206_11009_amd as otip
    rng = np.random.default_rng(2)
    P = cnn.param_count()
    th = rng.standard_normal(P).astype(np.float32)
    m = np.zeros(P, np.float32)
    v = np.zeros(P, np.float32)
    d = lambda a: torch.as_tensor(a, device="cuda:0")
    wt, mt, vt = d(th.copy()), d(m.copy()), d(v.copy())
    ref = (th.astype(np.float64), m.astype(np.float64), v.astype(np.float64))
    for step in range(1, 4):
        g = rng.standard_normal(P).astype(np.float32)
        otip.otip_ws_adam(ctx, wt, mt, vt, d(g), step, 1e-2)
        ref = cnn.adam(*ref, g.astype(np.float64), step, 1e-2)
    np.testing.assert_allclose(wt.cpu().numpy(), ref[0], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(vt.cpu().numpy(), ref[2], rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("side", [8, 20, 32, 64, 256])
def test_predict_matches_oracle(ctx, side):
    import torch
    import paper_2206_11009_amd as otip
    from synthetic import gaussian_mixture
    th = params(side).astype(np.float32).astype(np.float64)
    a = gaussian_mixture(side, 3, 11 + side)
    b = gaussian_mixture(side, 2, 12 + side)
    y0, z0 = otip.otip_ws_predict(ctx, torch.as_tensor(th, dtype=torch.float32, device="cuda:0"),
                                  side, a, b)
    ry, rz = cnn.predict_duals(th, a, b, side)
    scale = max(np.abs(ry).max(), np.abs(rz).max())
    assert np.abs(y0.cpu().numpy() - ry).max() <= 1e-5 * scale
    assert np.abs(z0.cpu().numpy() - rz).max() <= 1e-5 * scale
