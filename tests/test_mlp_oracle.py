"""Pins for the MLP reference (no GPU): bfloat16 rounding against torch's
conversion, forward and gradients against torch autograd in float64, the
analytic gradient against central finite differences, and Adam against
torch.optim.Adam."""
import numpy as np
import pytest

from oracle import mlp_ref as M

torch = pytest.importorskip("torch")


def test_param_count():
    assert M.NPARAM == 4481


def test_bf16_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-8, 8, 20000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, 1.0 + 2 ** -9, np.inf, -np.inf, 65504.0,
                         3.0e38, 1e-40]]).astype(np.float32)
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    got = M.bf16(x)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    # ties go to even: 1 + 2^-8 is halfway between 1 and 1 + 2^-7
    assert M.bf16(np.float32(1 + 2 ** -8)) == 1.0
    assert M.bf16(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def _torch_model(theta, x, emulate):
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in M.unpack(theta).items()}
    rb = (lambda v: v.to(torch.float32).to(torch.bfloat16).to(torch.float64)) if emulate else (lambda v: v)
    xt = torch.tensor(x, dtype=torch.float64)
    a1 = xt @ rb(p["W1"]).T + p["b1"]
    h1 = rb(torch.relu(a1))
    a2 = h1 @ rb(p["W2"]).T + p["b2"]
    h2 = rb(torch.relu(a2))
    y = h2 @ rb(p["w3"]) + p["b3"]
    return y, p


def test_forward_matches_torch_float64():
    rng = np.random.default_rng(1)
    theta = M.he_init(3)
    x = rng.random((100, 3))
    y, _ = M.forward(theta, x, emulate=False)
    yt, _ = _torch_model(theta, x, emulate=False)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_forward_emulated_matches_torch_casts():
    rng = np.random.default_rng(2)
    theta = M.he_init(4)
    x = M.bf16(rng.random((100, 3)))
    y, _ = M.forward(theta, x, emulate=True)
    yt, _ = _torch_model(theta, x, emulate=True)
    np.testing.assert_allclose(y, yt.detach().numpy(), rtol=1e-12, atol=1e-12)


def test_gradient_matches_torch_autograd():
    rng = np.random.default_rng(5)
    theta = M.he_init(6)
    x = rng.random((64, 3))
    t = rng.standard_normal(64) - 4.0
    L, g = M.backward(theta, x, t, emulate=False)
    yt, p = _torch_model(theta, x, emulate=False)
    lt = torch.mean((yt - torch.tensor(t)) ** 2)
    lt.backward()
    gt = M.pack({k: v.grad.numpy() for k, v in p.items()})
    assert abs(L - lt.item()) < 1e-12
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-13)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(7)
    theta = M.he_init(8) + 0.05 * rng.standard_normal(M.NPARAM)
    x = rng.random((32, 3))
    t = rng.standard_normal(32) - 3.0
    _, g = M.backward(theta, x, t, emulate=False)
    idx = rng.choice(M.NPARAM, 300, replace=False)
    idx = np.concatenate([idx, [M.NPARAM - 1, 0, 192]])
    h = 1e-6
    for i in idx:
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        fd = (M.loss(tp, x, t, emulate=False) - M.loss(tm, x, t, emulate=False)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-9, (i, fd, g[i])


def test_adam_matches_torch():
    rng = np.random.default_rng(9)
    theta = rng.standard_normal(50)
    m = np.zeros(50)
    v = np.zeros(50)
    w = torch.tensor(theta.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([w], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for step in range(1, 6):
        g = rng.standard_normal(50)
        theta, m, v = M.adam_step(theta, m, v, g, step)
        w.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(theta, w.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_worst0_rule():
    theta = M.he_init(1)
    q = np.array([[0.5, 0.5, 0.5]], np.float32)
    lo = np.zeros(3, np.float32)
    inv = np.ones(3, np.float32)
    w_inf = M.predict_worst0(theta, q, lo, inv, 0.0, np.float32(np.inf))
    w_small = M.predict_worst0(theta, q, lo, inv, 0.0, np.float32(1e-30))
    assert np.isfinite(w_inf).all() and w_small[0] == np.float32(1e-30)
    # huge margin overflows r0^2 to inf -> min(R2, inf) = R2
    w_big = M.predict_worst0(theta, q, lo, inv, 200.0, np.float32(2.0))
    assert w_big[0] == np.float32(2.0)
