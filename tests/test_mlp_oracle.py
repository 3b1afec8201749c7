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


class _RoundST(torch.autograd.Function):
    """bfloat16 rounding (through float32) in the forward pass, gradient
    passed straight through."""

    @staticmethod
    def forward(ctx, v):
        return v.to(torch.float32).to(torch.bfloat16).to(torch.float64)

    @staticmethod
    def backward(ctx, g):
        return g


class _GradRound(torch.autograd.Function):
    """Identity in the forward pass; the gradient flowing back through it is
    rounded to bfloat16 (through float32)."""

    @staticmethod
    def forward(ctx, v):
        return v.clone()

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.float32).to(torch.bfloat16).to(torch.float64)


def test_emulated_backward_matches_torch_straight_through():
    """backward(emulate=True): bfloat16 weights and activations with
    straight-through gradients, and the layer-2 output gradient rounded to
    bfloat16 before both products it feeds (the weight gradient of W2 and the
    input gradient of layer 2) but not before the bias gradient."""
    rng = np.random.default_rng(13)
    theta = M.he_init(14) + 0.05 * rng.standard_normal(M.NPARAM)
    x = M.bf16(rng.random((96, 3)))
    t = rng.standard_normal(96) * 0.3 - 4.0
    L, g = M.backward(theta, x, t, emulate=True)
    p = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in M.unpack(theta).items()}
    xt = torch.tensor(x, dtype=torch.float64)
    a1 = xt @ _RoundST.apply(p["W1"]).T + p["b1"]
    h1 = _RoundST.apply(torch.relu(a1))
    a2 = _GradRound.apply(h1 @ _RoundST.apply(p["W2"]).T) + p["b2"]
    h2 = _RoundST.apply(torch.relu(a2))
    y = h2 @ _RoundST.apply(p["w3"]) + p["b3"]
    lt = torch.mean((y - torch.tensor(t)) ** 2)
    lt.backward()
    gt = M.pack({k: v.grad.numpy() for k, v in p.items()})
    assert abs(L - lt.item()) < 1e-12
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-13)
    # the rounding point matters: without it the W2 gradient differs
    _, g_plain = M.backward(theta, x, t, emulate=False)
    assert not np.allclose(g[256:4352], g_plain[256:4352], rtol=1e-6, atol=0)


def _mlp_case(seed, n):
    rng = np.random.default_rng(seed)
    theta = M.fp32(M.he_init(seed + 1) + 0.05 * rng.standard_normal(M.NPARAM))
    x = M.normalize(rng.random((n, 3), dtype=np.float32), np.zeros(3, np.float32), np.ones(3, np.float32))
    t = M.fp32(rng.standard_normal(n) * 0.3 - 4.0)
    return theta, x, t


def test_forward_enclosure_accepts_float32_and_rejects_planted_error():
    from tests import mlp_bounds as MB
    theta, x, _ = _mlp_case(21, 4000)
    ok, e = MB.check_forward(theta, x, MB.float32_forward(theta, x))
    assert ok.all(), np.flatnonzero(~ok)[:10]
    yc, yr = e["y"]
    # tight where no rounding can flip: the plain accumulation bound
    # (about 1 % of activations can round either way, so most queries have
    # some interval widened by a possible flip)
    rel = yr / (1 + np.abs(yc))
    tight = ~e["flips"]
    assert tight.any() and np.max(rel[tight]) < 1e-4
    assert np.median(rel) < 1e-4
    ok_bad, _ = MB.check_forward(theta, x, MB.float32_forward(theta, x, W2_scale=1.01))
    assert ok_bad.mean() < 0.05


def test_gradient_enclosure_accepts_float32_and_rejects_planted_error():
    from tests import mlp_bounds as MB
    theta, x, t = _mlp_case(31, 1000)
    loss, g = MB.float32_backward(theta, x, t)
    lok, gok, (lc, lr, gc, gr, _) = MB.check_gradient(theta, x, t, loss, g)
    assert lok and gok.all(), np.flatnonzero(~gok)[:10]
    # a 1 % scale error in any one block is rejected
    o = 0
    for name, shape in M.SIZES:
        n = int(np.prod(shape))
        bad = g.astype(np.float64).copy()
        bad[o:o + n] *= 1.01
        _, gbad, _ = MB.check_gradient(theta, x, t, loss, bad)
        assert not gbad[o:o + n].all(), name
        o += n
    # and so is a gradient computed without the bfloat16 rounding of da2
    _, g_plain = M.backward(theta, x, t, emulate=False)
    _, gbad, _ = MB.check_gradient(theta, x, t, loss, g_plain)
    assert not gbad.all()


def test_adam_bounds_accept_float32_update_and_reject_planted_error():
    from tests import mlp_bounds as MB
    f = np.float32
    rng = np.random.default_rng(41)
    n = 4481
    b1, b2, eps, lr = float(f(0.9)), float(f(0.999)), float(f(1e-8)), float(f(1e-3))
    th = rng.standard_normal(n).astype(f)
    m = np.zeros(n, f)
    v = np.zeros(n, f)
    for step in (1, 2, 3, 50, 2000):
        g = (rng.standard_normal(n) * 10.0 ** rng.integers(-6, 1, n)).astype(f)
        # float32 evaluation in the trainer's order
        mm = (f(b1) * m + f(1 - b1) * g).astype(f)
        vv = (f(b2) * v + (f(1 - b2) * g) * g).astype(f)
        bc1, bc2 = f(1.0 - b1 ** step), f(1.0 - b2 ** step)
        upd = (f(lr) * (mm / bc1)) / (np.sqrt(vv / bc2) + f(eps))
        th_new = (th - upd.astype(f)).astype(f)
        (rt, rm, rv), (bt, bm, bv) = MB.adam_bounds(th.astype(np.float64), m.astype(np.float64),
                                                     v.astype(np.float64), g.astype(np.float64), step, lr, b1,
                                                     b2, eps)
        assert (np.abs(mm - rm) <= bm).all() and (np.abs(vv - rv) <= bv).all(), step
        assert (np.abs(th_new - rt) <= bt).all(), step
        # a bias correction off by 1e-5 relative (what a fast power costs at
        # step 1) moves the update outside the bound
        if step == 1:
            bad = (th - (f(lr) * (mm / f(bc1 * (1 + 1e-5)))) / (np.sqrt(vv / bc2) + f(eps))).astype(f)
            assert not (np.abs(bad - rt) <= bt).all()
        th, m, v = th_new, mm, vv
