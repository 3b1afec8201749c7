"""Rigorous per-output error bounds for the GPU's MLP arithmetic, around the
float64 reference with the GPU's bfloat16 rounding points (oracle.mlp_ref).

The GPU accumulates in float32 (matrix cores and vector ALU, in an order the
reference does not fix).  A sum of K products then differs from the exact sum
by at most K * 2^-23 * sum|a_i b_i| (any order, any float32 rounding mode).
Where such an error can move a pre-activation across a bfloat16 rounding
boundary (or across 0 for a ReLU mask) the GPU may round the other way; the
bounds below do not guess which: every quantity is carried as an interval
(midpoint, radius) that encloses every value the GPU can hold, the
monotone roundings map interval ends to interval ends, and the possible flips
widen only the outputs they feed.  An output is accepted when it lies inside
its interval.  Outputs untouched by any flip get the plain accumulation bound,
which is about 1e-5 relative for these sizes: a 1 % error in a weight block
falls far outside.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp_ref as M

GAMMA = 2.0 ** -23  # per-term accumulation factor of the bound
U32 = 2.0 ** -24    # float32 unit roundoff (one rounding)
SLACK = 1e-12       # float64 evaluation of the enclosures themselves


def _mr(lo, hi):
    return 0.5 * (lo + hi), 0.5 * (hi - lo)


def _act(c, r):
    """bf16(fp32(relu(a))) over a in [c - r, c + r]: the map is monotone, so
    the ends map to the ends.  Returns (midpoint, radius)."""
    lo = M.bf16(M.fp32(np.maximum(c - r, 0.0)))
    hi = M.bf16(M.fp32(np.maximum(c + r, 0.0)))
    return _mr(lo, hi)


def _matmul(Ac, Ar, Bc, Br, K):
    """Enclosure of A @ B over interval matrices, evaluated in float32 with
    K-term sums: (midpoint, radius)."""
    C = Ac @ Bc
    Amax, Bmax = np.abs(Ac) + Ar, np.abs(Bc) + Br
    R = np.abs(Ac) @ Br + Ar @ np.abs(Bc) + Ar @ Br + (K * GAMMA + SLACK) * (Amax @ Bmax)
    return C, R


def _add_bias(C, R, b, K):
    return C + b, R + (K * GAMMA + SLACK) * np.abs(b)


def _mask(c, r):
    """[a > 0] over a in [c - r, c + r]: 1, 0, or either (-1)."""
    return np.where(c - r > 0, 1, np.where(c + r <= 0, 0, -1))


def _apply_mask(vc, vr, mask):
    """v * [a > 0] with the mask possibly either value: the hull of {v, 0}."""
    lo, hi = vc - vr, vc + vr
    lo = np.where(mask == 0, 0.0, np.where(mask == -1, np.minimum(lo, 0.0), lo))
    hi = np.where(mask == 0, 0.0, np.where(mask == -1, np.maximum(hi, 0.0), hi))
    return _mr(lo, hi)


def forward_enclosure(theta, x):
    """Intervals of every forward quantity the GPU computes for inputs x
    (already normalised and rounded to bfloat16).  Returns a dict of
    (midpoint, radius) pairs plus the masks and weights."""
    p = M.unpack(theta)
    W1b, W2b, w3b = M.bf16(p["W1"]), M.bf16(p["W2"]), M.bf16(p["w3"])
    x = np.asarray(x, np.float64)
    zx = np.zeros_like(x)
    a1c, a1r = _matmul(x, zx, W1b.T, np.zeros_like(W1b.T), 4)
    a1c, a1r = _add_bias(a1c, a1r, p["b1"], 4)
    h1c, h1r = _act(a1c, a1r)
    a2c, a2r = _matmul(h1c, h1r, W2b.T, np.zeros_like(W2b.T), 65)
    a2c, a2r = _add_bias(a2c, a2r, p["b2"], 65)
    h2c, h2r = _act(a2c, a2r)
    yc, yr = _matmul(h2c, h2r, w3b[:, None], np.zeros((M.H, 1)), 65)
    yc, yr = _add_bias(yc[:, 0], yr[:, 0], p["b3"], 65)
    return dict(x=x, a1=(a1c, a1r), h1=(h1c, h1r), a2=(a2c, a2r), h2=(h2c, h2r), y=(yc, yr),
                W1b=W1b, W2b=W2b, w3b=w3b, flips=(h1r > 0).any(axis=1) | (h2r > 0).any(axis=1))


def check_forward(theta, x, y_gpu):
    """(ok mask per query, enclosure).  ok[i]: y_gpu[i] lies in its interval."""
    e = forward_enclosure(theta, x)
    yc, yr = e["y"]
    ok = np.abs(np.asarray(y_gpu, np.float64) - yc) <= yr
    return ok, e


def gradient_enclosure(theta, x, t):
    """Intervals of the loss and of the gradient (parameter order) the GPU's
    trainer computes for one batch (x normalised and rounded, targets t):
    ((loss midpoint, radius), (gradient midpoint, radius))."""
    e = forward_enclosure(theta, x)
    t = np.asarray(t, np.float64)
    B = len(t)
    s = 2.0 / B
    yc, yr = e["y"]
    # err = fl(y - t), dy = fl(fl(2 / B) * err): three roundings
    ec, er = yc - t, yr + U32 * (np.abs(yc - t) + yr)
    dyc, dyr = s * ec, s * er * (1 + 3 * U32) + 3 * U32 * s * np.abs(ec)
    emax = np.abs(ec) + er
    emin = np.maximum(np.abs(ec) - er, 0.0)
    lc, lr = _mr(np.sum(emin ** 2) / B, np.sum(emax ** 2) / B)
    lr = lr + (B * GAMMA + 2 * U32) * np.sum(emax ** 2) / B

    col = lambda v: v[:, None]
    h2c, h2r = e["h2"]
    h1c, h1r = e["h1"]
    gw3c, gw3r = _matmul(h2c.T, h2r.T, col(dyc), col(dyr), B)
    gb3c = dyc.sum()
    gb3r = dyr.sum() + (B * GAMMA + SLACK) * np.sum(np.abs(dyc) + dyr)
    # da2 = fl(dy * w3b) * [a2 > 0]
    w3b = e["w3b"][None, :]
    pc, pr = col(dyc) * w3b, col(dyr) * np.abs(w3b)
    pr = pr + U32 * (np.abs(pc) + pr)
    da2c, da2r = _apply_mask(pc, pr, _mask(*e["a2"]))
    gb2c = da2c.sum(axis=0)
    gb2r = da2r.sum(axis=0) + (B * GAMMA + SLACK) * np.sum(np.abs(da2c) + da2r, axis=0)
    # da2b = bf16(da2) (monotone)
    da2bc, da2br = _mr(M.bf16(M.fp32(da2c - da2r)), M.bf16(M.fp32(da2c + da2r)))
    gW2c, gW2r = _matmul(da2bc.T, da2br.T, h1c, h1r, B)
    dh1c, dh1r = _matmul(da2bc, da2br, e["W2b"], np.zeros_like(e["W2b"]), M.H)
    da1c, da1r = _apply_mask(dh1c, dh1r, _mask(*e["a1"]))
    gb1c = da1c.sum(axis=0)
    gb1r = da1r.sum(axis=0) + (B * GAMMA + SLACK) * np.sum(np.abs(da1c) + da1r, axis=0)
    gW1c, gW1r = _matmul(da1c.T, da1r.T, e["x"], np.zeros_like(e["x"]), B)
    gc = M.pack({"W1": gW1c, "b1": gb1c, "W2": gW2c, "b2": gb2c, "w3": gw3c[:, 0], "b3": gb3c})
    gr = M.pack({"W1": gW1r, "b1": gb1r, "W2": gW2r, "b2": gb2r, "w3": gw3r[:, 0], "b3": gb3r})
    return (lc, lr), (gc, gr), e


def check_gradient(theta, x, t, loss_gpu, g_gpu):
    """(loss ok, per-parameter ok mask, enclosures)."""
    (lc, lr), (gc, gr), e = gradient_enclosure(theta, x, t)
    g = np.asarray(g_gpu, np.float64)
    return abs(float(loss_gpu) - lc) <= lr, np.abs(g - gc) <= gr, (lc, lr, gc, gr, e)


def adam_bounds(theta, m0, v0, g, step, lr, b1, b2, eps):
    """Reference Adam step (oracle, float64) on the same float32 inputs and
    hyper-parameters, with the float32 evaluation's error bounds:
    returns (theta, m, v) references and their absolute bounds."""
    th, m, v = M.adam_step(theta, m0, v0, g, step, lr=lr, b1=b1, b2=b2, eps=eps)
    Mabs = np.abs(b1 * m0) + np.abs((1 - b1) * g)   # no cancellation bound for m
    Vabs = b2 * v0 + (1 - b2) * g * g                # v has none
    bm = 3 * U32 * Mabs + SLACK * Mabs
    bv = 4 * U32 * Vabs + SLACK * Vabs
    bc1, bc2 = 1 - b1 ** step, 1 - b2 ** step
    S = np.sqrt(v / bc2) + eps
    bth = 16 * U32 * lr * (Mabs / bc1) / S + U32 * np.abs(th) + SLACK * np.abs(th)
    return (th, m, v), (bth, bm, bv)


def float32_forward(theta, x, W2_scale=1.0):
    """The forward in float32 arithmetic (numpy), with the GPU's rounding
    points: used on the CPU to show the enclosure accepts a float32
    evaluation and rejects a planted error (W2_scale != 1)."""
    p = {k: np.asarray(v, np.float32) for k, v in M.unpack(theta).items()}
    b = lambda v: M.bf16(v).astype(np.float32)
    x = np.asarray(x, np.float32)
    a1 = x @ b(p["W1"]).T + p["b1"]
    h1 = b(np.maximum(a1, 0))
    a2 = h1 @ (b(p["W2"]) * np.float32(W2_scale)).T + p["b2"]
    h2 = b(np.maximum(a2, 0))
    return (h2 @ b(p["w3"]) + p["b3"]).astype(np.float64)


def float32_backward(theta, x, t):
    """The trainer's loss and gradient in float32 arithmetic (numpy), with the
    GPU's rounding points (CPU check of the enclosure)."""
    f = np.float32
    p = {k: np.asarray(v, f) for k, v in M.unpack(theta).items()}
    b = lambda v: M.bf16(v).astype(f)
    x = np.asarray(x, f)
    t = np.asarray(t, f)
    W1b, W2b, w3b = b(p["W1"]), b(p["W2"]), b(p["w3"])
    a1 = x @ W1b.T + p["b1"]
    h1 = b(np.maximum(a1, 0))
    a2 = h1 @ W2b.T + p["b2"]
    h2 = b(np.maximum(a2, 0))
    y = h2 @ w3b + p["b3"]
    err = (y - t).astype(f)
    dy = (f(2.0 / len(t)) * err).astype(f)
    gw3 = h2.T @ dy
    gb3 = dy.sum(dtype=f)
    da2 = np.where(a2 > 0, dy[:, None] * w3b[None, :], f(0)).astype(f)
    da2b = b(da2)
    gW2 = da2b.T @ h1
    gb2 = da2.sum(axis=0, dtype=f)
    da1 = np.where(a1 > 0, da2b @ W2b, f(0)).astype(f)
    gW1 = da1.T @ x
    gb1 = da1.sum(axis=0, dtype=f)
    loss = float(np.sum(err * err, dtype=f) / f(len(t)))
    g = M.pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "w3": gw3, "b3": gb3})
    return loss, g
