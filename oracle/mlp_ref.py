"""Reference of the radius-prediction MLP, in float64 with the GPU kernels'
bfloat16 rounding points emulated.

TEST INFRASTRUCTURE ONLY (see the oracle package header).  Written from the
model definition below; shares nothing with the HIP kernels.

Model (the learned part of the query path: it predicts, per query, the log
of the k-th neighbour distance, which becomes an initial search radius):
    x  = bf16((q - lo) * inv)                 inv = fl32(1 / extent), 0 on a flat axis
    a1 = W1 x + b1,   h1 = bf16(relu(a1))     W1: 64x3
    a2 = W2 h1 + b2,  h2 = bf16(relu(a2))     W2: 64x64
    y  = w3 . h2 + b3                         w3: 64
Weights enter every product as bfloat16 copies of float32 master weights;
biases stay float32; sums accumulate in float32 on the GPU (float64 here).
Label: t = 0.5 * ln(max(d2_k, 1e-14)) (log of the k-th neighbour distance).
Loss: mean over the batch of (y - t)^2.
Backward (straight through the bfloat16 casts):
    dy  = 2 (y - t) / B
    gw3 = sum_b dy h2,  gb3 = sum_b dy
    da2 = (dy w3b) * [a2 > 0],  da2b = bf16(da2)
    gW2 = sum_b da2b^T h1,  gb2 = sum_b da2
    da1 = (da2b W2b) * [a1 > 0]
    gW1 = sum_b da1^T x,  gb1 = sum_b da1
Adam (float32 master weights): beta1 0.9, beta2 0.999, eps 1e-8.
Parameter vector order (4481 floats): W1[64][3], b1[64], W2[64][64], b2[64],
w3[64], b3.
"""
from __future__ import annotations

import numpy as np

H = 64
DIN = 3
SIZES = [("W1", (H, DIN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("w3", (H,)), ("b3", ())]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)  # 4481


def bf16(x) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32; returned as float64."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    out = r.view(np.float32)
    out = np.where(np.isnan(f), f, out)
    return out.astype(np.float64)


def fp32(x) -> np.ndarray:
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], np.float64).reshape(-1) for name, _ in SIZES])


def he_init(seed: int) -> np.ndarray:
    """Float32 master weights: He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    p = {"W1": rng.standard_normal((H, DIN)) * np.sqrt(2.0 / DIN),
         "b1": np.zeros(H),
         "W2": rng.standard_normal((H, H)) * np.sqrt(2.0 / H),
         "b2": np.zeros(H),
         "w3": rng.standard_normal(H) * np.sqrt(1.0 / H),
         "b3": np.zeros(())}
    return fp32(pack(p))


def normalize(q, lo, inv, emulate=True) -> np.ndarray:
    q = np.asarray(q, np.float32)
    t = (q - np.asarray(lo, np.float32)).astype(np.float32)
    u = (t * np.asarray(inv, np.float32)).astype(np.float32).astype(np.float64)
    return bf16(u) if emulate else u


def label(d2k) -> np.ndarray:
    return 0.5 * np.log(np.maximum(np.asarray(d2k, np.float64), 1e-14))


def forward(theta, x, emulate=True):
    """Returns (y, cache)."""
    p = unpack(theta)
    rb = bf16 if emulate else (lambda v: np.asarray(v, np.float64))
    act = (lambda v: bf16(fp32(v))) if emulate else (lambda v: v)
    W1b, W2b, w3b = rb(p["W1"]), rb(p["W2"]), rb(p["w3"])
    x = np.asarray(x, np.float64)
    a1 = x @ W1b.T + p["b1"]
    h1 = act(np.maximum(a1, 0.0))
    a2 = h1 @ W2b.T + p["b2"]
    h2 = act(np.maximum(a2, 0.0))
    y = h2 @ w3b + p["b3"]
    return y, dict(x=x, a1=a1, h1=h1, a2=a2, h2=h2, W1b=W1b, W2b=W2b, w3b=w3b)


def loss(theta, x, t, emulate=True) -> float:
    y, _ = forward(theta, x, emulate)
    return float(np.mean((y - np.asarray(t, np.float64)) ** 2))


def backward(theta, x, t, emulate=True):
    """Returns (loss, gradient vector [NPARAM])."""
    y, c = forward(theta, x, emulate)
    t = np.asarray(t, np.float64)
    B = len(t)
    rb = (lambda v: bf16(fp32(v))) if emulate else (lambda v: v)
    dy = 2.0 * (y - t) / B
    gw3 = c["h2"].T @ dy
    gb3 = dy.sum()
    da2 = (dy[:, None] * c["w3b"][None, :]) * (c["a2"] > 0)
    da2b = rb(da2)
    gW2 = da2b.T @ c["h1"]
    gb2 = da2.sum(axis=0)
    da1 = (da2b @ c["W2b"]) * (c["a1"] > 0)
    gW1 = da1.T @ c["x"]
    gb1 = da1.sum(axis=0)
    g = pack({"W1": gW1, "b1": gb1, "W2": gW2, "b2": gb2, "w3": gw3, "b3": gb3})
    return float(np.mean((y - t) ** 2)), g


def adam_step(theta, m, v, g, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1).  Returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def predict_worst0(theta, q, lo, inv, margin, R2) -> np.ndarray:
    """Initial squared search radius per query: min(R2, fl32(r0^2)) with
    r0 = exp(y + margin); a non-finite or negative r0 gives R2."""
    y, _ = forward(theta, normalize(q, lo, inv))
    return worst0_from_y(y, margin, R2)


def worst0_from_y(y, margin, R2) -> np.ndarray:
    """The y -> worst0 step of predict_worst0: r0 = fl32(exp(y + margin)) in
    float64, then min(R2, fl32(r0 * r0)); R2 when r0 is not finite."""
    y = np.asarray(y, np.float64)
    with np.errstate(over="ignore"):
        r0 = fp32(np.exp(y + margin)).astype(np.float32)
    with np.errstate(over="ignore", invalid="ignore"):
        r2 = (r0 * r0).astype(np.float32)
    ok = np.isfinite(r0) & (r0 >= 0)
    return np.where(ok, np.minimum(r2, np.float32(R2)), np.float32(R2)).astype(np.float32)
