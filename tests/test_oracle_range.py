"""Pins of the oracle's radius and box queries (plain definitions, brute force):
the Figure 1 point set with hand-worked cases, exact radius boundaries,
closed forms (everything / nothing / duplicates only), NaN, and independent
numpy evaluations with explicit float32 operations on small random and
integer-grid inputs."""
import json
import math
import os

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def _d2_np(P, q):
    dx = (np.float32(1) * q[None, :] - P).astype(np.float32)
    s = (dx[:, 0] * dx[:, 0]).astype(np.float32)
    for j in range(1, P.shape[1]):
        s = (s + (dx[:, j] * dx[:, j]).astype(np.float32)).astype(np.float32)
    return s


def _fig1():
    d = json.load(open(os.path.join(HERE, "golden", "figure1.json")))
    return np.array(d["points"], np.float32)


def test_figure1_radius_cases(oracle_lib):
    P = _fig1()
    # q = (9, 2): d2 to the six points = 50, 20, 16, 50, 2, 4
    q = np.array([[9, 2]], np.float32)
    for maxr, want in [(1.4142135, 0), (1.5, 1), (2.0, 2), (4.0, 3), (math.sqrt(20.0), 4), (math.inf, 6)]:
        cnt, _, _ = oracle_lib.radius(P, q, maxr)
        assert cnt[0] == want, (maxr, cnt[0])
    # q = (3, 5): points 0, 1, 3 at d2 = 5 exactly (ties); radius sqrt(5) rounds to
    # fl32 = 2.236068 whose square rounds to 5.0 exactly -> all three included
    cnt, idx, d2 = oracle_lib.radius(P, np.array([[3, 5]], np.float32), math.sqrt(5.0), k=4)
    r2 = oracle_lib.sq_radius(math.sqrt(5.0))
    assert (cnt[0] == 3) == (r2 >= np.float32(5.0))
    assert list(idx[0][: cnt[0]]) == [0, 1, 3][: cnt[0]]


def test_figure1_box_cases(oracle_lib):
    P = _fig1()
    cnt, idx = oracle_lib.box(P, np.array([[0, 0]], np.float32), np.array([[10, 10]], np.float32), k=6)
    assert cnt[0] == 6 and list(idx[0]) == [0, 1, 2, 3, 4, 5]
    # [4, 8] x [1, 4]: (5,4) idx 1, (8,1) idx 4, (7,2) idx 5 (corners inclusive)
    cnt, idx = oracle_lib.box(P, np.array([[4, 1]], np.float32), np.array([[8, 4]], np.float32), k=4)
    assert cnt[0] == 3 and list(idx[0]) == [1, 4, 5, -1]
    # degenerate box on one point, and an empty (inverted) box
    cnt, _ = oracle_lib.box(P, np.array([[9, 6]], np.float32), np.array([[9, 6]], np.float32))
    assert cnt[0] == 1
    cnt, _ = oracle_lib.box(P, np.array([[5, 5]], np.float32), np.array([[4, 9]], np.float32))
    assert cnt[0] == 0


@pytest.mark.parametrize("kind,n,D", [("uniform", 500, 2), ("uniform", 800, 3), ("grid", 600, 3), ("uniform", 300, 4)])
def test_radius_against_numpy(oracle_lib, kind, n, D):
    rng = np.random.default_rng(n * D)
    if kind == "grid":
        P = rng.integers(0, 5, size=(n, D)).astype(np.float32)
        Qs = rng.integers(-1, 6, size=(60, D)).astype(np.float32)
        radii = [0.0, 1.0, 1.5, 2.0, math.inf]
    else:
        P = rng.random((n, D), dtype=np.float32)
        Qs = rng.random((60, D), dtype=np.float32)
        radii = [0.0, 0.05, 0.2, math.inf]
    for r in radii:
        cnt, idx, d2 = oracle_lib.radius(P, Qs, r, k=7)
        R2 = oracle_lib.sq_radius(r)
        for t, q in enumerate(Qs):
            dd = _d2_np(P, q)
            inside = np.nonzero(dd <= R2)[0]
            assert cnt[t] == len(inside)
            keys = sorted((float(dd[i]), int(i)) for i in inside)[:7]
            want = [i for _, i in keys] + [-1] * (7 - len(keys))
            assert list(idx[t]) == want
        bi, bd = oracle_lib.brute(P, Qs, 7, r)
        assert np.array_equal(bi, idx) and np.array_equal(bd.view(np.uint32), d2.view(np.uint32))
    # closed forms: duplicates only at radius 0, everything at infinity
    cnt0, _, _ = oracle_lib.radius(P, P[:20], 0.0)
    for t in range(20):
        assert cnt0[t] == int((P == P[t]).all(axis=1).sum())
    cinf, _, _ = oracle_lib.radius(P, Qs, math.inf)
    assert (cinf == n).all()


@pytest.mark.parametrize("kind,n,D", [("uniform", 500, 2), ("grid", 700, 3), ("uniform", 300, 4)])
def test_box_against_numpy(oracle_lib, kind, n, D):
    rng = np.random.default_rng(n + D)
    if kind == "grid":
        P = rng.integers(0, 5, size=(n, D)).astype(np.float32)
        a = rng.integers(-1, 6, size=(80, D)).astype(np.float32)
        b = rng.integers(-1, 6, size=(80, D)).astype(np.float32)
    else:
        P = rng.random((n, D), dtype=np.float32)
        a = rng.random((80, D), dtype=np.float32)
        b = rng.random((80, D), dtype=np.float32)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    lo[:10] = b[:10]  # some inverted (empty) boxes
    hi[:10] = a[:10]
    cnt, idx = oracle_lib.box(P, lo, hi, k=9)
    for t in range(len(lo)):
        inside = np.nonzero(((P >= lo[t]) & (P <= hi[t])).all(axis=1))[0]
        assert cnt[t] == len(inside)
        want = list(inside[:9]) + [-1] * max(0, 9 - len(inside))
        assert list(idx[t]) == want
    everything, _ = oracle_lib.box(P, np.full((3, D), -1e30, np.float32), np.full((3, D), 1e30, np.float32))
    assert (everything == n).all()


def test_nan_queries_find_nothing(oracle_lib):
    P = np.random.default_rng(0).random((100, 3), dtype=np.float32)
    q = np.array([[np.nan, 0.5, 0.5]], np.float32)
    cnt, idx, _ = oracle_lib.radius(P, q, math.inf, k=3)
    assert cnt[0] == 0 and (idx == -1).all()
    cnt, idx = oracle_lib.box(P, q, np.array([[1, 1, 1]], np.float32), k=3)
    assert cnt[0] == 0 and (idx == -1).all()
