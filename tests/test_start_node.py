"""CPU check of the start-node rule of the learned path (test-side, no GPU):
descending from the root while the split plane is farther than the initial
radius (fl32(sd*sd) > worst0), every point within worst0 lies in the subtree
of the node reached.  Checked on the oracle's canonical trees against brute
force with float32 arithmetic, for radii from 0 to well past the k-th
neighbour, on uniform data and on integer grids full of ties (points exactly
on split planes)."""
import numpy as np
import pytest

from paper_2210_12859_amd import datagen


def _f32(x):
    return np.float32(x)


def _subtree_positions(pos, n):
    """Level-order positions (0-based) of the subtree rooted at pos."""
    out, level = [], [pos]
    while level:
        level = [p for p in level if p < n]
        out.extend(level)
        level = [c for p in level for c in (2 * p + 1, 2 * p + 2)]
    return np.array(sorted(out), dtype=np.int64)


def _start_position(pts_lo, q, w0):
    """Descent with 0-based positions; split dim = level mod D."""
    n, D = pts_lo.shape
    pos = 0
    while True:
        level = int(np.floor(np.log2(pos + 1)))
        d = level % D
        sd = _f32(q[d] - pts_lo[pos, d])
        if not (_f32(sd * sd) > w0):
            return pos
        close = 2 * pos + 2 if sd > 0 else 2 * pos + 1
        if close >= n:
            return pos
        pos = close


def _d2(pts, q):
    dx = (q[None, :] - pts).astype(np.float32)
    s = dx[:, 0] * dx[:, 0]
    for j in range(1, pts.shape[1]):
        s = (s + dx[:, j] * dx[:, j]).astype(np.float32)
    return s


@pytest.mark.parametrize("kind,n,D", [("uniform", 3000, 3), ("uniform", 1000, 2), ("grid", 1500, 3), ("uniform", 777, 4)])
def test_points_within_radius_lie_below_start_node(oracle_lib, kind, n, D):
    rng = np.random.default_rng(n + D)
    if kind == "grid":
        P = rng.integers(0, 6, size=(n, D)).astype(np.float32) * 0.25
        Qs = rng.integers(-1, 7, size=(200, D)).astype(np.float32) * 0.25
    else:
        P = datagen.uniform(n, D, n)
        Qs = datagen.uniform(200, D, n + 1)
    order = oracle_lib.build_tree(P)
    pts_lo = P[order]
    descended = 0
    for q in Qs:
        d2_all = _d2(pts_lo, q)
        kth = np.sort(d2_all)[min(8, n) - 1]
        for w0 in (_f32(0.0), _f32(kth * 0.5), _f32(kth), _f32(kth * 1.5), _f32(kth * 4.0)):
            s = _start_position(pts_lo, q, w0)
            descended += s > 0
            inside = set(np.nonzero(d2_all <= w0)[0].tolist())
            assert inside <= set(_subtree_positions(s, n).tolist()), (q, w0, s)
    assert descended > 0  # the rule does skip levels on these inputs
