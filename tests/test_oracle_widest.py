"""Pins of the oracle's stored-split-dimension variant (the builder chooses
each node's split dimension and stores it, Sec. 3 and Sec. 4): the widest
extent of the node's point set, fl32(max - min), lowest dimension on ties.

The build is checked node by node against brute-force subtree sets (the
dimension, the left-balanced ranks, the (coordinate, index) order across the
node), on a hand-worked example, against the level rule where the two must
agree (D = 1), and the traversal over it against brute force and against an
independent explicit-stack walk reading the same dimensions."""
import numpy as np
import pytest

from tests import refimpl


def _widest_np(P):
    with np.errstate(over="ignore"):
        ext = (P.max(axis=0) - P.min(axis=0)).astype(np.float32)
    return int(np.argmax(ext))  # first of the largest


def _check_tree(oracle_lib, P, order, dims):
    N, D = P.shape
    assert sorted(order.tolist()) == list(range(N))
    assert dims.shape == (N,) and (dims < D).all()
    for pos in range(N):
        sub = refimpl.subtree_positions(pos, N)
        pts = P[order[sub]]
        d = int(dims[pos])
        assert d == _widest_np(pts), pos
        L = refimpl.subtree_positions(2 * pos + 1, N)
        R = refimpl.subtree_positions(2 * pos + 2, N)
        assert len(L) == oracle_lib.left_size(len(sub))
        me = (P[order[pos], d], order[pos])
        for q in L:
            assert (P[order[q], d], order[q]) < me
        for q in R:
            assert (P[order[q], d], order[q]) > me


def test_hand_worked_six_points(oracle_lib):
    # root: x spans 10, y spans 9 -> x; left set {0, 5, 2}: x spans 3, y 4 ->
    # y, placed idx 2; right set {3, 1}: x spans 3, y 2 -> x, placed idx 1
    # (the level rule would split this node on y and place idx 3)
    P = np.array([[0, 0], [10, 1], [3, 2], [7, 3], [5, 9], [1, 4]], np.float32)
    order, dims = oracle_lib.build_tree_widest(P)
    assert order.tolist() == [4, 2, 1, 0, 5, 3]
    assert dims.tolist() == [0, 1, 0, 0, 0, 0]
    assert oracle_lib.build_tree(P)[2] == 3
    # fcp of (8, 2): root (5, 9) d2 58, right child (10, 1) d2 5, its left
    # child (7, 3) d2 2; both far sides are out of range (9 > 2, 4 > 2)
    oi, od, vis, found, seq = oracle_lib.knn_one(P, order, [8, 2], 1, record_sequence=True, dims=dims)
    assert oi.tolist() == [3] and od.tolist() == [2.0] and vis == 3 and seq.tolist() == [0, 2, 5]


def test_three_points(oracle_lib):
    P = np.array([[0, 0], [1, 10], [2, 5]], np.float32)
    order, dims = oracle_lib.build_tree_widest(P)
    assert order.tolist() == [2, 0, 1] and dims.tolist() == [1, 0, 0]


@pytest.mark.parametrize("kind", ["uniform", "aspect", "grid", "dups", "clusters"])
@pytest.mark.parametrize("D", [2, 3, 4])
def test_every_node(oracle_lib, kind, D):
    rng = np.random.default_rng(["uniform", "aspect", "grid", "dups", "clusters"].index(kind) * 10 + D)
    N = 700
    if kind == "uniform":
        P = rng.random((N, D), dtype=np.float32)
    elif kind == "aspect":
        P = (rng.random((N, D)) * np.array([1, 30, 3, 0.1][:D])).astype(np.float32)
    elif kind == "grid":
        P = rng.integers(0, 5, (N, D)).astype(np.float32)
    elif kind == "dups":
        P = np.repeat(rng.random((70, D), dtype=np.float32), 10, axis=0)
    else:
        c = rng.random((6, D)) * 10
        P = (c[rng.integers(0, 6, N)] + rng.normal(0, 0.05, (N, D))).astype(np.float32)
    order, dims = oracle_lib.build_tree_widest(P)
    _check_tree(oracle_lib, P, order, dims)


def test_signed_zeros_and_huge_extents(oracle_lib):
    P = np.zeros((40, 3), np.float32)
    P[::2, 0] = -0.0
    P[:, 1] = np.linspace(-3e38, 3e38, 40, dtype=np.float32)  # extent overflows to inf
    P[:, 2] = np.linspace(-3e38, 3e38, 40, dtype=np.float32)[::-1]
    order, dims = oracle_lib.build_tree_widest(P)
    # inf extents in y and z: the lower dimension (y) wins at the root
    assert dims[0] == 1
    _check_tree(oracle_lib, P, order, dims)


def test_one_dimension_equals_level_rule(oracle_lib):
    P = np.random.default_rng(0).random((1000, 1), dtype=np.float32)
    order, dims = oracle_lib.build_tree_widest(P)
    assert np.array_equal(order, oracle_lib.build_tree(P)) and not dims.any()


@pytest.mark.parametrize("D", [2, 3, 4])
def test_traversal_exact_and_same_walk(oracle_lib, D):
    rng = np.random.default_rng(40 + D)
    P = (rng.random((3000, D)) * np.array([1, 8, 0.25, 3][:D])).astype(np.float32)
    Qs = (rng.random((400, D)) * np.array([1, 8, 0.25, 3][:D])).astype(np.float32)
    order, dims = oracle_lib.build_tree_widest(P)
    for k, maxr in ((1, np.inf), (8, np.inf), (5, 0.3)):
        oi, od, vis = oracle_lib.knn(P, order, Qs, k, maxr, dims=dims)
        bi, bd = oracle_lib.brute(P, Qs, k, maxr)
        assert np.array_equal(oi, bi) and np.array_equal(od.view(np.uint32), bd.view(np.uint32))
    for i in range(40):
        seq, tour, wi, _ = refimpl.ordered_walk(P, order, Qs[i], 4, np.float32(np.inf), dims=dims)
        oi, od, v, _, oseq = oracle_lib.knn_one(P, order, Qs[i], 4, record_sequence=True, dims=dims)
        assert oseq.tolist() == seq and v == len(seq) and oi.tolist() == wi.tolist()


def test_widest_rule_prunes_elongated_data(oracle_lib):
    """Points spread along one axis much more than the others (a thin slab):
    the level rule spends splits on the thin axes, the widest rule does not,
    and processes fewer nodes for the same (exact) results."""
    rng = np.random.default_rng(9)
    P = (rng.random((20000, 3)) * np.array([1.0, 0.01, 0.01])).astype(np.float32)
    Qs = (rng.random((300, 3)) * np.array([1.0, 0.01, 0.01])).astype(np.float32)
    lo = oracle_lib.build_tree(P)
    wo, wd = oracle_lib.build_tree_widest(P)
    li, ld, lv = oracle_lib.knn(P, lo, Qs, 8)
    wi, wdd, wv = oracle_lib.knn(P, wo, Qs, 8, dims=wd)
    assert np.array_equal(li, wi) and np.array_equal(ld.view(np.uint32), wdd.view(np.uint32))
    assert wv.mean() < 0.8 * lv.mean()
