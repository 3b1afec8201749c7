"""Pins for the CPU oracle (no GPU): the paper's Figure 1 example, brute force,
closed forms, invariants and the stack-free equivalence claim of Sec. 3.1."""
import json
import os

import numpy as np
import pytest

from tests import refimpl

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _f(x):
    return np.float32(np.inf) if x == "inf" else np.float32(x)


def _maxr(case):
    if "max_radius_bits" in case:
        return np.array([int(case["max_radius_bits"], 16)], np.uint32).view(np.float32)[0]
    return _f(case["max_radius"])


# ------------------------------------------------------------------ leftSize

def test_left_size_small_values(oracle_lib):
    assert [oracle_lib.left_size(n) for n in range(0, 9)] == [0, 0, 1, 1, 2, 3, 3, 3, 4]


def test_left_size_equals_counted_subtree(oracle_lib):
    # size of the subtree rooted at position 1 of an n-node complete tree
    for n in range(2, 700):
        assert oracle_lib.left_size(n) == len(refimpl.subtree_positions(1, n)), n


# ---------------------------------------------------------------- Figure 1

def test_figure1_tree(oracle_lib):
    g = json.load(open(os.path.join(GOLDEN, "figure1.json")))
    P = np.array(g["points"], np.float32)
    order = oracle_lib.build_tree(P)
    assert order.tolist() == g["order"]


@pytest.mark.parametrize("name", ["A", "A-prime", "A-1.5", "B", "B3", "B6", "B7"])
def test_figure1_queries(oracle_lib, name):
    g = json.load(open(os.path.join(GOLDEN, "figure1.json")))
    P = np.array(g["points"], np.float32)
    case = [c for c in g["queries"] if c["name"] == name][0]
    order = np.array(g["order"], np.int32)
    maxr = _maxr(case)
    if "r2_bits" in case:
        assert hex(oracle_lib.sq_radius(maxr).view(np.uint32)) == case["r2_bits"]
    idx, d2, vis, found = oracle_lib.knn_one(P, order, case["q"], case["k"], maxr)
    assert idx.tolist() == case["idx"]
    assert d2.tolist() == [float(_f(x)) for x in case["d2"]]
    if "processed" in case:
        assert vis == case["processed"]
    # brute force agrees
    bi, bd = oracle_lib.brute(P, np.array([case["q"]], np.float32), case["k"], maxr)
    assert bi[0].tolist() == case["idx"]


# ------------------------------------------------------------ build checks

def _check_tree_invariants(P, order, left_size):
    N, D = P.shape
    assert sorted(order.tolist()) == list(range(N))
    for pos in range(N):
        dim = int(np.floor(np.log2(pos + 1))) % D
        key = (P[order[pos], dim], order[pos])
        L = refimpl.subtree_positions(2 * pos + 1, N)
        R = refimpl.subtree_positions(2 * pos + 2, N)
        for p in L:
            assert (P[order[p], dim], order[p]) < key
        for p in R:
            assert (P[order[p], dim], order[p]) > key
        assert len(L) == left_size(len(L) + len(R) + 1)


@pytest.mark.parametrize("N,D,seed", [(1, 3, 0), (2, 2, 1), (7, 3, 2), (31, 2, 3), (100, 3, 4),
                                      (257, 4, 5), (300, 1, 6)])
def test_build_invariants_random(oracle_lib, N, D, seed):
    P = np.random.default_rng(seed).random((N, D), dtype=np.float32)
    _check_tree_invariants(P, oracle_lib.build_tree(P), oracle_lib.left_size)


def test_build_invariants_ties(oracle_lib):
    rng = np.random.default_rng(11)
    P = rng.integers(0, 3, size=(200, 3)).astype(np.float32)
    _check_tree_invariants(P, oracle_lib.build_tree(P), oracle_lib.left_size)


@pytest.mark.parametrize("N", [1, 2, 5, 16, 17, 100, 1023, 1024, 1025])
def test_build_1d_is_eytzinger(oracle_lib, N):
    rng = np.random.default_rng(N)
    P = rng.integers(0, N // 3 + 2, size=(N, 1)).astype(np.float32)
    sorted_ids = np.lexsort((np.arange(N), P[:, 0]))
    assert oracle_lib.build_tree(P).tolist() == refimpl.eytzinger(sorted_ids).tolist()


# ------------------------------------------------- traversal vs brute force

def _cases():
    out = []
    for N in [0, 1, 2, 3, 4, 5, 7, 8, 15, 16, 17, 100, 1000]:
        for D in [1, 2, 3, 4]:
            out.append((N, D))
    return out


@pytest.mark.parametrize("N,D", _cases())
def test_traversal_equals_brute_random(oracle_lib, N, D):
    rng = np.random.default_rng(1000 * N + D)
    P = rng.random((N, D), dtype=np.float32)
    Qs = rng.random((24, D), dtype=np.float32)
    order = oracle_lib.build_tree(P) if N else np.zeros(0, np.int32)
    for k in sorted({1, 2, 3, min(N + 2, 9), N + 2} - {0}):
        for maxr in [0.0, 0.05, 0.3, np.inf]:
            R2 = oracle_lib.sq_radius(maxr)
            ti, td, _ = oracle_lib.knn(P, order, Qs, k, maxr)
            for i, q in enumerate(Qs):
                bi, bd = refimpl.brute_np(P, q, k, R2)
                assert ti[i].tolist() == bi.tolist(), (N, D, k, maxr, i)
                assert td[i].view(np.uint32).tolist() == bd.view(np.uint32).tolist()


@pytest.mark.parametrize("D", [2, 3])
def test_traversal_equals_brute_integer_grid(oracle_lib, D):
    # coordinates in {0..7}: masses of exact d2 ties and sd^2 == worst cases
    rng = np.random.default_rng(77 + D)
    P = rng.integers(0, 8, size=(400, D)).astype(np.float32)
    Qs = rng.integers(0, 8, size=(64, D)).astype(np.float32)
    Qs[::2] += 0.5
    order = oracle_lib.build_tree(P)
    for k in [1, 4, 8, 33]:
        for maxr in [0.0, 1.0, 2.0, np.inf]:
            ti, td, _ = oracle_lib.knn(P, order, Qs, k, maxr)
            bi, bd = oracle_lib.brute(P, Qs, k, maxr)
            assert np.array_equal(ti, bi)
            assert np.array_equal(td.view(np.uint32), bd.view(np.uint32))
            for i in range(0, 64, 7):
                ni, nd = refimpl.brute_np(P, Qs[i], k, oracle_lib.sq_radius(maxr))
                assert ti[i].tolist() == ni.tolist()


def test_brute_c_equals_brute_numpy(oracle_lib):
    rng = np.random.default_rng(5)
    P = rng.random((500, 3), dtype=np.float32)
    Qs = rng.random((40, 3), dtype=np.float32)
    for k in [1, 8, 64]:
        bi, bd = oracle_lib.brute(P, Qs, k)
        for i in range(40):
            ni, nd = refimpl.brute_np(P, Qs[i], k, np.float32(np.inf))
            assert bi[i].tolist() == ni.tolist()
            assert bd[i].view(np.uint32).tolist() == nd.view(np.uint32).tolist()


# --------------------------------------------------------------- closed forms

def test_k_at_least_n_returns_all_sorted(oracle_lib):
    rng = np.random.default_rng(3)
    P = rng.random((13, 3), dtype=np.float32)
    q = rng.random(3, dtype=np.float32)
    order = oracle_lib.build_tree(P)
    idx, d2, _, found = oracle_lib.knn_one(P, order, q, 16)
    s = refimpl.d2_np(P, q)
    exp = np.lexsort((np.arange(13), s))
    assert found == 13
    assert idx[:13].tolist() == exp.tolist()
    assert idx[13:].tolist() == [-1, -1, -1]
    assert np.all(np.isinf(d2[13:]))


def test_zero_radius_returns_exact_duplicates_only(oracle_lib):
    rng = np.random.default_rng(4)
    P = rng.random((50, 3), dtype=np.float32)
    P[10] = P[3]
    P[40] = P[3]
    order = oracle_lib.build_tree(P)
    idx, d2, _, found = oracle_lib.knn_one(P, order, P[3], 8, 0.0)
    assert found == 3
    assert idx[:3].tolist() == [3, 10, 40]
    assert d2[:3].tolist() == [0.0, 0.0, 0.0]


def test_all_points_identical(oracle_lib):
    P = np.full((37, 3), 0.25, np.float32)
    order = oracle_lib.build_tree(P)
    idx, d2, _, _ = oracle_lib.knn_one(P, order, np.array([0.5, 0.5, 0.5], np.float32), 8)
    assert idx.tolist() == list(range(8))


def test_query_equal_to_unique_point(oracle_lib):
    rng = np.random.default_rng(9)
    P = rng.random((300, 3), dtype=np.float32)
    order = oracle_lib.build_tree(P)
    for i in [0, 17, 299]:
        idx, d2, _, _ = oracle_lib.knn_one(P, order, P[i], 3)
        assert idx[0] == i and d2[0] == 0.0


def test_nan_query_gives_empty(oracle_lib):
    rng = np.random.default_rng(10)
    P = rng.random((100, 3), dtype=np.float32)
    order = oracle_lib.build_tree(P)
    q = np.array([np.nan, 0.5, 0.5], np.float32)
    idx, d2, _, found = oracle_lib.knn_one(P, order, q, 4)
    assert found == 0 and idx.tolist() == [-1] * 4
    bi, _ = refimpl.brute_np(P, q, 4, np.float32(np.inf))
    assert bi.tolist() == [-1] * 4


# ---------------------------------------------------------------- invariants

def test_prefix_and_filter_properties(oracle_lib):
    rng = np.random.default_rng(12)
    P = rng.random((2000, 3), dtype=np.float32)
    Qs = rng.random((50, 3), dtype=np.float32)
    order = oracle_lib.build_tree(P)
    i16, d16, _ = oracle_lib.knn(P, order, Qs, 16)
    for k in [1, 4, 8, 15]:
        ik, dk, _ = oracle_lib.knn(P, order, Qs, k)
        assert np.array_equal(ik, i16[:, :k])
    r = 0.07
    ir, dr, _ = oracle_lib.knn(P, order, Qs, 16, r)
    R2 = oracle_lib.sq_radius(r)
    keep = d16 <= R2
    assert np.array_equal(np.where(keep, i16, -1), ir)


# ---------------------------------------------- stack-free equivalence claim

@pytest.mark.parametrize("N,D,k", [(1, 2, 1), (6, 2, 2), (17, 3, 1), (100, 3, 4), (255, 2, 8),
                                   (256, 3, 8), (513, 4, 3)])
def test_stackfree_processes_same_sequence(oracle_lib, N, D, k):
    """The oracle's recursion processes the nodes of an independent
    explicit-stack walk, in the same order, with the same result; the walk's
    tour moves only between parent and child (what lets two integers carry
    the state, Sec. 3.1), so consecutive entries determine each move."""
    rng = np.random.default_rng(N + 31 * D)
    P = rng.random((N, D), dtype=np.float32)
    order = oracle_lib.build_tree(P)
    R2 = np.float32(np.inf)
    for t in range(12):
        q = rng.random(D, dtype=np.float32)
        if t == 11:
            q = P[order[N // 2]].copy()
        seq, tour, sidx, sd = refimpl.ordered_walk(P, order, q, k, R2)
        oi, od, vis, _, oseq = oracle_lib.knn_one(P, order, q, k, record_sequence=True)
        assert oseq.tolist() == seq
        assert vis == len(seq)
        assert oi.tolist() == sidx.tolist()
        assert tour[0] == 0 and tour[-1] == 0
        for a, b in zip(tour, tour[1:]):
            assert b in (2 * a + 1, 2 * a + 2) or a in (2 * b + 1, 2 * b + 2), (a, b)
        # every entry but the root's comes down one edge and goes back up it
        entries = sum(1 for a, b in zip([-1] + tour, tour) if b > a)
        assert len(tour) == 2 * entries - 1


def test_figure1_stackfree_iterations():
    """Loop trips of the two-integer traversal on the Figure 1 tree: one per
    entry in the tour (9 for fcp at (9, 2), 15 for k = 2 at (3, 5))."""
    g = json.load(open(os.path.join(GOLDEN, "figure1.json")))
    P = np.array(g["points"], np.float32)
    order = np.array(g["order"], np.int32)
    seq, tour, idx, _ = refimpl.ordered_walk(P, order, [9, 2], 1, np.float32(np.inf))
    assert seq == [0, 2, 5] and len(tour) == 9 and idx.tolist() == [4]
    seq, tour, idx, _ = refimpl.ordered_walk(P, order, [3, 5], 2, np.float32(np.inf))
    assert seq == [0, 1, 4, 3] and len(tour) == 15 and idx.tolist() == [0, 1]


# ------------------------------------------------------------ learned rule

def test_learned_rule_is_exact_for_any_radius(oracle_lib):
    rng = np.random.default_rng(21)
    P = rng.random((3000, 3), dtype=np.float32)
    Qs = rng.random((200, 3), dtype=np.float32)
    order = oracle_lib.build_tree(P)
    k = 8
    pi, pd, pv = oracle_lib.knn(P, order, Qs, k)
    kth = np.sqrt(pd[:, -1].astype(np.float64))
    for r0 in [np.zeros(200), np.full(200, 1e-30), np.full(200, -1.0), np.full(200, np.nan),
               np.full(200, np.inf), rng.random(200) * 0.1, kth * 1.0001, kth * 0.9]:
        li, ld, lv, fb = oracle_lib.knn_learned(P, order, Qs, k, r0.astype(np.float32))
        assert np.array_equal(li, pi)
        assert np.array_equal(ld.view(np.uint32), pd.view(np.uint32))
        w0 = np.array([oracle_lib.worst0(np.inf, r) for r in r0.astype(np.float32)], np.float32)
        # fallback exactly when fewer than k points lie within worst0
        within = np.array([(refimpl.d2_np(P, Qs[i]) <= w0[i]).sum() for i in range(200)])
        assert np.array_equal(fb, (within < k) & (w0 < np.float32(np.inf)))


def test_learned_perfect_radius_saves_visits(oracle_lib):
    rng = np.random.default_rng(22)
    P = rng.random((20000, 3), dtype=np.float32)
    Qs = rng.random((300, 3), dtype=np.float32)
    order = oracle_lib.build_tree(P)
    pi, pd, pv = oracle_lib.knn(P, order, Qs, 8)
    r0 = np.sqrt(pd[:, -1].astype(np.float64)) * (1 + 2.0**-20)
    li, ld, lv, fb = oracle_lib.knn_learned(P, order, Qs, 8, r0.astype(np.float32))
    assert not fb.any()
    assert lv.sum() < pv.sum()
