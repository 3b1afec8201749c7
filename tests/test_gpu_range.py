"""GPU parity of the range queries (radius and box search) against the
oracle's plain definitions, through the C ABI.

The traversal is the un-ordered form of the stack-free loop (Sec. 3): it
must process every point inside the query region exactly once, so the bar is
exact: counts equal, indices byte-identical and squared distances
bit-identical, row by row.  Radius rows are also kd_knn's rows for
k = cap within the same radius.  Both pruning modes are covered: split planes
only (the paper's traversal, the default) and subtree bounding boxes on
request (disjoint subtrees skipped, subtrees inside the region counted whole
when only counts are asked for)."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2210_12859_amd as kd  # noqa: E402
from paper_2210_12859_amd import datagen  # noqa: E402


def _dev():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(_dev())


def _build(P):
    print(f"[gpu] range: build N={P.shape[0]} D={P.shape[1]}", flush=True)
    return kd.kd_build(_t(P))


BOXES = kd.KD_RANGE_BOXES


def _radius(tree, Qs, maxr, cap, flags=0):
    c, i, d = kd.kd_radius_search(tree, _t(Qs), maxr, cap, flags=flags)
    torch.cuda.synchronize()
    Q = Qs.shape[0]
    return (c.cpu().numpy().astype(np.int64),
            None if i is None else i.cpu().numpy().reshape(Q, cap),
            None if d is None else d.cpu().numpy().reshape(Q, cap))


def _box(tree, lo, hi, cap, flags=0):
    c, i = kd.kd_box_search(tree, _t(lo), _t(hi), cap, flags=flags)
    torch.cuda.synchronize()
    return c.cpu().numpy().astype(np.int64), None if i is None else i.cpu().numpy().reshape(lo.shape[0], cap)


def _same_radius(got, want, cap, ctx):
    gc, gi, gd = got
    oc, oi, od = want
    bad = np.nonzero(gc != oc)[0]
    assert len(bad) == 0, f"{ctx}: counts differ at {bad[:5]} gpu={gc[bad[:3]]} oracle={oc[bad[:3]]}"
    if cap:
        bad = np.nonzero((gi != oi).any(axis=1))[0]
        assert len(bad) == 0, f"{ctx}: idx differ at {bad[:5]} gpu={gi[bad[:1]]} oracle={oi[bad[:1]]}"
        assert np.array_equal(gd.view(np.uint32), od.view(np.uint32)), f"{ctx}: d2 bits differ"


def _same_box(got, want, cap, ctx):
    gc, gi = got
    oc, oi = want
    bad = np.nonzero(gc != oc)[0]
    assert len(bad) == 0, f"{ctx}: counts differ at {bad[:5]} gpu={gc[bad[:3]]} oracle={oc[bad[:3]]}"
    if cap:
        bad = np.nonzero((gi != oi).any(axis=1))[0]
        assert len(bad) == 0, f"{ctx}: idx differ at {bad[:5]} gpu={gi[bad[:1]]} oracle={oi[bad[:1]]}"


def _boxes(rng, Qs, D, scale):
    """Boxes around the query points, per-dimension half-widths drawn up to
    `scale` (several boxes empty, several holding hundreds of points)."""
    h = rng.random((Qs.shape[0], D), dtype=np.float32) * np.float32(scale)
    return (Qs - h).astype(np.float32), (Qs + h).astype(np.float32)


@pytest.mark.parametrize("D", [2, 3, 4])
def test_radius_uniform(oracle_lib, D):
    rng = np.random.default_rng(D)
    N, Q = 40_000, 12_000
    P = rng.random((N, D), dtype=np.float32)
    Qs = rng.random((Q, D), dtype=np.float32)
    tree = _build(P)
    maxr = {2: 0.02, 3: 0.05, 4: 0.12}[D]  # about 50 points per ball
    for cap in (0, 1, 7, 64):
        print(f"[gpu] radius uniform D={D} cap={cap}", flush=True)
        want = oracle_lib.radius(P, Qs, maxr, cap)
        for flags in (0, BOXES):
            _same_radius(_radius(tree, Qs, maxr, cap, flags), want, cap, f"D={D} cap={cap} flags={flags}")
    # rows equal kd_knn's within the same radius
    gi, gd = kd.kd_knn(tree, _t(Qs), 8, maxr)
    _, ri, rd = _radius(tree, Qs, maxr, 8)
    assert np.array_equal(ri, gi.cpu().numpy()) and np.array_equal(rd.view(np.uint32), gd.cpu().numpy().view(np.uint32))
    tree.close()


@pytest.mark.parametrize("D", [2, 3, 4])
def test_box_uniform(oracle_lib, D):
    rng = np.random.default_rng(10 + D)
    N, Q = 40_000, 12_000
    P = rng.random((N, D), dtype=np.float32)
    Qs = rng.random((Q, D), dtype=np.float32)
    lo, hi = _boxes(rng, Qs, D, {2: 0.03, 3: 0.08, 4: 0.15}[D])
    tree = _build(P)
    for cap in (0, 1, 5, 64):
        print(f"[gpu] box uniform D={D} cap={cap}", flush=True)
        want = oracle_lib.box(P, lo, hi, cap)
        for flags in (0, BOXES):
            _same_box(_box(tree, lo, hi, cap, flags), want, cap, f"D={D} cap={cap} flags={flags}")
    tree.close()


def test_radius_ties_on_grid(oracle_lib):
    """Points and queries on a 1/8 grid: many points lie exactly on the ball's
    boundary (d2 == R2 is inside) and on split planes; the split values equal
    query coordinates, so both sides of a plane are reachable."""
    rng = np.random.default_rng(3)
    P = (rng.integers(0, 9, (30_000, 3)) / 8).astype(np.float32)
    Qs = (rng.integers(0, 9, (5_000, 3)) / 8).astype(np.float32)
    tree = _build(P)
    for maxr in (0.0, 0.125, 0.25, math.sqrt(2) * 0.125):
        for cap in (0, 16, 64):
            print(f"[gpu] radius grid maxr={maxr} cap={cap}", flush=True)
            want = oracle_lib.radius(P, Qs, maxr, cap)
            for flags in (0, BOXES):
                _same_radius(_radius(tree, Qs, maxr, cap, flags), want, cap, f"grid maxr={maxr} cap={cap} f={flags}")
    tree.close()


def test_box_ties_degenerate_and_invalid(oracle_lib):
    """Boxes whose faces lie on point coordinates (inclusive), zero-width
    boxes (a single coordinate value), inverted boxes and NaN bounds (empty)."""
    rng = np.random.default_rng(4)
    P = (rng.integers(0, 9, (30_000, 2)) / 8).astype(np.float32)
    Q = 6_000
    a = (rng.integers(0, 9, (Q, 2)) / 8).astype(np.float32)
    b = (rng.integers(0, 9, (Q, 2)) / 8).astype(np.float32)
    lo, hi = np.minimum(a, b), np.maximum(a, b)
    lo[:500] = hi[:500]                # zero-width boxes
    lo[500:1000], hi[500:1000] = hi[500:1000] + 0.0625, lo[500:1000]  # inverted
    lo[1000:1100, 0] = np.nan
    hi[1100:1200, 1] = np.nan
    tree = _build(P)
    for cap in (0, 3, 64):
        print(f"[gpu] box grid cap={cap}", flush=True)
        want = oracle_lib.box(P, lo, hi, cap)
        for flags in (0, BOXES):
            _same_box(_box(tree, lo, hi, cap, flags), want, cap, f"grid boxes cap={cap} flags={flags}")
    c, _ = _box(tree, lo[500:1200], hi[500:1200], 0)
    assert not c.any()
    tree.close()


def test_radius_infinite_nan_and_small_trees(oracle_lib):
    rng = np.random.default_rng(5)
    for N in (1, 2, 3, 7, 64, 65, 1000):
        P = rng.random((N, 3), dtype=np.float32)
        Qs = rng.random((300, 3), dtype=np.float32)
        Qs[7] = np.nan
        Qs[8, 1] = np.nan
        tree = _build(P)
        for maxr, cap in ((math.inf, 64), (math.inf, 0), (0.3, 5), (0.0, 1)):
            want = oracle_lib.radius(P, Qs, maxr, cap)
            for flags in (0, BOXES):
                got = _radius(tree, Qs, maxr, cap, flags)
                _same_radius(got, want, cap, f"N={N} maxr={maxr} cap={cap} flags={flags}")
                if maxr == math.inf:
                    assert (got[0][np.isfinite(Qs).all(axis=1)] == N).all()
                    assert got[0][7] == 0 and got[0][8] == 0
        tree.close()


def test_visited_counts_and_unbounded_regions(oracle_lib):
    """Entered-node counts under split planes only (the default): every point
    in the region is entered, nothing is entered twice, and an unbounded
    region (infinite radius, infinite box faces) enters all N nodes.  With
    subtree boxes and counts only, the unbounded region is counted at the
    root."""
    rng = np.random.default_rng(8)
    N, Q = 20_000, 4_000
    P = rng.random((N, 3), dtype=np.float32)
    Qs = rng.random((Q, 3), dtype=np.float32)
    tree = _build(P)
    q = _t(Qs)
    vis = torch.empty(Q, dtype=torch.int32, device=_dev())
    for maxr in (0.03, math.inf):
        c, _, _ = kd.kd_radius_search(tree, q, maxr, 0, visited=vis)
        torch.cuda.synchronize()
        c, v = c.cpu().numpy(), vis.cpu().numpy()
        assert (v >= c).all() and (v <= N).all() and (v >= 1).all()
        if maxr == math.inf:
            assert (c == N).all() and (v == N).all()
    lo, hi = _boxes(rng, Qs, 3, 0.05)
    lo[:100] = -np.inf
    hi[:100] = np.inf
    hi[100:200, 2] = np.inf
    c, _ = kd.kd_box_search(tree, _t(lo), _t(hi), 4, visited=vis)
    torch.cuda.synchronize()
    c, v = c.cpu().numpy(), vis.cpu().numpy()
    assert (v >= c).all() and (v <= N).all()
    assert (c[:100] == N).all() and (v[:100] == N).all()
    oc, _ = oracle_lib.box(P, lo, hi, 0)
    assert np.array_equal(c, oc)
    # subtree boxes, counts only: the whole tree is counted at the root
    c, _ = kd.kd_box_search(tree, _t(lo), _t(hi), 0, visited=vis, flags=BOXES)
    cr, _, _ = kd.kd_radius_search(tree, q, math.inf, 0, flags=BOXES)
    torch.cuda.synchronize()
    assert np.array_equal(c.cpu().numpy(), oc) and (vis.cpu().numpy()[:100] == 1).all()
    assert (cr.cpu().numpy() == N).all()
    tree.close()


def test_whole_subtree_counts_on_large_regions(oracle_lib):
    """Count-only queries over regions holding thousands of clustered points:
    with subtree boxes, subtrees inside the region are counted without being
    visited, the counts still equal the definition's, and far fewer nodes are
    entered than with split planes alone."""
    P, Qs = datagen.workload("gmm64-1m")
    rows = np.random.default_rng(12).choice(Qs.shape[0], 3000, replace=False)
    Qs = Qs[rows]
    tree = _build(P)
    q = _t(Qs)
    v0 = torch.empty(len(Qs), dtype=torch.int32, device=_dev())
    v1 = torch.empty(len(Qs), dtype=torch.int32, device=_dev())
    for maxr in (0.01, 0.03):
        print(f"[gpu] range gmm64 count-only radius {maxr}", flush=True)
        c0, _, _ = kd.kd_radius_search(tree, q, maxr, 0, visited=v0, flags=BOXES)
        c1, _, _ = kd.kd_radius_search(tree, q, maxr, 0, visited=v1)
        torch.cuda.synchronize()
        oc, _, _ = oracle_lib.radius(P, Qs, maxr, 0)
        assert np.array_equal(c0.cpu().numpy(), oc) and np.array_equal(c1.cpu().numpy(), oc)
        assert v0.sum().item() * 2 < v1.sum().item()
        h = np.float32(maxr)
        b0, _ = kd.kd_box_search(tree, _t(Qs - h), _t(Qs + h), 0, visited=v0, flags=BOXES)
        b1, _ = kd.kd_box_search(tree, _t(Qs - h), _t(Qs + h), 0, visited=v1)
        torch.cuda.synchronize()
        ob, _ = oracle_lib.box(P, Qs - h, Qs + h, 0)
        assert np.array_equal(b0.cpu().numpy(), ob) and np.array_equal(b1.cpu().numpy(), ob)
        assert v0.sum().item() * 2 < v1.sum().item()
    tree.close()


def test_empty_inputs():
    dev = _dev()
    tree = kd.kd_build(torch.zeros((0, 3), dtype=torch.float32, device=dev))
    q = torch.rand((100, 3), device=dev)
    c, i, d = kd.kd_radius_search(tree, q, math.inf, 4)
    bc, bi = kd.kd_box_search(tree, q - 1, q + 1, 4)
    torch.cuda.synchronize()
    assert (c == 0).all() and (i == -1).all() and torch.isinf(d).all()
    assert (bc == 0).all() and (bi == -1).all()
    tree.close()
    tree = kd.kd_build(torch.rand((1000, 3), device=dev))
    e = torch.zeros((0, 3), dtype=torch.float32, device=dev)
    c, i, d = kd.kd_radius_search(tree, e, 0.1, 4)
    bc, bi = kd.kd_box_search(tree, e, e, 4)
    torch.cuda.synchronize()
    assert c.numel() == 0 and i.numel() == 0 and bc.numel() == 0
    tree.close()


def test_radius_box_clustered_1m_sampled(oracle_lib):
    """1M clustered points (the shape of the kNN workloads), 1M queries in one
    launch each: counts and rows of 4,000 sampled queries against the
    definitions, radius rows of every query against kd_knn."""
    P, Qs = datagen.workload("gmm64-1m")
    rng = np.random.default_rng(6)
    tree = _build(P)
    maxr, cap = 0.01, 16
    print("[gpu] range gmm64-1m: radius and box over 1M queries", flush=True)
    gc, gi, gd = _radius(tree, Qs, maxr, cap)
    lo, hi = _boxes(rng, Qs, 3, 0.01)
    bc, bi = _box(tree, lo, hi, cap)
    ki, kd2 = kd.kd_knn(tree, _t(Qs), cap, maxr)
    torch.cuda.synchronize()
    assert np.array_equal(gi, ki.cpu().numpy()), "radius rows differ from kd_knn"
    assert np.array_equal(gd.view(np.uint32), kd2.cpu().numpy().view(np.uint32))
    rows = rng.choice(Qs.shape[0], 4000, replace=False)
    print("[gpu] range gmm64-1m: oracle on 4000 sampled rows", flush=True)
    oc, oi, od = oracle_lib.radius(P, Qs[rows], maxr, cap)
    _same_radius((gc[rows], gi[rows], gd[rows]), (oc, oi, od), cap, "gmm64 radius")
    oc, oi = oracle_lib.box(P, lo[rows], hi[rows], cap)
    _same_box((bc[rows], bi[rows]), (oc, oi), cap, "gmm64 box")
    assert gc.sum() > 10 * Qs.shape[0] and bc.sum() > Qs.shape[0]  # non-trivial regions
    tree.close()


def test_clustered_10m_sampled_rows(oracle_lib):
    """10M clustered points, 1M queries in one launch per call (radius with
    cap 16, radius counts with and without subtree boxes, box counts): 400
    sampled rows against the definitions over the points whose x lies in
    the query's slab (every point in range is among them)."""
    P, Qs = datagen.workload("clustered-10m")
    Qs = Qs[: 1 << 20]
    tree = _build(P)
    q = _t(Qs)
    maxr, cap, h = 0.01, 16, np.float32(0.008)
    print("[gpu] range clustered-10m: radius and box over 1M queries", flush=True)
    rc, ri, rd = kd.kd_radius_search(tree, q, maxr, cap)
    cc, _, _ = kd.kd_radius_search(tree, q, maxr, 0, flags=BOXES)
    bc, _ = kd.kd_box_search(tree, _t(Qs - h), _t(Qs + h), 0, flags=BOXES)
    bp, _ = kd.kd_box_search(tree, _t(Qs - h), _t(Qs + h), 0)
    torch.cuda.synchronize()
    rc, ri, rd = rc.cpu().numpy(), ri.cpu().numpy(), rd.cpu().numpy()
    cc, bc, bp = cc.cpu().numpy(), bc.cpu().numpy(), bp.cpu().numpy()
    assert np.array_equal(rc, cc) and np.array_equal(bc, bp)
    order = np.argsort(P[:, 0], kind="stable")
    xs = P[order, 0].astype(np.float64)
    rows = np.random.default_rng(13).choice(len(Qs), 400, replace=False)
    print("[gpu] range clustered-10m: definitions on 400 sampled rows", flush=True)
    for row in rows:
        x = float(Qs[row, 0])
        r = maxr * (1 + 1e-5) + 1e-12
        cand = np.sort(order[np.searchsorted(xs, x - r, "left"):np.searchsorted(xs, x + r, "right")])
        oc, oi, od = oracle_lib.radius(P[cand], Qs[row][None, :], maxr, cap)
        oi = np.where(oi[0] >= 0, cand[np.maximum(oi[0], 0)], -1)
        assert rc[row] == oc[0] and np.array_equal(ri[row], oi), f"radius row {row}"
        assert np.array_equal(rd[row].view(np.uint32), od[0].view(np.uint32)), f"radius d2 row {row}"
        lo, hi = Qs[row] - h, Qs[row] + h
        cand = np.sort(order[np.searchsorted(xs, float(lo[0]), "left"):np.searchsorted(xs, float(hi[0]), "right")])
        ob, _ = oracle_lib.box(P[cand], lo[None, :], hi[None, :], 0)
        assert bc[row] == ob[0], f"box row {row}"
    tree.close()


def _all_same(offsets, idx, want_lists, ctx):
    off = offsets.cpu().numpy()
    got = idx.cpu().numpy()
    assert off[0] == 0 and off[-1] == len(got), ctx
    for q, w in enumerate(want_lists):
        g = np.sort(got[off[q]:off[q + 1]])
        assert np.array_equal(g, np.sort(w)), f"{ctx}: query {q} gpu {len(g)} oracle {len(w)}"


@pytest.mark.parametrize("D", [2, 3, 4])
def test_all_results(oracle_lib, D):
    """Every point in range, variable-length output: each query's slice holds
    exactly the definition's points (compared as sets: the order is the
    traversal's), with and without subtree boxes in the counting pass."""
    rng = np.random.default_rng(30 + D)
    P = rng.random((20_000, D), dtype=np.float32)
    P[:500] = P[500:1000]  # duplicates
    Qs = rng.random((3_000, D), dtype=np.float32)
    Qs[5] = np.nan
    tree = _build(P)
    maxr = {2: 0.03, 3: 0.08, 4: 0.15}[D]
    h = np.float32({2: 0.03, 3: 0.07, 4: 0.12}[D])
    oc, _, _ = oracle_lib.radius(P, Qs, maxr, 0)
    kmax = int(oc.max())
    _, oi, _ = oracle_lib.radius(P, Qs, maxr, kmax)
    want = [oi[q][oi[q] >= 0] for q in range(len(Qs))]
    bc, _ = oracle_lib.box(P, Qs - h, Qs + h, 0)
    _, bi = oracle_lib.box(P, Qs - h, Qs + h, int(bc.max()))
    bwant = [bi[q][bi[q] >= 0] for q in range(len(Qs))]
    for flags in (0, BOXES):
        print(f"[gpu] range all D={D} flags={flags}", flush=True)
        off, idx = kd.kd_radius_search_all(tree, _t(Qs), maxr, flags=flags)
        torch.cuda.synchronize()
        _all_same(off, idx, want, f"radius D={D} flags={flags}")
        off, idx = kd.kd_box_search_all(tree, _t(Qs - h), _t(Qs + h), flags=flags)
        torch.cuda.synchronize()
        _all_same(off, idx, bwant, f"box D={D} flags={flags}")
    tree.close()


def test_all_results_capacity_and_empty():
    dev = _dev()
    rng = np.random.default_rng(40)
    P = rng.random((5_000, 3), dtype=np.float32)
    Qs = rng.random((700, 3), dtype=np.float32)
    tree = _build(P)
    q = _t(Qs)
    L = kd.lib()
    import ctypes
    offsets = torch.empty(len(Qs) + 1, dtype=torch.int64, device=dev)
    out = torch.full((8,), -7, dtype=torch.int32, device=dev)
    tot = ctypes.c_int64()
    st = torch.cuda.current_stream().cuda_stream
    rc = L.kd_radius_search_all(tree.handle, ctypes.c_void_p(q.data_ptr()), len(Qs), 0.1,
                                ctypes.c_void_p(offsets.data_ptr()), ctypes.c_void_p(out.data_ptr()), 8,
                                ctypes.byref(tot), 0, ctypes.c_void_p(st))
    assert rc == kd.KD_OK and tot.value > 8
    assert offsets[-1].item() == tot.value and (out == -7).all()  # too small: indices untouched
    c, _, _ = kd.kd_radius_search(tree, q, 0.1, 0)
    assert np.array_equal(np.diff(offsets.cpu().numpy()), c.cpu().numpy().astype(np.int64))
    # exact capacity, then empty query sets and an empty tree
    off2, idx2 = kd.kd_radius_search_all(tree, q, 0.1, capacity=tot.value)
    assert len(idx2) == tot.value and torch.equal(off2, offsets)
    off3, idx3 = kd.kd_radius_search_all(tree, q[:0], 0.1)
    assert off3.tolist() == [0] and idx3.numel() == 0
    tree.close()
    empty = kd.kd_build(torch.zeros((0, 3), dtype=torch.float32, device=dev))
    off4, idx4 = kd.kd_box_search_all(empty, q - 1, q + 1)
    assert (off4 == 0).all() and idx4.numel() == 0
    empty.close()


def test_all_results_offsets_at_scale(oracle_lib):
    """The offsets of large query sets: 300K queries (73 scan blocks) against
    the per-query counts, with sampled slices against the definition; and
    17M queries over a small tree (more block totals than one pass of the
    totals scan holds) against the counts."""
    rng = np.random.default_rng(50)
    P = rng.random((50_000, 3), dtype=np.float32)
    Qs = rng.random((300_000, 3), dtype=np.float32)
    tree = _build(P)
    q = _t(Qs)
    off, idx = kd.kd_radius_search_all(tree, q, 0.03)
    c, _, _ = kd.kd_radius_search(tree, q, 0.03, 0)
    torch.cuda.synchronize()
    off, idx = off.cpu().numpy(), idx.cpu().numpy()
    assert np.array_equal(np.diff(off), c.cpu().numpy().astype(np.int64)) and off[-1] == len(idx)
    rows = rng.choice(len(Qs), 300, replace=False)
    oc, _, _ = oracle_lib.radius(P, Qs[rows], 0.03, 0)
    _, oi, _ = oracle_lib.radius(P, Qs[rows], 0.03, int(oc.max()))
    for t, r in enumerate(rows):
        assert np.array_equal(np.sort(idx[off[r]:off[r + 1]]), np.sort(oi[t][oi[t] >= 0])), f"row {r}"
    tree.close()
    small = kd.kd_build(_t(rng.random((64, 3), dtype=np.float32)))
    print("[gpu] range all: 17M queries over 64 points", flush=True)
    q2 = torch.rand((17_000_000, 3), device=_dev())
    off2, idx2 = kd.kd_radius_search_all(small, q2, 0.05)
    c2, _, _ = kd.kd_radius_search(small, q2, 0.05, 0)
    torch.cuda.synchronize()
    assert torch.equal(torch.diff(off2), c2.to(torch.int64)) and off2[0].item() == 0
    assert off2[-1].item() == idx2.numel()
    small.close()
