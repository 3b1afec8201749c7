"""GPU parity of trees with stored split dimensions (the widest extent of
each node's points, 2 bits per node) against the oracle's variant, through
the C ABI.

Bar: the GPU builder's level order and dimensions byte-identical to the
oracle's; kNN indices byte-identical, squared distances bit-identical and,
under the paper's pruning rule, per-query processed-node counts equal to the
oracle's recursion over the same tree; range queries exact."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2210_12859_amd as kd  # noqa: E402
from paper_2210_12859_amd import datagen  # noqa: E402

W = kd.KD_SPLIT_WIDEST


def _dev():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda:0")


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(_dev())


def _build(P):
    print(f"[gpu] widest build N={P.shape[0]} D={P.shape[1]}", flush=True)
    return kd.kd_build(_t(P), split=W)


def _same_tree(oracle_lib, tree, P, ctx):
    oo, od = oracle_lib.build_tree_widest(P)
    go = tree.order()
    gd, rule = tree.dims()
    assert rule == W
    assert np.array_equal(go, oo), f"{ctx}: order differs at {np.nonzero(go != oo)[0][:5]}"
    assert np.array_equal(gd, od), f"{ctx}: dims differ at {np.nonzero(gd != od)[0][:5]}"
    return oo, od


def _same_knn(tree, P, Qs, order, dims, oracle_lib, k, maxr, opts, ctx, visited=True):
    gi, gd, gv = kd.kd_knn_ex(tree, _t(Qs), k, maxr, want_visited=visited, opts=opts)
    torch.cuda.synchronize()
    oi, od, ov = oracle_lib.knn(P, order, Qs, k, maxr, dims=dims)
    gi = gi.cpu().numpy().reshape(oi.shape)
    gd = gd.cpu().numpy().reshape(od.shape)
    bad = np.nonzero((gi != oi).any(axis=1))[0]
    assert len(bad) == 0, f"{ctx}: idx differ at {bad[:5]}"
    assert np.array_equal(gd.view(np.uint32), od.view(np.uint32)), f"{ctx}: d2 bits differ"
    if visited:
        gv = gv.cpu().numpy().astype(np.int64)
        vb = np.nonzero(gv != ov)[0]
        assert len(vb) == 0, f"{ctx}: visited differ at {vb[:5]} gpu={gv[vb[:3]]} oracle={ov[vb[:3]]}"
    return ov


def _data(kind, N, D, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.random((N, D), dtype=np.float32)
    if kind == "aspect":
        return (rng.random((N, D)) * np.array([1, 30, 3, 0.1][:D])).astype(np.float32)
    if kind == "grid":
        return rng.integers(0, 9, (N, D)).astype(np.float32)
    if kind == "dups":
        return np.repeat(rng.random((N // 8, D), dtype=np.float32), 8, axis=0)
    c = rng.random((16, D)) * np.array([1, 4, 0.5, 2][:D])
    return (c[rng.integers(0, 16, N)] + rng.normal(0, 0.01, (N, D))).astype(np.float32)


@pytest.mark.parametrize("kind", ["uniform", "aspect", "grid", "dups", "clusters"])
@pytest.mark.parametrize("D", [2, 3, 4])
def test_builder_and_knn(oracle_lib, kind, D):
    P = _data(kind, 60_000, D, 100 + D)
    Qs = _data(kind, 8_000, D, 200 + D)
    tree = _build(P)
    order, dims = _same_tree(oracle_lib, tree, P, f"{kind} D={D}")
    for k, maxr in ((1, math.inf), (8, math.inf), (5, 0.05)):
        print(f"[gpu] widest {kind} D={D} k={k} maxr={maxr}", flush=True)
        _same_knn(tree, P, Qs, order, dims, oracle_lib, k, maxr, {"prune": 1}, f"{kind} D={D} k={k}")
        _same_knn(tree, P, Qs, order, dims, oracle_lib, k, maxr, None, f"{kind} D={D} k={k} default",
                  visited=False)
    tree.close()


def test_small_trees_and_k64(oracle_lib):
    rng = np.random.default_rng(3)
    for N in (1, 2, 3, 7, 64, 65, 1000):
        for D in (2, 3, 4):
            P = (rng.random((N, D)) * np.array([1, 5, 0.3, 2][:D])).astype(np.float32)
            Qs = rng.random((300, D), dtype=np.float32)
            tree = _build(P)
            order, dims = _same_tree(oracle_lib, tree, P, f"N={N} D={D}")
            for k in (1, 64):
                _same_knn(tree, P, Qs, order, dims, oracle_lib, k, math.inf, {"prune": 1}, f"N={N} D={D} k={k}")
            tree.close()


def test_handoff_and_noalloc(oracle_lib):
    """Queries finished by the cooperative kernel (tiny trip budgets) and the
    no-allocation entry point read the stored dimensions too."""
    P = _data("clusters", 100_000, 3, 7)
    Qs = _data("uniform", 6_000, 3, 8) * np.float32(2.0)
    tree = _build(P)
    order, dims = _same_tree(oracle_lib, tree, P, "handoff")
    for trips in (4, 40):
        for prune in (1, 2):
            _same_knn(tree, P, Qs, order, dims, oracle_lib, 8, math.inf,
                      {"heavy_trips": trips, "prune": prune}, f"handoff trips={trips} prune={prune}", visited=False)
    ni, nd = kd.kd_knn_noalloc(tree, _t(Qs), 8)
    torch.cuda.synchronize()
    oi, od, _ = oracle_lib.knn(P, order, Qs, 8, dims=dims)
    assert np.array_equal(ni.cpu().numpy(), oi) and np.array_equal(nd.cpu().numpy().view(np.uint32), od.view(np.uint32))
    tree.close()


def test_range_queries(oracle_lib):
    P = _data("aspect", 50_000, 3, 11)
    Qs = _data("aspect", 6_000, 3, 12)
    tree = _build(P)
    _same_tree(oracle_lib, tree, P, "range")
    c, i, d = kd.kd_radius_search(tree, _t(Qs), 0.2, 16)
    h = np.float32(0.15)
    bc, bi = kd.kd_box_search(tree, _t(Qs - h), _t(Qs + h), 16)
    torch.cuda.synchronize()
    oc, oi, od = oracle_lib.radius(P, Qs, 0.2, 16)
    assert np.array_equal(c.cpu().numpy(), oc) and np.array_equal(i.cpu().numpy(), oi)
    assert np.array_equal(d.cpu().numpy().view(np.uint32), od.view(np.uint32))
    oc, oi = oracle_lib.box(P, Qs - h, Qs + h, 16)
    assert np.array_equal(bc.cpu().numpy(), oc) and np.array_equal(bi.cpu().numpy(), oi)
    # counts only, with and without subtree boxes
    orc, _, _ = oracle_lib.radius(P, Qs, 0.5, 0)
    for flags in (0, kd.KD_RANGE_BOXES):
        c, _, _ = kd.kd_radius_search(tree, _t(Qs), 0.5, 0, flags=flags)
        bc, _ = kd.kd_box_search(tree, _t(Qs - h), _t(Qs + h), 0, flags=flags)
        torch.cuda.synchronize()
        assert np.array_equal(c.cpu().numpy(), orc) and np.array_equal(bc.cpu().numpy(), oc)
    # rows kept with subtree boxes (disjoint subtrees skipped)
    c, i, d = kd.kd_radius_search(tree, _t(Qs), 0.2, 16, flags=kd.KD_RANGE_BOXES)
    torch.cuda.synchronize()
    orc2, ori2, ord2 = oracle_lib.radius(P, Qs, 0.2, 16)
    assert np.array_equal(c.cpu().numpy(), orc2) and np.array_equal(i.cpu().numpy(), ori2)
    assert np.array_equal(d.cpu().numpy().view(np.uint32), ord2.view(np.uint32))
    # every point in range, as offsets + indices
    off, idx = kd.kd_box_search_all(tree, _t(Qs - h), _t(Qs + h))
    torch.cuda.synchronize()
    off, idx = off.cpu().numpy(), idx.cpu().numpy()
    _, oall = oracle_lib.box(P, Qs - h, Qs + h, int(oc.max()))
    for q in range(len(Qs)):
        assert np.array_equal(np.sort(idx[off[q]:off[q + 1]]), oall[q][oall[q] >= 0]), f"box all, query {q}"
    tree.close()


@pytest.mark.parametrize("D", [2, 4])
def test_range_queries_2d_4d(oracle_lib, D):
    P = _data("aspect", 30_000, D, 60 + D)
    Qs = _data("aspect", 4_000, D, 70 + D)
    tree = _build(P)
    _same_tree(oracle_lib, tree, P, f"range D={D}")
    r = {2: 0.3, 4: 0.6}[D]
    h = np.float32({2: 0.2, 4: 0.4}[D])
    for flags in (0, kd.KD_RANGE_BOXES):
        c, i, d = kd.kd_radius_search(tree, _t(Qs), r, 8, flags=flags)
        bc, bi = kd.kd_box_search(tree, _t(Qs - h), _t(Qs + h), 8, flags=flags)
        torch.cuda.synchronize()
        oc, oi, od = oracle_lib.radius(P, Qs, r, 8)
        ob, obi = oracle_lib.box(P, Qs - h, Qs + h, 8)
        assert np.array_equal(c.cpu().numpy(), oc) and np.array_equal(i.cpu().numpy(), oi)
        assert np.array_equal(d.cpu().numpy().view(np.uint32), od.view(np.uint32))
        assert np.array_equal(bc.cpu().numpy(), ob) and np.array_equal(bi.cpu().numpy(), obi)
    tree.close()


def test_autotune_and_unsupported(oracle_lib):
    P = _data("clusters", 50_000, 3, 13)
    Qs = _data("clusters", 20_000, 3, 14)
    tree = _build(P)
    order, dims = _same_tree(oracle_lib, tree, P, "autotune")
    kd.kd_autotune(tree, _t(Qs[:8192]), 8)
    _same_knn(tree, P, Qs, order, dims, oracle_lib, 8, math.inf, None, "tuned default", visited=False)
    q = _t(Qs)
    with pytest.raises(kd.KdError) as e:
        kd.kd_knn_ex(tree, q, 8, opts={"lds_levels": 8})
    assert e.value.status == kd.KD_EINVAL
    r0 = torch.full((Qs.shape[0],), 0.01, device=_dev())
    with pytest.raises(kd.KdError) as e:
        kd.kd_knn_with_radius(tree, r0, q, 8)
    assert e.value.status == kd.KD_EUNSUPPORTED
    with pytest.raises(kd.KdError) as e:
        kd.kd_knn_batched([dict(tree=tree, queries=q, k=8,
                                out_idx=torch.empty((Qs.shape[0], 8), dtype=torch.int32, device=_dev()))])
    assert e.value.status == kd.KD_EUNSUPPORTED
    tree.close()


def test_level_rule_trees_report_level_dims():
    P = _data("uniform", 1000, 3, 15)
    tree = kd.kd_build(_t(P))
    dims, rule = tree.dims()
    lvl = np.floor(np.log2(np.arange(1000) + 1)).astype(np.int64) % 3
    assert rule == kd.KD_SPLIT_LEVEL and np.array_equal(dims, lvl)
    tree.close()


def test_gmm64_1m_every_row_and_clustered_10m_subset(oracle_lib):
    """The clustered workloads at full size: gmm64-1m (1M points, 1M queries,
    k = 8, every row, processed counts) and clustered-10m (k = 16, rows
    0 .. 2^18 - 1)."""
    P, Qs = datagen.workload("gmm64-1m")
    tree = _build(P)
    order, dims = _same_tree(oracle_lib, tree, P, "gmm64-1m")
    print("[gpu] widest gmm64-1m k=8 every row", flush=True)
    _same_knn(tree, P, Qs, order, dims, oracle_lib, 8, math.inf, {"prune": 1}, "gmm64-1m")
    tree.close()
    P, Qs = datagen.workload("clustered-10m")
    tree = _build(P)
    print("[gpu] widest clustered-10m: oracle build", flush=True)
    order, dims = _same_tree(oracle_lib, tree, P, "clustered-10m")
    m = 1 << 18
    print("[gpu] widest clustered-10m k=16 subset", flush=True)
    _same_knn(tree, P, Qs[:m], order, dims, oracle_lib, 16, math.inf, {"prune": 1}, "clustered-10m", visited=False)
    tree.close()
