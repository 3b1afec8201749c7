"""GPU parity of the cooperative hand-off: queries whose single-lane
traversal runs past the trip budget are finished by a whole wave
(kd_opts.heavy_trips).  Small budgets force most queries through that kernel;
indices and squared distances must still equal the oracle's bit for bit, on
clustered data (where far-off queries visit many nodes), on duplicated points
(every tie decided by the smaller index), with a finite radius, and for every
list size."""
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


def _check(oracle_lib, P, Qs, k, maxr, opts, tag):
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    print(f"[gpu] hand-off {tag} N={len(P)} Q={len(Qs)} k={k} maxr={maxr} opts={opts}", flush=True)
    gi, gd, _ = kd.kd_knn_ex(tree, q, k, maxr, opts=opts)
    torch.cuda.synchronize()
    order = oracle_lib.build_tree(P)
    oi, od, _ = oracle_lib.knn(P, order, Qs, k, maxr)
    gi = gi.cpu().numpy().reshape(len(Qs), k)
    gd = gd.cpu().numpy().reshape(len(Qs), k)
    assert np.array_equal(gi, oi), tag
    assert np.array_equal(gd.view(np.uint32), od.view(np.uint32)), tag
    tree.close()


@pytest.mark.parametrize("k", [1, 2, 8, 13, 32, 64])
@pytest.mark.parametrize("trips", [1, 16, 200])
def test_handoff_gmm_exact(oracle_lib, k, trips):
    P = datagen.gmm(20000, 3, 3, n_centers=16, sigma=0.004)
    Qs = np.concatenate([datagen.gmm(3000, 3, 4, n_centers=16, sigma=0.004), datagen.uniform(1000, 3, 5)])
    _check(oracle_lib, P, Qs, k, math.inf, dict(heavy_trips=trips), "gmm")


@pytest.mark.parametrize("dim", [2, 3, 4])
def test_handoff_dims_and_radius(oracle_lib, dim):
    P = datagen.gmm(9000, dim, 6, n_centers=8, sigma=0.01)
    Qs = datagen.uniform(2500, dim, 7)
    _check(oracle_lib, P, Qs, 8, math.inf, dict(heavy_trips=8), f"dim{dim}")
    _check(oracle_lib, P, Qs, 8, 0.05, dict(heavy_trips=8), f"dim{dim}-r0.05")


def test_handoff_duplicates_and_ties(oracle_lib):
    rng = np.random.default_rng(11)
    base = rng.integers(0, 6, size=(700, 3)).astype(np.float32)
    P = np.concatenate([base, base, base[:300], np.zeros((200, 3), np.float32)])
    Qs = rng.integers(-1, 7, size=(900, 3)).astype(np.float32) * 0.5
    for k in (1, 8, 64):
        _check(oracle_lib, P, Qs, k, math.inf, dict(heavy_trips=4), f"ties-k{k}")


def test_handoff_small_trees(oracle_lib):
    for n in (1, 2, 3, 5, 64, 127, 128, 129, 1500):
        P = datagen.uniform(n, 3, n)
        Qs = datagen.uniform(300, 3, n + 1)
        _check(oracle_lib, P, Qs, 8, math.inf, dict(heavy_trips=1), f"n{n}")


def test_handoff_default_equals_none_at_scale(oracle_lib):
    """gmm64-1m k=8 with the default budget vs no hand-off: identical."""
    P, Qs = datagen.workload("gmm64-1m")
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    ai, ad, _ = kd.kd_knn_ex(tree, q, 8, opts=dict(heavy_trips=-1))
    bi, bd = kd.kd_knn(tree, q, 8)
    ci, cd, _ = kd.kd_knn_ex(tree, q, 8, opts=dict(heavy_trips=64))
    torch.cuda.synchronize()
    assert torch.equal(ai, bi) and torch.equal(ad.view(torch.int32), bd.view(torch.int32))
    assert torch.equal(ai, ci) and torch.equal(ad.view(torch.int32), cd.view(torch.int32))
    rows = np.random.default_rng(0).choice(len(Qs), 300, replace=False)
    oi, od = oracle_lib.brute(P, Qs[rows], 8, math.inf)
    assert np.array_equal(bi.cpu().numpy()[rows], oi)


def test_handoff_learned_exact(oracle_lib):
    P = datagen.gmm(30000, 3, 8, n_centers=16, sigma=0.004)
    Qs = np.concatenate([datagen.gmm(3000, 3, 9, n_centers=16, sigma=0.004), datagen.uniform(1000, 3, 10)])
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    order = oracle_lib.build_tree(P)
    oi, od, _ = oracle_lib.knn(P, order, Qs, 8)
    kth = np.sqrt(od[:, -1].astype(np.float64))
    for name, r0 in [("under", kth * 0.5), ("over", kth * 2.0), ("zero", np.zeros(len(Qs)))]:
        r = torch.from_numpy(r0.astype(np.float32)).to(_dev())
        gi, gd, _, gf = kd.kd_knn_with_radius(tree, r, q, 8, want_flags=True, opts=dict(heavy_trips=6))
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy().reshape(-1, 8), oi), name
        assert np.array_equal(gd.cpu().numpy().reshape(-1, 8).view(np.uint32), od.view(np.uint32)), name
        assert set(np.unique(gf.cpu().numpy())) <= {0, 1, 2}, name
