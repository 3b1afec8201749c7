"""GPU parity with the top tree levels staged in LDS (kd_opts.lds_levels): the
traversal is unchanged, only where the records of the top levels are read
from, so indices, squared distances and the paper's processed-node counts
must equal the oracle's for every dimension, staged depth (including trees
smaller than the staged levels), list size and radius, also with the
subtree-box rule and through the cooperative hand-off; the learned path
ignores the option.  Invalid depths are rejected before any launch."""
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


def _check(oracle_lib, P, Qs, k, maxr, opts, tag, visited=True):
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    print(f"[gpu] lds {tag} N={len(P)} D={P.shape[1]} k={k} maxr={maxr} opts={opts}", flush=True)
    gi, gd, gv = kd.kd_knn_ex(tree, q, k, maxr, opts=opts, want_visited=visited)
    torch.cuda.synchronize()
    order = oracle_lib.build_tree(P)
    oi, od, ov = oracle_lib.knn(P, order, Qs, k, maxr)
    assert np.array_equal(gi.cpu().numpy().reshape(len(Qs), k), oi), tag
    assert np.array_equal(gd.cpu().numpy().reshape(len(Qs), k).view(np.uint32), od.view(np.uint32)), tag
    if visited:
        assert np.array_equal(gv.cpu().numpy().astype(np.int64), np.asarray(ov, np.int64)), tag
    tree.close()


@pytest.mark.parametrize("dim,levels", [(2, 1), (2, 8), (2, 12), (3, 1), (3, 7), (3, 10), (3, 12),
                                        (4, 3), (4, 9), (4, 11)])
def test_lds_levels_exact(oracle_lib, dim, levels):
    P = datagen.gmm(20000, dim, dim, n_centers=8, sigma=0.02)
    Qs = datagen.uniform(2000, dim, dim + 1)
    for k in (1, 8, 32):
        _check(oracle_lib, P, Qs, k, math.inf, dict(lds_levels=levels), f"L{levels}-k{k}")
    _check(oracle_lib, P, Qs, 8, 0.03, dict(lds_levels=levels), f"L{levels}-r0.03")


def test_lds_small_trees(oracle_lib):
    for n in (1, 2, 3, 5, 63, 64, 65, 1023, 1024, 1025):
        P = datagen.uniform(n, 3, n)
        Qs = datagen.uniform(200, 3, n + 1)
        _check(oracle_lib, P, Qs, 8, math.inf, dict(lds_levels=10), f"n{n}")


def test_lds_with_boxes_and_handoff(oracle_lib):
    P = datagen.gmm(20000, 3, 8, n_centers=16, sigma=0.004)
    Qs = np.concatenate([datagen.gmm(2000, 3, 9, n_centers=16, sigma=0.004), datagen.uniform(1000, 3, 10)])
    for opts in (dict(lds_levels=10, prune=2), dict(lds_levels=10, heavy_trips=16),
                 dict(lds_levels=12, prune=2, heavy_trips=16)):
        _check(oracle_lib, P, Qs, 8, math.inf, opts, "boxes/handoff", visited=False)


def test_lds_learned_path_ignores_option(oracle_lib):
    P = datagen.uniform(30000, 3, 1)
    Qs = datagen.uniform(3000, 3, 2)
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    order = oracle_lib.build_tree(P)
    oi, od, _ = oracle_lib.knn(P, order, Qs, 8)
    r = torch.full((len(Qs),), 0.02, dtype=torch.float32, device=_dev())
    gi, gd, _, _ = kd.kd_knn_with_radius(tree, r, q, 8, opts=dict(lds_levels=10))
    torch.cuda.synchronize()
    assert np.array_equal(gi.cpu().numpy(), oi)
    assert np.array_equal(gd.cpu().numpy().view(np.uint32), od.view(np.uint32))
    tree.close()


def test_lds_levels_rejected():
    P = datagen.uniform(1000, 4, 3)
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(datagen.uniform(10, 4, 4)).to(_dev())
    for bad in (13, 12):  # 13: too deep for any dim; 12: 128 KB of 32-byte records
        with pytest.raises(kd.KdError):
            kd.kd_knn_ex(tree, q, 8, opts=dict(lds_levels=bad))
    tree.close()


def test_lds_at_scale_equals_global():
    """uniform-1m k = 8: staging 10 and 12 levels gives the same output."""
    P, Qs = datagen.workload("uniform-1m")
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    ai, ad = kd.kd_knn(tree, q, 8)
    for L in (10, 12):
        bi, bd, _ = kd.kd_knn_ex(tree, q, 8, opts=dict(lds_levels=L))
        torch.cuda.synchronize()
        assert torch.equal(ai, bi) and torch.equal(ad.view(torch.int32), bd.view(torch.int32)), L
    tree.close()
