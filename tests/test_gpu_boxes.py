"""GPU parity of subtree bounding-box pruning (kd_opts.prune): on entering a
subtree the traversal leaves it at once when the bounding box of its points
is farther than the current k-th distance.  This prunes more than the paper's
split-plane rule but never a point of the result, so indices and squared
distances must equal the oracle's bit for bit under both rules: uniform and
clustered data, queries far outside the data, duplicated points (ties decided
by the smaller index), a finite radius, every list size, D = 2, 3, 4, the
learned-radius path and small trees.  The entered-node count under the box
rule is at most the paper's processed-node count."""
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


def _check(oracle_lib, P, Qs, k, maxr, tag, extra=None):
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    order = oracle_lib.build_tree(P)
    oi, od, ov = oracle_lib.knn(P, order, Qs, k, maxr)
    for prune in (1, 2):
        opts = dict(prune=prune, **(extra or {}))
        print(f"[gpu] boxes {tag} N={len(P)} Q={len(Qs)} k={k} maxr={maxr} opts={opts}", flush=True)
        gi, gd, _ = kd.kd_knn_ex(tree, q, k, maxr, opts=opts)
        torch.cuda.synchronize()
        gi = gi.cpu().numpy().reshape(len(Qs), k)
        gd = gd.cpu().numpy().reshape(len(Qs), k)
        assert np.array_equal(gi, oi), (tag, prune)
        assert np.array_equal(gd.view(np.uint32), od.view(np.uint32)), (tag, prune)
    # entered nodes: the paper's count under prune 1 (and by default when
    # the count is requested), never more under the box rule
    _, _, v1 = kd.kd_knn_ex(tree, q, k, maxr, want_visited=True)
    _, _, v2 = kd.kd_knn_ex(tree, q, k, maxr, want_visited=True, opts=dict(prune=2))
    torch.cuda.synchronize()
    v1 = v1.cpu().numpy().astype(np.int64)
    v2 = v2.cpu().numpy().astype(np.int64)
    assert np.array_equal(v1, np.asarray(ov, np.int64)), tag
    assert np.all(v2 <= v1), tag
    tree.close()
    return int(v1.sum()), int(v2.sum())


@pytest.mark.parametrize("k", [1, 2, 8, 13, 32, 64])
def test_boxes_uniform(oracle_lib, k):
    P = datagen.uniform(30000, 3, 1)
    Qs = datagen.uniform(4000, 3, 2)
    a, b = _check(oracle_lib, P, Qs, k, math.inf, f"uniform-k{k}")
    print(f"[gpu] uniform k={k} processed {a} entered with boxes {b}", flush=True)


@pytest.mark.parametrize("k", [1, 8, 16, 64])
def test_boxes_clustered_and_far_queries(oracle_lib, k):
    P = datagen.gmm(25000, 3, 3, n_centers=16, sigma=0.004)
    far = datagen.uniform(800, 3, 5) * 4.0 - 1.5  # mostly outside the data's box
    Qs = np.concatenate([datagen.gmm(2500, 3, 4, n_centers=16, sigma=0.004), datagen.uniform(1000, 3, 6), far])
    a, b = _check(oracle_lib, P, Qs.astype(np.float32), k, math.inf, f"gmm-k{k}")
    print(f"[gpu] gmm k={k} processed {a} entered with boxes {b}", flush=True)


@pytest.mark.parametrize("dim", [2, 3, 4])
def test_boxes_dims_and_radius(oracle_lib, dim):
    P = datagen.gmm(12000, dim, 6, n_centers=8, sigma=0.01)
    Qs = datagen.uniform(2500, dim, 7)
    for k in (1, 8):
        _check(oracle_lib, P, Qs, k, math.inf, f"dim{dim}-k{k}")
        _check(oracle_lib, P, Qs, k, 0.05, f"dim{dim}-k{k}-r0.05")
        _check(oracle_lib, P, Qs, k, 0.0, f"dim{dim}-k{k}-r0")


def test_boxes_duplicates_and_ties(oracle_lib):
    rng = np.random.default_rng(11)
    base = rng.integers(0, 6, size=(700, 3)).astype(np.float32)
    P = np.concatenate([base, base, base[:300], np.zeros((200, 3), np.float32)])
    Qs = rng.integers(-1, 7, size=(900, 3)).astype(np.float32) * 0.5
    for k in (1, 8, 64):
        _check(oracle_lib, P, Qs, k, math.inf, f"ties-k{k}")
        _check(oracle_lib, P, Qs, k, 1.0, f"ties-k{k}-r1")


def test_boxes_small_trees(oracle_lib):
    for n in (1, 2, 3, 5, 64, 127, 128, 129, 1500):
        P = datagen.uniform(n, 3, n)
        Qs = np.concatenate([datagen.uniform(300, 3, n + 1), datagen.uniform(50, 3, n + 2) * 3.0 - 1.0])
        _check(oracle_lib, P, Qs.astype(np.float32), 8, math.inf, f"n{n}")


def test_boxes_with_handoff_and_learned_radius(oracle_lib):
    """Box pruning combined with the cooperative hand-off and with injected
    initial radii (restarts from R2 included): identical to the oracle."""
    P = datagen.gmm(20000, 3, 8, n_centers=16, sigma=0.004)
    Qs = np.concatenate([datagen.gmm(2000, 3, 9, n_centers=16, sigma=0.004), datagen.uniform(1000, 3, 10)])
    _check(oracle_lib, P, Qs, 8, math.inf, "handoff", extra=dict(heavy_trips=16))
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    order = oracle_lib.build_tree(P)
    oi, od, _ = oracle_lib.knn(P, order, Qs, 8, math.inf)
    kth = np.sqrt(od[:, -1].astype(np.float64))
    rng = np.random.default_rng(3)
    r = (kth * rng.choice([0.5, 0.99, 1.0, 1.5], size=len(kth))).astype(np.float32)
    for prune in (1, 2):
        gi, gd, _, gf = kd.kd_knn_with_radius(tree, torch.from_numpy(r).to(_dev()), q, 8, want_flags=True,
                                              opts=dict(prune=prune))
        torch.cuda.synchronize()
        assert np.array_equal(gi.cpu().numpy(), oi), prune
        assert np.array_equal(gd.cpu().numpy().view(np.uint32), od.view(np.uint32)), prune
        assert int((gf.cpu().numpy() == 1).sum()) > 0
    tree.close()


def test_boxes_default_equals_planes_at_scale():
    """uniform-1m and gmm64-1m, k = 8: the default (boxes) equals the
    paper's rule, and enters fewer nodes."""
    for name in ("uniform-1m", "gmm64-1m"):
        P, Qs = datagen.workload(name)
        tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
        q = torch.from_numpy(Qs).to(_dev())
        print(f"[gpu] boxes at scale {name}", flush=True)
        ai, ad = kd.kd_knn(tree, q, 8)
        bi, bd, bv = kd.kd_knn_ex(tree, q, 8, opts=dict(prune=1), want_visited=True)
        _, _, cv = kd.kd_knn_ex(tree, q, 8, opts=dict(prune=2), want_visited=True)
        torch.cuda.synchronize()
        assert torch.equal(ai, bi) and torch.equal(ad.view(torch.int32), bd.view(torch.int32)), name
        nb, nc = int(bv.to(torch.int64).sum()), int(cv.to(torch.int64).sum())
        print(f"[gpu] {name}: processed (paper) {nb / len(Qs):.1f}/query, entered with boxes {nc / len(Qs):.1f}/query",
              flush=True)
        assert nc < nb
        tree.close()
