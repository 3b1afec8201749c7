"""Full-size GPU parity on the large workloads, checked on sampled queries
against the oracle's brute force (the plain definition), and learned vs plain
byte-identical over every query.

* clustered 10M: 256-cluster mixture, sigma log-uniform [0.002, 0.05], 10M
  points and 10M queries (90 % mixture, 10 % uniform), kNN k = 16.
* shells: points on 1000 random sphere shells (radius 0.01-0.1, radial noise
  1e-4), queries near the shells, kNN k = 32 with maxRadius = 0.005 (a
  10M-point instance of the 100M surface-like workload)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2210_12859_amd as kd  # noqa: E402
from paper_2210_12859_amd import datagen  # noqa: E402


def _dev():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda:0")


def _sample_check(oracle_lib, P, Qs, gi, gd, k, maxr, n=400, seed=0):
    rows = np.random.default_rng(seed).choice(len(Qs), n, replace=False)
    bi, bd = oracle_lib.brute(P, Qs[rows], k, maxr)
    assert np.array_equal(gi[rows], bi)
    assert np.array_equal(gd[rows].view(np.uint32), bd.view(np.uint32))


def test_clustered_10m_plain_and_learned(oracle_lib):
    P, Qs = datagen.workload("clustered-10m")
    print("[gpu] clustered-10m: build", flush=True)
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    k = 16
    gi, gd = kd.kd_knn(tree, q, k)
    torch.cuda.synchronize()
    gi_np, gd_np = gi.cpu().numpy(), gd.cpu().numpy()
    _sample_check(oracle_lib, P, Qs, gi_np, gd_np, k, np.inf)
    print("[gpu] clustered-10m: train", flush=True)
    train = torch.from_numpy(datagen.clustered_lr_queries(1 << 20, seed=2)).to(_dev())
    model = kd.kd_radius_model_train(tree, train, k, epochs=4, batch=8192, seed=0)
    li, ld, lv, st = kd.kd_knn_learned(tree, model, q, k, want_stats=True)
    torch.cuda.synchronize()
    print(f"[gpu] clustered-10m learned fallbacks {st['fallbacks']}", flush=True)
    assert torch.equal(li, gi)
    assert torch.equal(ld.view(torch.int32), gd.view(torch.int32))


def test_shells_10m_bounded_k32(oracle_lib):
    n = 10_000_000
    P = datagen.shells(n, seed=0)
    Qs = datagen.shells(2_000_000, seed=1)
    print("[gpu] shells-10m: build", flush=True)
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    q = torch.from_numpy(Qs).to(_dev())
    gi, gd = kd.kd_knn(tree, q, 32, 0.005)
    torch.cuda.synchronize()
    gi_np, gd_np = gi.cpu().numpy(), gd.cpu().numpy()
    _sample_check(oracle_lib, P, Qs, gi_np, gd_np, 32, 0.005, n=300)
    # within the radius only
    R2 = oracle_lib.sq_radius(0.005)
    assert (gd_np[gi_np >= 0] <= R2).all()
