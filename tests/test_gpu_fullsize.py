"""GPU parity at the full sizes of the batched and the surface-like
workloads, in the launch configuration the library uses by default, checked
on sampled queries against the oracle's brute force (the plain definition).

* batched: 512 trees, N log-uniform in [1K, 2M] (sum about 135M points),
  D in {2, 3, 4}, uniform or 64-cluster Gaussian, k in {1, 8, 32}, Q = N,
  one captured launch pipeline;
* surface-like: 100M points on 1000 sphere shells (radius 0.01-0.1, radial
  noise 1e-4), 100M queries near the shells, kNN k = 32 within maxRadius
  0.005."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2210_12859_amd as kd  # noqa: E402
from paper_2210_12859_amd import datagen  # noqa: E402


def _dev():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda:0")


def test_batched_512_trees_full_size(oracle_lib):
    meta = datagen.batched_jobs(512, seed=42)
    print(f"[gpu] batched-512: sum N = {sum(m['n'] for m in meta)}", flush=True)
    jobs, host = [], []
    for t, m in enumerate(meta):
        P, Qs = datagen.job_arrays(m)
        tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
        q = torch.from_numpy(Qs).to(_dev())
        Q, k = len(Qs), m["k"]
        jobs.append(dict(tree=tree, queries=q, k=k, out_idx=torch.empty((Q, k), dtype=torch.int32, device=_dev()),
                         out_d2=torch.empty((Q, k), dtype=torch.float32, device=_dev())))
        # keep a few sampled queries per job for the check
        rows = np.random.default_rng(t).choice(Q, min(Q, 3), replace=False)
        host.append((P, Qs[rows], rows))
        if t % 64 == 63:
            print(f"[gpu] batched-512: {t + 1} trees built", flush=True)
    batch = kd.Batch(jobs)
    batch.run()
    torch.cuda.synchronize()
    print("[gpu] batched-512: checking samples", flush=True)
    for j, (P, qs, rows) in zip(jobs, host):
        bi, bd = oracle_lib.brute(P, qs, j["k"])
        r = torch.from_numpy(rows).to(_dev())
        gi = j["out_idx"][r].cpu().numpy()
        gd = j["out_d2"][r].cpu().numpy()
        assert np.array_equal(gi, bi)
        assert np.array_equal(gd.view(np.uint32), bd.view(np.uint32))
    batch.close()
    for j in jobs:
        j["tree"].close()


def test_shells_100m_bounded_k32(oracle_lib):
    n = 100_000_000
    print("[gpu] shells-100m: generating", flush=True)
    P = datagen.shells(n, seed=0)
    print("[gpu] shells-100m: build", flush=True)
    tree = kd.kd_build(torch.from_numpy(P).to(_dev()))
    Qs = datagen.shells(n, seed=1)
    q = torch.from_numpy(Qs).to(_dev())
    print("[gpu] shells-100m: query", flush=True)
    gi, gd = kd.kd_knn(tree, q, 32, 0.005)
    torch.cuda.synchronize()
    rows = np.random.default_rng(0).choice(n, 64, replace=False)
    print("[gpu] shells-100m: brute-force check of 64 queries", flush=True)
    bi, bd = oracle_lib.brute(P, Qs[rows], 32, 0.005)
    r = torch.from_numpy(rows).to(_dev())
    assert np.array_equal(gi[r].cpu().numpy(), bi)
    assert np.array_equal(gd[r].cpu().numpy().view(np.uint32), bd.view(np.uint32))
    # every query: found points within the radius, empty slots (-1, +inf)
    R2 = float(oracle_lib.sq_radius(0.005))
    assert not bool(((gi >= 0) & (gd > R2)).any())
    assert not bool(((gi < 0) & ~torch.isinf(gd)).any())
    tree.close()
