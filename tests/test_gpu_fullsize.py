"""GPU parity at the full size of the batched workload, in the launch
configuration the library uses by default, checked on 200 sampled queries per
tree against the oracle's brute force (the plain definition): 512 trees, N
log-uniform in [1K, 2M] (sum about 135M points), D in {2, 3, 4}, uniform or
64-cluster Gaussian, k in {1, 8, 32}, Q = N, one captured launch pipeline.
(The surface-like 100M workload is checked in test_gpu_timed_configs.)"""
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
        # 200 sampled queries per job for the check
        rows = np.random.default_rng(t).choice(Q, min(Q, 200), replace=False)
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
