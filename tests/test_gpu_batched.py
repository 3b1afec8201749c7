"""GPU tests of the batched path: many trees of mixed dimension, size and k in
one captured pipeline; every job must equal the oracle (and kd_knn) exactly,
and every graph replay must equal the eager result."""
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


def _t(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).to(_dev())


def _mixed_jobs(seed=0):
    rng = np.random.default_rng(seed)
    specs = []
    for i, (N, D, k, Q, maxr) in enumerate([
        (5000, 3, 8, 3000, math.inf), (0, 3, 8, 100, math.inf), (1, 2, 1, 50, math.inf), (100, 4, 32, 200, math.inf),
        (30000, 2, 8, 4000, 0.01), (7000, 4, 1, 2500, math.inf), (2000, 3, 5, 0, math.inf), (12345, 3, 32, 3000, 0.05),
        (64, 2, 64, 100, math.inf), (20000, 3, 1, 5000, math.inf), (3000, 4, 8, 1000, 0.2), (999, 2, 3, 999, math.inf),
    ]):
        P = rng.random((N, D), dtype=np.float32)
        Qs = rng.random((Q, D), dtype=np.float32)
        if i == 3:
            P = rng.integers(0, 3, size=(N, D)).astype(np.float32)
            Qs = rng.integers(0, 3, size=(Q, D)).astype(np.float32)
        specs.append((P, Qs, k, maxr))
    return specs


def _make_jobs(specs):
    jobs, trees = [], []
    for P, Qs, k, maxr in specs:
        tree = kd.kd_build(_t(P))
        trees.append(tree)
        Q = Qs.shape[0]
        jobs.append(dict(tree=tree, queries=_t(Qs), k=k, max_radius=maxr,
                         out_idx=torch.full((Q, k), -7, dtype=torch.int32, device=_dev()),
                         out_d2=torch.zeros((Q, k), dtype=torch.float32, device=_dev())))
    return jobs, trees


def _check_against_oracle(oracle_lib, specs, jobs):
    for (P, Qs, k, maxr), j in zip(specs, jobs):
        gi = j["out_idx"].cpu().numpy()
        gd = j["out_d2"].cpu().numpy()
        if len(P) == 0:
            assert (gi == -1).all() and np.isinf(gd).all()
            continue
        order = oracle_lib.build_tree(P)
        oi, od, _ = oracle_lib.knn(P, order, Qs, k, maxr)
        assert np.array_equal(gi, oi), (P.shape, k, maxr)
        assert np.array_equal(gd.view(np.uint32), od.view(np.uint32))


@pytest.mark.parametrize("sort_bits", [0, 16, 32])
def test_batched_mixed_jobs_exact(oracle_lib, sort_bits):
    specs = _mixed_jobs(1)
    jobs, trees = _make_jobs(specs)
    print(f"[gpu] batched mixed sort_bits={sort_bits}", flush=True)
    kd.kd_knn_batched(jobs, opts=dict(sort_bits=sort_bits))
    torch.cuda.synchronize()
    _check_against_oracle(oracle_lib, specs, jobs)


def test_batched_graph_replays_match_eager(oracle_lib):
    specs = _mixed_jobs(2)
    jobs, trees = _make_jobs(specs)
    kd.kd_knn_batched(jobs)
    torch.cuda.synchronize()
    eager = [(j["out_idx"].clone(), j["out_d2"].clone()) for j in jobs]
    _check_against_oracle(oracle_lib, specs, jobs)
    b = kd.Batch(jobs)
    for rep in range(4):
        for j in jobs:
            j["out_idx"].fill_(-5)
            j["out_d2"].zero_()
        torch.cuda.synchronize()
        # some eager work between replays
        x = torch.randn(1 << 20, device=_dev())
        _ = (x * 2).sum().item()
        b.run()
        torch.cuda.synchronize()
        for j, (ei, ed) in zip(jobs, eager):
            assert torch.equal(j["out_idx"], ei), rep
            assert torch.equal(j["out_d2"].view(torch.int32), ed.view(torch.int32)), rep
    b.close()


def test_batched_generated_jobs_equal_single_calls(oracle_lib):
    meta = datagen.batched_jobs(n_jobs=48, seed=42, n_max=60000)
    jobs, trees, singles = [], [], []
    for m in meta:
        P, Qs = datagen.job_arrays(m)
        tree = kd.kd_build(_t(P))
        trees.append(tree)
        q = _t(Qs)
        k = m["k"]
        jobs.append(dict(tree=tree, queries=q, k=k, out_idx=torch.empty((len(Qs), k), dtype=torch.int32, device=_dev()),
                         out_d2=torch.empty((len(Qs), k), dtype=torch.float32, device=_dev())))
        si, sd = kd.kd_knn(tree, q, k)
        singles.append((si.reshape(len(Qs), k), sd.reshape(len(Qs), k)))
    print(f"[gpu] batched generated jobs: {sum(m['n'] for m in meta)} queries", flush=True)
    kd.kd_knn_batched(jobs)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    for m, j, (si, sd) in zip(meta, jobs, singles):
        assert torch.equal(j["out_idx"], si)
        assert torch.equal(j["out_d2"].view(torch.int32), sd.view(torch.int32))
    # spot-check a few jobs against brute force
    for t in rng.choice(len(meta), 4, replace=False):
        P, Qs = datagen.job_arrays(meta[t])
        rows = rng.choice(len(Qs), 50, replace=False)
        bi, bd = oracle_lib.brute(P, Qs[rows], meta[t]["k"])
        assert np.array_equal(jobs[t]["out_idx"].cpu().numpy()[rows], bi)


def _clustered_specs(seed=5):
    """3-D and 2-D jobs with tight clusters and far-off queries (long chains),
    plus a 4-D job, mixed k."""
    rng = np.random.default_rng(seed)
    specs = []
    for N, D, k in [(40000, 3, 8), (25000, 3, 1), (30000, 2, 8), (20000, 4, 32), (15000, 3, 16)]:
        c = rng.random((16, D))
        P = (c[rng.integers(0, 16, N)] + 0.003 * rng.standard_normal((N, D))).astype(np.float32)
        Qs = np.concatenate([(c[rng.integers(0, 16, 3000)] + 0.003 * rng.standard_normal((3000, D))),
                             rng.random((1000, D))]).astype(np.float32)
        specs.append((P, Qs, k, math.inf))
    return specs


@pytest.mark.parametrize("heavy", [4, 64, -1])
def test_batched_handoff_exact(oracle_lib, heavy):
    """Trip budgets that hand most long queries to the cooperative kernel:
    every job equals the oracle, under both pruning rules."""
    specs = _clustered_specs()
    jobs, trees = _make_jobs(specs)
    for prune in (1, 2):
        print(f"[gpu] batched hand-off heavy_trips={heavy} prune={prune}", flush=True)
        kd.kd_knn_batched(jobs, opts=dict(heavy_trips=heavy, prune=prune))
        torch.cuda.synchronize()
        _check_against_oracle(oracle_lib, specs, jobs)


def test_batched_learned_exact(oracle_lib):
    """3-D jobs start from a radius model: a model trained on one of the
    trees serves as the call's model, another job carries its own, and a
    model from an unrelated tree is used for a third; every job equals the
    oracle and the single-tree learned call."""
    specs = _clustered_specs(7)
    jobs, trees = _make_jobs(specs)
    P0, Q0, k0, _ = specs[0]
    train0 = _t(datagen.gmm(1 << 16, 3, 11, n_centers=16, sigma=0.003))
    m_call = kd.kd_radius_model_train(trees[0], train0, k0, epochs=3)
    m_own = kd.kd_radius_model_train(trees[4], _t(specs[4][1]), specs[4][2], epochs=2)
    u = datagen.uniform(20000, 3, 3)
    tu = kd.kd_build(_t(u))
    m_other = kd.kd_radius_model_train(tu, _t(datagen.uniform(1 << 14, 3, 4)), 1, epochs=2)
    jobs[4]["model"] = m_own
    jobs[1]["model"] = m_other
    for heavy in (0, 8):
        print(f"[gpu] batched learned heavy_trips={heavy}", flush=True)
        for j in jobs:
            j["out_idx"].fill_(-9)
        kd.kd_knn_batched(jobs, model=m_call, opts=dict(heavy_trips=heavy))
        torch.cuda.synchronize()
        _check_against_oracle(oracle_lib, specs, jobs)
    # the graph path (create once, replay) with the learned radii
    b = kd.Batch(jobs, model=m_call)
    for j in jobs:
        j["out_idx"].fill_(-9)
    b.run()
    torch.cuda.synchronize()
    _check_against_oracle(oracle_lib, specs, jobs)
    b.close()
    li, ld, _, _ = kd.kd_knn_learned(trees[0], m_call, jobs[0]["queries"], k0)
    torch.cuda.synchronize()
    assert torch.equal(li.reshape(jobs[0]["out_idx"].shape), jobs[0]["out_idx"])
    for m in (m_call, m_own, m_other):
        m.close()


def test_batched_autotune_keeps_results(oracle_lib):
    specs = _mixed_jobs(3)
    jobs, trees = _make_jobs(specs)
    b = kd.Batch(jobs)
    groups = b.info()
    print(f"[gpu] batched autotune over {len(groups)} groups", flush=True)
    chosen = b.autotune(reps=1)
    assert len(chosen) == len(groups)
    for o in chosen:
        assert o["block"] in (256, 512) and o["waves_per_cu"] in (16, 24, 32) and o["sort_bits"] in (16, 24, 32)
    for j in jobs:
        j["out_idx"].fill_(-3)
    b.run()
    torch.cuda.synchronize()
    _check_against_oracle(oracle_lib, specs, jobs)
    b.close()
