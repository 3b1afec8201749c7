"""GPU parity of the plain traversal against the CPU oracle, through the C ABI.

Bar: result indices byte-identical, squared distances bit-identical, and the
per-query count of processed nodes equal to the recursive oracle's (the paper's
Sec. 3.1 claim that the stack-free loop processes the same nodes)."""
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


def gpu_knn(tree, Qs, k, maxr=math.inf, opts=None, want_visited=True):
    q = torch.from_numpy(np.ascontiguousarray(Qs, np.float32)).to(_dev())
    oi, od, vis = kd.kd_knn_ex(tree, q, k, maxr, want_visited=want_visited, opts=opts)
    torch.cuda.synchronize()
    Q = Qs.shape[0]
    return (oi.cpu().numpy().reshape(Q, k), od.cpu().numpy().reshape(Q, k),
            None if vis is None else vis.cpu().numpy().astype(np.int64))


def build(P):
    print(f"[gpu] build N={P.shape[0]} D={P.shape[1]}", flush=True)
    return kd.kd_build(torch.from_numpy(np.ascontiguousarray(P)).to(_dev()))


def assert_same(gi, gd, gv, oi, od, ov, ctx=""):
    bad = np.nonzero((gi != oi).any(axis=1))[0]
    assert len(bad) == 0, f"{ctx}: idx differ at {bad[:5]} gpu={gi[bad[:1]]} oracle={oi[bad[:1]]}"
    assert np.array_equal(gd.view(np.uint32), od.view(np.uint32)), f"{ctx}: d2 bits differ"
    if gv is not None and ov is not None:
        vb = np.nonzero(gv != ov)[0]
        assert len(vb) == 0, f"{ctx}: visited differ at {vb[:5]} gpu={gv[vb[:3]]} oracle={ov[vb[:3]]}"


# ------------------------------------------------------------ small config

@pytest.fixture(scope="module")
def c1(oracle_lib):
    P, Qs = datagen.workload("uniform-16k")
    tree = build(P)
    return P, Qs, tree, oracle_lib.build_tree(P)


def test_c1_tree_equals_oracle(c1):
    P, Qs, tree, order = c1
    assert np.array_equal(tree.order(), order)


@pytest.mark.parametrize("k", [1, 8])
def test_c1_exact(c1, oracle_lib, k):
    P, Qs, tree, order = c1
    print(f"[gpu] c1 k={k}", flush=True)
    gi, gd, gv = gpu_knn(tree, Qs, k)
    oi, od, ov = oracle_lib.knn(P, order, Qs, k)
    assert_same(gi, gd, gv, oi, od, ov, f"c1 k={k}")


def test_c1_fcp_entry(c1, oracle_lib):
    P, Qs, tree, order = c1
    q = torch.from_numpy(Qs).to(_dev())
    oi, od = kd.kd_fcp(tree, q)
    torch.cuda.synchronize()
    ri, rd, _ = oracle_lib.knn(P, order, Qs, 1)
    assert np.array_equal(oi.cpu().numpy(), ri[:, 0])
    assert np.array_equal(od.cpu().numpy().view(np.uint32), rd[:, 0].view(np.uint32))


def test_c1_knn_entry_without_d2(c1, oracle_lib):
    P, Qs, tree, order = c1
    q = torch.from_numpy(Qs).to(_dev())
    oi, od = kd.kd_knn(tree, q, 8, want_d2=False)
    torch.cuda.synchronize()
    assert od is None
    ri, _, _ = oracle_lib.knn(P, order, Qs, 8)
    assert np.array_equal(oi.cpu().numpy(), ri)


@pytest.mark.parametrize("opts", [
    dict(block=64), dict(block=128), dict(block=256), dict(block=512), dict(block=1024),
    dict(block=64, waves_per_cu=2), dict(block=256, waves_per_cu=32), dict(block=1024, waves_per_cu=32),
    dict(sort_bits=0), dict(sort_bits=1), dict(sort_bits=8), dict(sort_bits=12), dict(sort_bits=14),
    dict(sort_bits=15), dict(sort_bits=16), dict(sort_bits=24), dict(sort_bits=32),
    dict(lds_levels=1), dict(lds_levels=6), dict(lds_levels=10), dict(lds_levels=12),
    dict(lds_levels=10, block=1024, waves_per_cu=32),
])
def test_c1_all_launch_options_identical(c1, oracle_lib, opts):
    P, Qs, tree, order = c1
    print(f"[gpu] c1 opts={opts}", flush=True)
    gi, gd, gv = gpu_knn(tree, Qs, 8, opts=opts)
    oi, od, ov = oracle_lib.knn(P, order, Qs, 8)
    assert_same(gi, gd, gv, oi, od, ov, f"opts {opts}")


# --------------------------------------------------------- random small

CASES = []
for N in [1, 2, 3, 7, 64, 65, 1000, 4097]:
    for D in [2, 3, 4]:
        CASES.append((N, D))


@pytest.mark.parametrize("N,D", CASES)
def test_random_small_all_k(oracle_lib, N, D):
    rng = np.random.default_rng(N * 10 + D)
    P = rng.random((N, D), dtype=np.float32)
    Qs = rng.random((300, D), dtype=np.float32)
    tree = build(P)
    order = oracle_lib.build_tree(P)
    for k in [1, 2, 3, 5, 8, 13, 16, 32, 33, 64]:
        for maxr in [0.0, 0.02, 0.2, math.inf]:
            gi, gd, gv = gpu_knn(tree, Qs, k, maxr)
            oi, od, ov = oracle_lib.knn(P, order, Qs, k, maxr)
            assert_same(gi, gd, gv, oi, od, ov, f"N={N} D={D} k={k} maxr={maxr}")


@pytest.mark.parametrize("D", [2, 3, 4])
def test_integer_grid_ties(oracle_lib, D):
    rng = np.random.default_rng(40 + D)
    P = rng.integers(0, 6, size=(3000, D)).astype(np.float32)
    Qs = rng.integers(0, 6, size=(500, D)).astype(np.float32)
    Qs[1::2] += 0.5
    tree = build(P)
    order = oracle_lib.build_tree(P)
    for k in [1, 4, 8, 32, 64]:
        for maxr in [0.0, 1.0, 1.5, math.inf]:
            gi, gd, gv = gpu_knn(tree, Qs, k, maxr)
            oi, od, ov = oracle_lib.knn(P, order, Qs, k, maxr)
            assert_same(gi, gd, gv, oi, od, ov, f"grid D={D} k={k} maxr={maxr}")


def test_edge_cases(oracle_lib):
    # empty tree: all -1 / +inf, nothing traversed
    tree0 = kd.kd_build(torch.zeros((0, 3), dtype=torch.float32, device=_dev()))
    Qs = np.random.default_rng(1).random((100, 3), dtype=np.float32)
    gi, gd, gv = gpu_knn(tree0, Qs, 8)
    assert (gi == -1).all() and np.isinf(gd).all() and (gv == 0).all()
    # zero queries
    P = np.random.default_rng(2).random((50, 3), dtype=np.float32)
    tree = build(P)
    gi, gd, gv = gpu_knn(tree, np.zeros((0, 3), np.float32), 4)
    assert gi.shape == (0, 4)
    # NaN query coordinates give empty rows; the rest are unaffected
    Qs = np.random.default_rng(3).random((70, 3), dtype=np.float32)
    Qs[5, 0] = np.nan
    Qs[9, 2] = np.nan
    order = oracle_lib.build_tree(P)
    gi, gd, gv = gpu_knn(tree, Qs, 4)
    oi, od, ov = oracle_lib.knn(P, order, Qs, 4)
    assert_same(gi, gd, gv, oi, od, ov, "nan queries")
    assert (gi[5] == -1).all() and (gi[9] == -1).all()
    # maximum k on a tree smaller than k
    gi, gd, gv = gpu_knn(tree, Qs[:10], 64)
    oi, od, ov = oracle_lib.knn(P, order, Qs[:10], 64)
    assert_same(gi, gd, gv, oi, od, ov, "k=64 > N")


def test_run_twice_identical(c1):
    P, Qs, tree, order = c1
    a = gpu_knn(tree, Qs, 8)
    b = gpu_knn(tree, Qs, 8)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


# ------------------------------------------------------------ full scale

@pytest.mark.parametrize("wl", ["uniform-1m", "gmm64-1m"])
def test_c2_full_scale(oracle_lib, wl):
    P, Qs = datagen.workload(wl)
    tree = build(P)
    order = oracle_lib.build_tree(P)
    assert np.array_equal(tree.order(), order)
    for k in [1, 8, 64]:
        print(f"[gpu] {wl} k={k}", flush=True)
        sub = Qs if k < 64 else Qs[: 1 << 18]
        gi, gd, gv = gpu_knn(tree, Qs, k)
        oi, od, ov = oracle_lib.knn(P, order, sub, k)
        n = sub.shape[0]
        assert_same(gi[:n], gd[:n], gv[:n], oi, od, ov, f"{wl} k={k}")
        # the rest of the rows: sampled brute force
        rest = np.arange(n, Qs.shape[0], 997)
        if len(rest):
            bi, bd = oracle_lib.brute(P, Qs[rest], k)
            assert np.array_equal(gi[rest], bi) and np.array_equal(gd[rest].view(np.uint32), bd.view(np.uint32))


def test_autotune_choice_gives_identical_results(c1, oracle_lib, tmp_path):
    P, Qs, tree, order = c1
    q = torch.from_numpy(Qs).to(_dev())
    opts, ms = kd.kd_autotune(tree, q, 8)
    print(f"[gpu] autotune k=8: {opts} {ms:.3f} ms", flush=True)
    assert ms > 0 and opts["block"] in (256, 512, 1024)
    assert kd.kd_tree_get_tuned(tree, 8) == opts
    gi, gd, gv = gpu_knn(tree, Qs, 8)  # default options now resolve to the tuned ones
    oi, od, ov = oracle_lib.knn(P, order, Qs, 8)
    assert_same(gi, gd, gv, oi, od, ov, "tuned")
    path = str(tmp_path / "tune.json")
    kd.save_tuning(tree, [8], path)
    tree2 = build(P)
    kd.load_tuning(tree2, path)
    assert kd.kd_tree_get_tuned(tree2, 8) == opts
    with pytest.raises(kd.KdError):
        kd.kd_tree_get_tuned(tree2, 1)
