"""GPU tests of the learned initial radius: exactness of the restart rule for
any radius (results byte-identical to the plain traversal and to the oracle,
fallback set equal to the oracle's), the MLP kernels against the float64
reference, on-GPU training, and what the trained network gains."""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2210_12859_amd as kd  # noqa: E402
from paper_2210_12859_amd import datagen  # noqa: E402
from oracle import mlp_ref as M  # noqa: E402
from tests import mlp_bounds as MB  # noqa: E402


def _dev():
    assert torch.cuda.is_available(), "GPU test run without a GPU"
    return torch.device("cuda:0")


def _t(a, dtype=np.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).to(_dev())


@pytest.fixture(scope="module")
def c1(oracle_lib):
    P, Qs = datagen.workload("uniform-16k")
    tree = kd.kd_build(_t(P))
    return P, Qs, tree, oracle_lib.build_tree(P)


def _radii(Qs, pd, rng):
    kth = np.sqrt(pd[:, -1].astype(np.float64))
    n = len(Qs)
    return {
        "zero": np.zeros(n), "tiny": np.full(n, 1e-30), "negative": np.full(n, -1.0),
        "nan": np.full(n, np.nan), "inf": np.full(n, np.inf), "random": rng.random(n) * 0.05,
        "perfect": kth * (1 + 2.0 ** -20), "under": kth * 0.9, "mixed": np.where(rng.random(n) < 0.5, kth, 0.0),
    }


@pytest.mark.parametrize("k,maxr", [(1, math.inf), (8, math.inf), (8, 0.03), (13, math.inf), (64, math.inf)])
def test_injected_radius_is_exact(c1, oracle_lib, k, maxr):
    P, Qs, tree, order = c1
    pi, pd, pv = oracle_lib.knn(P, order, Qs, k, maxr)
    rng = np.random.default_rng(k)
    for name, r0 in _radii(Qs, pd, rng).items():
        r0 = r0.astype(np.float32)
        print(f"[gpu] injected radius {name} k={k} maxr={maxr}", flush=True)
        gi, gd, gv, gf = kd.kd_knn_with_radius(tree, _t(r0), _t(Qs), k, maxr, want_visited=True, want_flags=True)
        torch.cuda.synchronize()
        gi = gi.cpu().numpy().reshape(-1, k)
        gd = gd.cpu().numpy().reshape(-1, k)
        assert np.array_equal(gi, pi), name
        assert np.array_equal(gd.view(np.uint32), pd.view(np.uint32)), name
        li, ld, lv, lfb = oracle_lib.knn_learned(P, order, Qs, k, r0, maxr)
        assert np.array_equal(gf.cpu().numpy().astype(bool), lfb), name


def test_mlp_forward_matches_reference():
    """y of the inference kernel inside its rigorous enclosure around the
    float64 reference: float32 accumulation bound per layer, bfloat16 rounding
    flips allowed only where the accumulation error reaches a rounding
    boundary (tests/mlp_bounds.py)."""
    rng = np.random.default_rng(3)
    theta = (M.he_init(11) + 0.05 * rng.standard_normal(M.NPARAM)).astype(np.float32)
    lo = np.array([0.1, -0.2, 0.0], np.float32)
    inv = np.array([1.0, 0.5, 2.0], np.float32)
    model = kd.kd_model_create(theta, lo, inv, 0.0, 8)
    q = rng.random((5000, 3), dtype=np.float32)
    y = kd.kd_mlp_predict(model, _t(q)).cpu().numpy().astype(np.float64)
    ok, e = MB.check_forward(theta.astype(np.float64), M.normalize(q, lo, inv), y)
    yc, yr = e["y"]
    rel = np.abs(y - yc) / (1 + np.abs(yc))
    print(f"[gpu] forward: outside {int((~ok).sum())}, err rel median {np.median(rel):.2e} max {rel.max():.2e}, "
          f"queries with a possible flip {e['flips'].mean():.3f}", flush=True)
    assert ok.all(), np.flatnonzero(~ok)[:10]


def test_mlp_gradient_matches_reference():
    """Loss and every gradient element of the training kernels inside their
    rigorous enclosures (float32 accumulation over the batch, possible
    bfloat16 and ReLU-mask flips propagated)."""
    rng = np.random.default_rng(4)
    theta = (M.he_init(12) + 0.05 * rng.standard_normal(M.NPARAM)).astype(np.float32)
    lo = np.zeros(3, np.float32)
    inv = np.ones(3, np.float32)
    model = kd.kd_model_create(theta, lo, inv, 0.0, 8)
    for n in (1000, 64, 100):
        q = rng.random((n, 3), dtype=np.float32)
        t = (rng.standard_normal(n) * 0.3 - 4.0).astype(np.float32)
        loss, g = kd.kd_mlp_grad(model, _t(q), _t(t))
        lok, gok, (lc, lr, gc, gr, _) = MB.check_gradient(theta.astype(np.float64), M.normalize(q, lo, inv),
                                                          t.astype(np.float64), loss, g)
        rel = np.abs(g - gc) / np.maximum(np.abs(gc), 1e-30)
        print(f"[gpu] grad n={n}: outside {int((~gok).sum())}, median rel err {np.median(rel):.2e}, "
              f"median bound/|g| {np.median(gr / np.maximum(np.abs(gc), 1e-30)):.2e}", flush=True)
        assert lok, (loss, lc, lr)
        assert gok.all(), np.flatnonzero(~gok)[:10]


def test_adam_step_matches_reference():
    """The trainer's Adam update on the GPU (float32 master weights and
    moments) against the oracle's Adam step applied to the gradient the GPU
    used, over several consecutive steps, at the float32 evaluation bound."""
    rng = np.random.default_rng(8)
    theta = (M.he_init(15) + 0.05 * rng.standard_normal(M.NPARAM)).astype(np.float32)
    lo = np.zeros(3, np.float32)
    inv = np.ones(3, np.float32)
    model = kd.kd_model_create(theta, lo, inv, 0.0, 8)
    m = np.zeros(M.NPARAM, np.float32)
    v = np.zeros(M.NPARAM, np.float32)
    f = np.float32
    b1, b2, eps = float(f(0.9)), float(f(0.999)), float(f(1e-8))
    lr = float(f(3e-3))
    th = theta.copy()
    for step in range(1, 6):
        q = rng.random((512, 3), dtype=np.float32)
        t = (rng.standard_normal(512) * 0.3 - 4.0).astype(np.float32)
        m0, v0 = m.copy(), v.copy()
        loss, g = kd.kd_mlp_train_step(model, _t(q), _t(t), step, lr, m, v)
        th_gpu = model.params()[0]
        (rt, rm, rv), (bt, bm, bv) = MB.adam_bounds(th.astype(np.float64), m0.astype(np.float64),
                                                     v0.astype(np.float64), g.astype(np.float64), step, lr, b1, b2,
                                                     eps)
        for name, got, ref, bound in (("m", m, rm, bm), ("v", v, rv, bv), ("theta", th_gpu, rt, bt)):
            out = np.abs(got.astype(np.float64) - ref) > bound
            print(f"[gpu] adam step {step} {name}: outside {int(out.sum())}, max err "
                  f"{np.max(np.abs(got - ref)):.2e}", flush=True)
            assert not out.any(), (step, name, np.flatnonzero(out)[:10])
        assert not np.array_equal(th_gpu, th)
        th = th_gpu.copy()
    model.close()


def test_worst0_matches_reference():
    """The learned path's initial squared radius, read back in caller order:
    (a) the kernel's y -> worst0 step against the oracle's on the same y, to
    a few float32 ulp (exp of a rounded argument); (b) the whole prediction
    against the oracle's within the forward enclosure; (c) the min with R2
    exact."""
    rng = np.random.default_rng(9)
    theta = (M.he_init(16) + 0.05 * rng.standard_normal(M.NPARAM)).astype(np.float32)
    lo = np.array([0.0, 0.1, -0.1], np.float32)
    inv = np.array([1.0, 0.9, 1.1], np.float32)
    q = rng.random((4000, 3), dtype=np.float32)
    u = 2.0 ** -24
    for margin, maxr in ((0.0, math.inf), (0.7, math.inf), (-1.5, math.inf), (0.0, 0.02), (30.0, 0.5)):
        model = kd.kd_model_create(theta, lo, inv, margin, 8)
        R2 = np.float32(np.float32(maxr) * np.float32(maxr))
        w = kd.kd_mlp_worst0(model, _t(q), maxr).cpu().numpy()
        y = kd.kd_mlp_predict(model, _t(q)).cpu().numpy().astype(np.float64)
        model.close()
        # (a) the step on the kernel's own y
        wr = M.worst0_from_y(y, margin, R2).astype(np.float64)
        eps = 2 * u * (np.abs(y) + abs(margin)) + 16 * u
        assert (np.abs(w - wr) <= eps * wr).all(), (margin, maxr)
        # (b) the whole prediction: worst0 is monotone in y
        ok, e = MB.check_forward(theta.astype(np.float64), M.normalize(q, lo, inv), y)
        assert ok.all()
        yc, yr = e["y"]
        wlo = M.worst0_from_y(yc - yr, margin, R2) * (1 - eps)
        whi = M.worst0_from_y(yc + yr, margin, R2) * (1 + eps)
        assert ((w >= wlo) & (w <= whi)).all(), (margin, maxr)
        # (c) never above R2, equal to it where the radius is capped
        assert (w <= R2).all()
        print(f"[gpu] worst0 margin {margin} maxr {maxr}: capped {int((w == R2).sum())}, max rel err "
              f"{np.max(np.abs(w - wr) / wr):.2e}", flush=True)


def test_train_and_learned_query_exact(oracle_lib, tmp_path):
    P = datagen.uniform(1 << 16, 3, 0)
    train = datagen.uniform(1 << 16, 3, 5)
    Qs = datagen.uniform(20000, 3, 6)
    tree = kd.kd_build(_t(P))
    print("[gpu] training", flush=True)
    model = kd.kd_radius_model_train(tree, _t(train), 8, epochs=12, batch=1024, seed=1)
    info = model.info()
    assert len(info["loss_curve"]) == 12
    assert info["loss_curve"][-1] < info["loss_curve"][0]
    # labels on the held-out tail vary; the model must explain part of it
    order = oracle_lib.build_tree(P)
    _, d_hold, _ = oracle_lib.knn(P, order, train[-6553:], 8)
    assert info["holdout_rmse"] < np.std(M.label(d_hold[:, -1]))
    gi, gd, gv, st = kd.kd_knn_learned(tree, model, _t(Qs), 8, want_visited=True, want_stats=True)
    torch.cuda.synchronize()
    pi, pd, pv = oracle_lib.knn(P, order, Qs, 8)
    assert np.array_equal(gi.cpu().numpy(), pi)
    assert np.array_equal(gd.cpu().numpy().view(np.uint32), pd.view(np.uint32))
    assert st["queries"] == len(Qs)
    assert st["fallbacks"] < 0.2 * len(Qs)
    # the stats' entered-node total is the sum of the per-query counts (no
    # hand-off when the counts are requested), and every stage took time
    assert st["visited"] == int(gv.to(torch.int64).sum().item())
    assert st["handed_off"] == 0
    assert st["sort_ms"] > 0 and st["radius_ms"] > 0 and st["traverse_ms"] > 0 and st["handoff_ms"] >= 0
    # without the per-query counts the hand-off may run; the total still
    # covers every single-lane step
    _, _, _, st2 = kd.kd_knn_learned(tree, model, _t(Qs), 8, want_stats=True)
    assert st2["queries"] == len(Qs) and st2["visited"] > 0 and st2["fallbacks"] <= st["fallbacks"]
    # save / load round trip
    path = os.path.join(str(tmp_path), "m.kdm")
    model.save(path)
    m2 = kd.kd_model_load(path)
    p1, lo1, inv1 = model.params()
    p2, lo2, inv2 = m2.params()
    assert np.array_equal(p1, p2) and np.array_equal(lo1, lo2) and m2.info()["margin"] == info["margin"]
    gi2, _, _, _ = kd.kd_knn_learned(tree, m2, _t(Qs), 8)
    torch.cuda.synchronize()
    assert np.array_equal(gi2.cpu().numpy(), pi)


def test_learned_gain_report(oracle_lib):
    """What the trained network gains: processed nodes and time of plain vs
    learned vs constant radius vs perfect radius on 1M uniform points, k=8.
    Results are asserted identical; the gain is reported, not asserted."""
    P, Qs = datagen.workload("uniform-1m")
    train = datagen.uniform(1 << 20, 3, 7)
    tree = kd.kd_build(_t(P))
    q = _t(Qs)
    model = kd.kd_radius_model_train(tree, _t(train), 8, epochs=4, batch=8192, seed=2)
    pi, pd, pv = kd.kd_knn_ex(tree, q, 8, want_visited=True)
    li, ld, lv, st = kd.kd_knn_learned(tree, model, q, 8, want_visited=True, want_stats=True)
    kth = torch.sqrt(pd[:, -1].double()).float()
    ci, cd, cv, _ = kd.kd_knn_with_radius(tree, torch.full_like(kth, float(torch.quantile(kth, 0.95))), q, 8,
                                          want_visited=True)
    fi, fd, fv, _ = kd.kd_knn_with_radius(tree, kth * (1 + 2 ** -20), q, 8, want_visited=True)
    torch.cuda.synchronize()
    for a, b in [(li, pi), (ci, pi), (fi, pi)]:
        assert torch.equal(a, b)
    tot = lambda v: int(v.to(torch.int64).sum().item())
    print(f"[gpu] processed nodes: plain {tot(pv)} learned {tot(lv)} constant {tot(cv)} perfect {tot(fv)}; "
          f"fallbacks {st['fallbacks']}", flush=True)
