"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every declared entry point, argument validation rejects bad calls before any
device work, and the host builder produces the oracle's canonical tree."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_2210_12859_amd as kd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"^\s*(?:kd_status|const\s+char\s*\*)\s*(kd_\w+)\s*\(", src, flags=re.M))
    return sorted(names)


def test_header_declares_core_entry_points():
    names = _declared_symbols()
    for n in ["kd_build", "kd_fcp", "kd_knn", "kd_tree_free", "kd_status_str", "kd_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    L = kd.lib()
    for name in _declared_symbols():
        assert hasattr(L, name), name


def test_status_strings():
    L = kd.lib()
    for s in [0, -1, -2, -3, -4]:
        assert L.kd_status_str(s).decode().startswith("KD_")
    assert kd.version().startswith("kdtree-gfx950")


# Validation paths return before any HIP call, so they run without a device.
P = ctypes.c_void_p


def _knn(tree=None, queries=P(8), Q=4, k=8, maxr=math.inf, out_idx=P(8)):
    return kd.lib().kd_knn(tree, queries, Q, k, maxr, out_idx, None, None)


@pytest.mark.parametrize("kw,frag", [
    (dict(k=0), "k out of range"), (dict(k=65), "k out of range"), (dict(Q=-1), "Q out of range"),
    (dict(maxr=-1.0), "maxRadius"), (dict(maxr=float("nan")), "maxRadius"),
    (dict(), "tree is NULL"),
])
def test_query_validation(kw, frag):
    assert _knn(**kw) == kd.KD_EINVAL
    assert frag in kd.lib().kd_last_error().decode()


def test_fcp_validation():
    L = kd.lib()
    assert L.kd_fcp(None, P(8), 4, -2.0, P(8), None, None) == kd.KD_EINVAL
    assert L.kd_fcp(None, P(8), 4, 1.0, P(8), None, None) == kd.KD_EINVAL


def test_range_validation():
    L = kd.lib()
    cnt = P(8)
    # radius: cap, Q, radius, tree, NULL outputs
    assert L.kd_radius_search(None, P(8), 4, 1.0, 65, P(8), None, cnt, None, 0, None) == kd.KD_EINVAL
    assert "cap out of range" in L.kd_last_error().decode()
    assert L.kd_radius_search(None, P(8), 4, 1.0, -1, P(8), None, cnt, None, 0, None) == kd.KD_EINVAL
    assert L.kd_radius_search(None, P(8), -1, 1.0, 1, P(8), None, cnt, None, 0, None) == kd.KD_EINVAL
    assert "Q out of range" in L.kd_last_error().decode()
    assert L.kd_radius_search(None, P(8), 4, -1.0, 1, P(8), None, cnt, None, 0, None) == kd.KD_EINVAL
    assert "maxRadius" in L.kd_last_error().decode()
    assert L.kd_radius_search(None, P(8), 4, float("nan"), 1, P(8), None, cnt, None, 0, None) == kd.KD_EINVAL
    assert L.kd_radius_search(None, P(8), 4, 1.0, 1, P(8), None, cnt, None, 0, None) == kd.KD_EINVAL
    assert "tree is NULL" in L.kd_last_error().decode()
    # box: cap, Q, tree
    assert L.kd_box_search(None, P(8), 4, 65, P(8), cnt, None, 0, None) == kd.KD_EINVAL
    assert "cap out of range" in L.kd_last_error().decode()
    assert L.kd_box_search(None, P(8), 1 << 31, 1, P(8), cnt, None, 0, None) == kd.KD_EINVAL
    assert L.kd_box_search(None, P(8), 4, 0, None, cnt, None, 0, None) == kd.KD_EINVAL
    assert "tree is NULL" in L.kd_last_error().decode()


def test_range_all_validation():
    L = kd.lib()
    tot = ctypes.c_int64()
    off = P(8)
    # radius: total NULL, Q, flags, radius, capacity, out_idx, tree
    assert L.kd_radius_search_all(None, P(8), 4, 1.0, off, P(8), 10, None, 0, None) == kd.KD_EINVAL
    assert "total is NULL" in L.kd_last_error().decode()
    assert L.kd_radius_search_all(None, P(8), -1, 1.0, off, P(8), 10, ctypes.byref(tot), 0, None) == kd.KD_EINVAL
    assert L.kd_radius_search_all(None, P(8), 4, 1.0, off, P(8), 10, ctypes.byref(tot), 4, None) == kd.KD_EINVAL
    assert "unknown flags" in L.kd_last_error().decode()
    assert L.kd_radius_search_all(None, P(8), 4, -1.0, off, P(8), 10, ctypes.byref(tot), 0, None) == kd.KD_EINVAL
    assert L.kd_radius_search_all(None, P(8), 4, 1.0, off, P(8), -1, ctypes.byref(tot), 0, None) == kd.KD_EINVAL
    assert "capacity" in L.kd_last_error().decode()
    assert L.kd_radius_search_all(None, P(8), 4, 1.0, off, None, 10, ctypes.byref(tot), 0, None) == kd.KD_EINVAL
    assert "out_idx is NULL" in L.kd_last_error().decode()
    assert L.kd_radius_search_all(None, P(8), 4, 1.0, off, None, 0, ctypes.byref(tot), 0, None) == kd.KD_EINVAL
    assert "tree is NULL" in L.kd_last_error().decode()
    assert L.kd_box_search_all(None, P(8), 4, off, None, 0, ctypes.byref(tot), 0, None) == kd.KD_EINVAL
    assert "tree is NULL" in L.kd_last_error().decode()


def test_build_validation():
    L = kd.lib()
    h = ctypes.c_void_p()
    pts = np.zeros((4, 3), np.float32)
    pp = pts.ctypes.data_as(P)
    assert L.kd_build(pp, 4, 5, None, ctypes.byref(h)) == kd.KD_EINVAL
    assert L.kd_build(pp, 4, 1, None, ctypes.byref(h)) == kd.KD_EINVAL
    assert L.kd_build(pp, -1, 3, None, ctypes.byref(h)) == kd.KD_EINVAL
    assert L.kd_build(pp, (1 << 30) + 1, 3, None, ctypes.byref(h)) == kd.KD_EINVAL
    # N = 2^30: the largest 1-based node id would be 2^30, whose child ids
    # 2^31 and 2^31 + 1 overflow int32; rejected before anything is read or
    # allocated (the 4-point buffer is never touched)
    for n in (1 << 30, (1 << 31) - 1):
        assert L.kd_build(pp, n, 3, None, ctypes.byref(h)) == kd.KD_EINVAL
        assert "2^30 - 1" in L.kd_last_error().decode()
        assert L.kd_build_host(pp, n, 3, ctypes.byref(h)) == kd.KD_EINVAL
        assert L.kd_build_order_host(pp, n, 3, None) == kd.KD_EINVAL
    assert L.kd_build(None, 4, 3, None, ctypes.byref(h)) == kd.KD_EINVAL
    assert L.kd_build_ex(pp, 4, 3, 2, None, ctypes.byref(h)) == kd.KD_EINVAL
    assert "split" in L.kd_last_error().decode()
    assert L.kd_build_ex(pp, 4, 3, -1, None, ctypes.byref(h)) == kd.KD_EINVAL
    assert L.kd_build(pp, 4, 3, None, None) == kd.KD_EINVAL
    bad = pts.copy()
    bad[2, 1] = np.nan
    assert L.kd_build_host(bad.ctypes.data_as(P), 4, 3, ctypes.byref(h)) == kd.KD_EINVAL
    bad[2, 1] = np.inf
    assert L.kd_build_host(bad.ctypes.data_as(P), 4, 3, ctypes.byref(h)) == kd.KD_EINVAL
    assert "NaN or inf" in L.kd_last_error().decode()


# ------------------------------------------------------------ host builder

@pytest.mark.parametrize("N,D,seed", [(0, 3, 0), (1, 3, 0), (2, 2, 1), (6, 2, 2), (17, 3, 3), (1000, 3, 4),
                                      (4097, 4, 5), (3000, 1, 6), (50000, 3, 7)])
def test_host_builder_equals_oracle(oracle_lib, N, D, seed):
    P_ = np.random.default_rng(seed).random((N, D), dtype=np.float32)
    assert np.array_equal(kd.kd_build_order_host(P_), oracle_lib.build_tree(P_) if N else np.zeros(0, np.int32))


def test_host_builder_equals_oracle_ties(oracle_lib):
    rng = np.random.default_rng(8)
    P_ = rng.integers(0, 4, size=(5000, 3)).astype(np.float32)
    assert np.array_equal(kd.kd_build_order_host(P_), oracle_lib.build_tree(P_))


def test_host_builder_figure1(oracle_lib):
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "figure1.json")))
    assert kd.kd_build_order_host(np.array(g["points"], np.float32)).tolist() == g["order"]


@pytest.mark.slow
def test_host_builder_equals_oracle_1m(oracle_lib):
    from paper_2210_12859_amd import datagen
    P_, _ = datagen.workload("uniform-1m")
    assert np.array_equal(kd.kd_build_order_host(P_), oracle_lib.build_tree(P_))


def test_workspace_size():
    """kd_workspace_size: host only; grows with Q, covers the traversal
    records (32 B per query for D = 4) and the sort buffers, adds the
    per-query radii for learned calls, validates its arguments."""
    assert kd.kd_workspace_size(0, 8) == 0
    a = kd.kd_workspace_size(1 << 20, 8)
    b = kd.kd_workspace_size(1 << 21, 8)
    assert b > a >= (1 << 20) * (32 + 2 * (4 + 32))
    assert kd.kd_workspace_size(1 << 20, 1) == a == kd.kd_workspace_size(1 << 20, 64)
    assert kd.kd_workspace_size(1 << 20, 8, learned=True) >= a + (1 << 20) * 4
    L = kd.lib()
    out = ctypes.c_size_t()
    for Q, k, flags in [(-1, 8, 0), (1 << 31, 8, 0), (10, 0, 0), (10, 65, 0), (10, 8, 2)]:
        assert L.kd_workspace_size(Q, k, flags, ctypes.byref(out)) == kd.KD_EINVAL
    assert L.kd_workspace_size(10, 8, 0, None) == kd.KD_EINVAL
