"""CPU oracle for exact fcp / kNN over left-balanced level-order k-d trees.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product library never does.  It
shares no code with the HIP path (``paper_2210_12859_amd``), and neither side
imports the other.

Contents
  * ``kd_oracle.c`` (loaded through ctypes): canonical build (split
    dimension by level, or stored per node: the widest extent), the ordered
    recursive traversal of the paper's Sec. 3.1, brute force, the
    learned-radius rule, radius and box queries by their plain definitions
    (the sphere and box query variants that Sec. 3 names),
    threaded batch drivers.
  * ``mlp_ref``: float64 reference of the radius-prediction MLP with the
    bfloat16 rounding points of the GPU kernels emulated.

Conventions (same as the product's public contract): points and queries are
float32 ``[n][D]`` row-major; results are ``int32`` caller indices and float32
squared distances ``[Q][k]``, ascending by (d2, index); empty slots are
``(-1, +inf)``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kd_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libkd_oracle.so")
# IEEE binary32 left-to-right sums: no contraction into fused multiply-add,
# no fast-math; plain x86-64 code so the library runs on any host.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
          "-fno-unsafe-math-optimizations", "-pthread"]

_lib = None


def build(force: bool = True) -> str:
    """Compile kd_oracle.c into libkd_oracle.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int
    f32 = ctypes.c_float
    lib.oracle_left_size.argtypes = [i64]
    lib.oracle_left_size.restype = i64
    lib.oracle_build.argtypes = [P, i64, i32, P]
    lib.oracle_build.restype = i32
    lib.oracle_build_rule.argtypes = [P, i64, i32, i32, P, P]
    lib.oracle_build_rule.restype = i32
    lib.oracle_knn_one_dims.argtypes = [P, P, P, i64, i32, P, i32, f32, P, P, P, P, i64]
    lib.oracle_knn_one_dims.restype = i32
    lib.oracle_knn_batch_dims.argtypes = [P, P, P, i64, i32, P, i64, i32, f32, P, P, P, i32]
    lib.oracle_knn_batch_dims.restype = i32
    lib.oracle_knn_one.argtypes = [P, P, i64, i32, P, i32, f32, P, P, P, P, i64]
    lib.oracle_knn_one.restype = i32
    lib.oracle_worst0.argtypes = [f32, f32]
    lib.oracle_worst0.restype = f32
    lib.oracle_knn_learned_one.argtypes = [P, P, i64, i32, P, i32, f32, f32, P, P, P, P]
    lib.oracle_knn_learned_one.restype = i32
    lib.oracle_brute_one.argtypes = [P, i64, i32, P, i32, f32, P, P]
    lib.oracle_brute_one.restype = None
    lib.oracle_knn_batch.argtypes = [P, P, i64, i32, P, i64, i32, f32, P, P, P, i32]
    lib.oracle_knn_batch.restype = i32
    lib.oracle_brute_batch.argtypes = [P, i64, i32, P, i64, i32, f32, P, P, i32]
    lib.oracle_brute_batch.restype = i32
    lib.oracle_knn_learned_batch.argtypes = [P, P, i64, i32, P, i64, i32, f32, P, P, P, P, P, i32]
    lib.oracle_knn_learned_batch.restype = i32
    lib.oracle_radius_batch.argtypes = [P, i64, i32, P, i64, i32, f32, P, P, P, i32]
    lib.oracle_radius_batch.restype = i32
    lib.oracle_box_batch.argtypes = [P, i64, i32, P, i64, i32, P, P, i32]
    lib.oracle_box_batch.restype = i32
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32c(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def default_threads() -> int:
    return len(os.sched_getaffinity(0))


def sq_radius(max_radius: float) -> np.float32:
    """R2 = fl32(maxR * maxR); +inf stays +inf."""
    r = np.float32(max_radius)
    with np.errstate(over="ignore"):
        return np.float32(r * r)


def left_size(n: int) -> int:
    return int(_load().oracle_left_size(n))


def build_tree(points) -> np.ndarray:
    """Level-order permutation: order[pos] = caller index stored at pos."""
    P = _f32c(points)
    N, D = P.shape
    order = np.empty(N, dtype=np.int32)
    rc = _load().oracle_build(_ptr(P), N, D, _ptr(order))
    if rc != 0:
        raise ValueError("oracle_build failed")
    return order


def build_tree_widest(points):
    """Tree with stored split dimensions, each node's the widest extent of its
    point set.  Returns (order[N], dims[N] uint8), by level-order position."""
    P = _f32c(points)
    N, D = P.shape
    order = np.empty(N, dtype=np.int32)
    dims = np.empty(N, dtype=np.uint8)
    rc = _load().oracle_build_rule(_ptr(P), N, D, 1, _ptr(order), _ptr(dims))
    if rc != 0:
        raise ValueError("oracle_build_rule failed")
    return order, dims


def _dims_arg(dims):
    return None if dims is None else np.ascontiguousarray(dims, np.uint8)


def knn_one(points, order, q, k, max_radius=np.inf, worst0=None, record_sequence=False, dims=None):
    """One query (dims: stored split dimensions, else by level).
    Returns (idx[k], d2[k], visited, found[, sequence])."""
    P = _f32c(points)
    N, D = P.shape
    q = _f32c(q).reshape(D)
    R2 = sq_radius(max_radius)
    w0 = R2 if worst0 is None else np.float32(worst0)
    oi = np.empty(k, np.int32)
    od = np.empty(k, np.float32)
    vis = np.zeros(1, np.int64)
    seq = np.full(max(N, 1), -1, np.int32) if record_sequence else None
    found = _load().oracle_knn_one_dims(_ptr(P), _ptr(np.ascontiguousarray(order, np.int32)),
                                        _ptr(_dims_arg(dims)), N, D, _ptr(q), k, w0, _ptr(oi), _ptr(od),
                                        _ptr(vis), _ptr(seq), len(seq) if seq is not None else 0)
    if record_sequence:
        return oi, od, int(vis[0]), found, seq[: int(vis[0])].copy()
    return oi, od, int(vis[0]), found


def knn(points, order, queries, k, max_radius=np.inf, nthreads=None, dims=None):
    """Batch of queries through the recursive traversal (dims: stored split
    dimensions by position, else by level).
    Returns (idx[Q][k], d2[Q][k], visited[Q])."""
    P = _f32c(points)
    Qs = _f32c(queries)
    N, D = P.shape
    Q = Qs.shape[0]
    oi = np.empty((Q, k), np.int32)
    od = np.empty((Q, k), np.float32)
    vis = np.empty(Q, np.int64)
    rc = _load().oracle_knn_batch_dims(_ptr(P), _ptr(np.ascontiguousarray(order, np.int32)),
                                       _ptr(_dims_arg(dims)), N, D, _ptr(Qs), Q, k, sq_radius(max_radius),
                                       _ptr(oi), _ptr(od), _ptr(vis), nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_knn_batch failed")
    return oi, od, vis


def brute(points, queries, k, max_radius=np.inf, nthreads=None):
    """Plain definition, O(N) per query.  Returns (idx[Q][k], d2[Q][k])."""
    P = _f32c(points)
    Qs = _f32c(queries)
    N, D = P.shape if P.size else (0, Qs.shape[1])
    Q = Qs.shape[0]
    oi = np.empty((Q, k), np.int32)
    od = np.empty((Q, k), np.float32)
    rc = _load().oracle_brute_batch(_ptr(P), N, D, _ptr(Qs), Q, k, sq_radius(max_radius),
                                    _ptr(oi), _ptr(od), nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_brute_batch failed")
    return oi, od


def worst0(max_radius, r0) -> np.float32:
    return np.float32(_load().oracle_worst0(sq_radius(max_radius), np.float32(r0)))


def knn_learned(points, order, queries, k, r0, max_radius=np.inf, nthreads=None):
    """Learned-radius rule with exact fallback.
    Returns (idx, d2, visited, fell_back[Q] bool)."""
    P = _f32c(points)
    Qs = _f32c(queries)
    N, D = P.shape
    Q = Qs.shape[0]
    r0 = _f32c(r0).reshape(Q)
    oi = np.empty((Q, k), np.int32)
    od = np.empty((Q, k), np.float32)
    vis = np.empty(Q, np.int64)
    fb = np.empty(Q, np.int32)
    rc = _load().oracle_knn_learned_batch(_ptr(P), _ptr(np.ascontiguousarray(order, np.int32)),
                                          N, D, _ptr(Qs), Q, k, sq_radius(max_radius), _ptr(r0),
                                          _ptr(oi), _ptr(od), _ptr(vis), _ptr(fb),
                                          nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_knn_learned_batch failed")
    return oi, od, vis, fb.astype(bool)


def radius(points, queries, max_radius, k=0, nthreads=None):
    """All points within max_radius (d2 <= fl32(maxR^2)) of each query, by the
    plain definition.  Returns (count[Q], idx[Q][k], d2[Q][k]): the number of
    such points and the k nearest of them by (d2, caller index)."""
    P = _f32c(points)
    Qs = _f32c(queries)
    N, D = P.shape if P.size else (0, Qs.shape[1])
    Q = Qs.shape[0]
    oi = np.empty((Q, k), np.int32)
    od = np.empty((Q, k), np.float32)
    cnt = np.empty(Q, np.int64)
    rc = _load().oracle_radius_batch(_ptr(P), N, D, _ptr(Qs), Q, k, sq_radius(max_radius),
                                     _ptr(oi) if k else None, _ptr(od) if k else None, _ptr(cnt),
                                     nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_radius_batch failed")
    return cnt, oi, od


def box(points, lo, hi, k=0, nthreads=None):
    """All points inside the axis-aligned boxes [lo, hi] (inclusive in every
    dimension), by the plain definition.  Returns (count[Q], idx[Q][k]): the
    number of such points and the k smallest caller indices of them."""
    P = _f32c(points)
    lo = _f32c(lo)
    hi = _f32c(hi)
    Q, D = lo.shape
    N = P.shape[0] if P.size else 0
    boxes = np.ascontiguousarray(np.stack([lo, hi], axis=1), np.float32)  # [Q][2][D]
    oi = np.empty((Q, k), np.int32)
    cnt = np.empty(Q, np.int64)
    rc = _load().oracle_box_batch(_ptr(P), N, D, _ptr(boxes), Q, k, _ptr(oi) if k else None, _ptr(cnt),
                                  nthreads or default_threads())
    if rc != 0:
        raise ValueError("oracle_box_batch failed")
    return cnt, oi
