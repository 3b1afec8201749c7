"""Python binding of libkdtree.so (exact fcp / kNN over left-balanced k-d trees
on MI355X).  Argument marshalling only: every step of the query path runs in
the library's HIP kernels.  Tensors are torch CUDA (HIP) tensors; the stream
is torch's current stream unless one is passed.

The library must have been built (``python -m paper_2210_12859_amd.build``);
there is no fallback: a missing library raises ``KdLibraryMissing``.
"""
from __future__ import annotations

import ctypes
import math
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libkdtree.so")

KD_OK, KD_EINVAL, KD_ENOMEM, KD_EHIP, KD_EUNSUPPORTED = 0, -1, -2, -3, -4
KD_MAX_K = 64

_lib = None


class KdLibraryMissing(RuntimeError):
    pass


class KdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class KdTrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("seed", ctypes.c_uint64), ("holdout", ctypes.c_int64), ("margin_quantile", ctypes.c_float)]


class KdStats(ctypes.Structure):
    _fields_ = [("queries", ctypes.c_int64), ("fallbacks", ctypes.c_int64), ("handed_off", ctypes.c_int64),
                ("visited", ctypes.c_int64), ("sort_ms", ctypes.c_float), ("radius_ms", ctypes.c_float),
                ("traverse_ms", ctypes.c_float), ("handoff_ms", ctypes.c_float)]


class KdJob(ctypes.Structure):
    _fields_ = [("tree", ctypes.c_void_p), ("queries", ctypes.c_void_p), ("Q", ctypes.c_int64),
                ("k", ctypes.c_int), ("maxRadius", ctypes.c_float), ("out_idx", ctypes.c_void_p),
                ("out_d2", ctypes.c_void_p), ("model", ctypes.c_void_p)]


class KdOpts(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("lds_levels", ctypes.c_int),
                ("sort_bits", ctypes.c_int), ("waves_per_cu", ctypes.c_int), ("heavy_trips", ctypes.c_int),
                ("prune", ctypes.c_int)]


def lib():
    """Load libkdtree.so (once)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise KdLibraryMissing(f"{LIB_PATH} is not built; run python -m paper_2210_12859_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, i32, f32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_float
    sig = {
        "kd_build": ([P, i64, i32, P, P], i32),
        "kd_build_ex": ([P, i64, i32, i32, P, P], i32),
        "kd_tree_dims": ([P, P, P], i32),
        "kd_build_host": ([P, i64, i32, P], i32),
        "kd_build_order_host": ([P, i64, i32, P], i32),
        "kd_tree_free": ([P], i32),
        "kd_tree_info": ([P, P, P, P, P], i32),
        "kd_tree_order": ([P, P], i32),
        "kd_fcp": ([P, P, i64, f32, P, P, P], i32),
        "kd_knn": ([P, P, i64, i32, f32, P, P, P], i32),
        "kd_knn_ex": ([P, P, i64, i32, f32, P, P, P, P, P], i32),
        "kd_knn_noalloc": ([P, P, i64, i32, f32, P, P, P], i32),
        "kd_radius_search": ([P, P, i64, f32, i32, P, P, P, P, i32, P], i32),
        "kd_box_search": ([P, P, i64, i32, P, P, P, i32, P], i32),
        "kd_radius_search_all": ([P, P, i64, f32, P, P, i64, P, i32, P], i32),
        "kd_box_search_all": ([P, P, i64, P, P, i64, P, i32, P], i32),
        "kd_radius_model_train": ([P, P, i64, i32, P, P, P], i32),
        "kd_knn_learned": ([P, P, P, i64, i32, f32, P, P, P, P, P, P], i32),
        "kd_knn_with_radius": ([P, P, P, i64, i32, f32, P, P, P, P, P, P], i32),
        "kd_model_info": ([P, P, P, P, P, P, i32], i32),
        "kd_model_get_params": ([P, P, P, P], i32),
        "kd_model_create": ([P, P, P, f32, i32, P], i32),
        "kd_model_save": ([P, ctypes.c_char_p], i32),
        "kd_model_load": ([ctypes.c_char_p, P], i32),
        "kd_model_free": ([P], i32),
        "kd_mlp_predict": ([P, P, i64, P, P], i32),
        "kd_mlp_grad": ([P, P, P, i64, P, P, P], i32),
        "kd_mlp_worst0": ([P, P, i64, f32, P, P], i32),
        "kd_mlp_train_step": ([P, P, P, i64, i32, f32, P, P, P, P, P], i32),
        "kd_batch_create": ([P, i32, P, P, P, P], i32),
        "kd_batch_run": ([P, P], i32),
        "kd_batch_free": ([P], i32),
        "kd_knn_batched": ([P, i32, P, P, P], i32),
        "kd_batch_autotune": ([P, i32, P, P, P], i32),
        "kd_batch_info": ([P, P, P, P, P, i32], i32),
        "kd_autotune": ([P, P, i64, i32, f32, P, P, P], i32),
        "kd_tree_get_tuned": ([P, i32, P], i32),
        "kd_tree_set_tuned": ([P, i32, P], i32),
        "kd_workspace_size": ([i64, i32, i32, P], i32),
        "kd_timing_enable": ([i32], i32),
        "kd_timing_collect": ([ctypes.c_char_p, P, P], i32),
        "kd_status_str": ([i32], ctypes.c_char_p),
        "kd_last_error": ([], ctypes.c_char_p),
        "kd_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(status: int):
    if status != KD_OK:
        msg = lib().kd_last_error().decode()
        raise KdError(status, msg or lib().kd_status_str(status).decode())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _require(t, dtype, name, shape=None):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


class Tree:
    """Handle of a kd_tree built by kd_build; freed with close() or on GC."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("tree is closed")
        return self._h

    def info(self):
        n = ctypes.c_int64()
        d = ctypes.c_int()
        lo = (ctypes.c_float * 4)()
        hi = (ctypes.c_float * 4)()
        _check(lib().kd_tree_info(self.handle, ctypes.byref(n), ctypes.byref(d), lo, hi))
        return dict(N=n.value, dim=d.value, lo=list(lo)[: d.value], hi=list(hi)[: d.value])

    def order(self):
        import numpy as np
        n = self.info()["N"]
        out = np.empty(n, np.int32)
        _check(lib().kd_tree_order(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def dims(self):
        """(split dimension of every tree position, uint8 [N]; the rule,
        KD_SPLIT_LEVEL or KD_SPLIT_WIDEST)."""
        import numpy as np
        n = self.info()["N"]
        out = np.empty(n, np.uint8)
        rule = ctypes.c_int()
        _check(lib().kd_tree_dims(self.handle, out.ctypes.data_as(ctypes.c_void_p), ctypes.byref(rule)))
        return out, rule.value

    def close(self):
        if self._h:
            lib().kd_tree_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


KD_SPLIT_LEVEL = 0
KD_SPLIT_WIDEST = 1


def kd_build(points, stream=None, split=KD_SPLIT_LEVEL) -> Tree:
    """Canonical left-balanced tree over device float32 points [N][dim];
    split: KD_SPLIT_LEVEL (dimension by level) or KD_SPLIT_WIDEST (stored
    per node, the widest extent of its subtree)."""
    import torch
    _require(points, torch.float32, "points")
    if points.dim() != 2:
        raise ValueError("points must be [N][dim]")
    h = ctypes.c_void_p()
    _check(lib().kd_build_ex(_ptr(points), points.shape[0], points.shape[1], int(split), _stream_handle(stream),
                             ctypes.byref(h)))
    return Tree(h.value)


def kd_build_host(points_np) -> Tree:
    import numpy as np
    P = np.ascontiguousarray(points_np, dtype=np.float32)
    h = ctypes.c_void_p()
    _check(lib().kd_build_host(P.ctypes.data_as(ctypes.c_void_p), P.shape[0], P.shape[1], ctypes.byref(h)))
    return Tree(h.value)


def kd_build_order_host(points_np):
    """Canonical level-order permutation computed on the host (no device)."""
    import numpy as np
    P = np.ascontiguousarray(points_np, dtype=np.float32)
    out = np.empty(P.shape[0], np.int32)
    _check(lib().kd_build_order_host(P.ctypes.data_as(ctypes.c_void_p), P.shape[0], P.shape[1],
                                     out.ctypes.data_as(ctypes.c_void_p)))
    return out


def _outputs(queries, k, out_idx, out_d2, want_d2):
    import torch
    Q = queries.shape[0]
    if out_idx is None:
        out_idx = torch.empty((Q, k) if k > 1 else (Q,), dtype=torch.int32, device=queries.device)
    if out_d2 is None and want_d2:
        out_d2 = torch.empty_like(out_idx, dtype=torch.float32)
    _require(out_idx, torch.int32, "out_idx")
    if out_idx.numel() != Q * k:
        raise ValueError("out_idx must hold Q*k entries")
    if out_d2 is not None:
        _require(out_d2, torch.float32, "out_d2")
        if out_d2.numel() != Q * k:
            raise ValueError("out_d2 must hold Q*k entries")
    return out_idx, out_d2


def _opts(opts):
    if opts is None:
        return None
    if isinstance(opts, KdOpts):
        return ctypes.byref(opts)
    o = KdOpts(opts.get("block", 0), opts.get("lds_levels", -1), opts.get("sort_bits", -1),
               opts.get("waves_per_cu", 0), opts.get("heavy_trips", 0), opts.get("prune", 0))
    return ctypes.byref(o)


def kd_fcp(tree: Tree, queries, max_radius=math.inf, out_idx=None, out_d2=None, want_d2=True, stream=None):
    import torch
    _require(queries, torch.float32, "queries")
    out_idx, out_d2 = _outputs(queries, 1, out_idx, out_d2, want_d2)
    _check(lib().kd_fcp(tree.handle, _ptr(queries), queries.shape[0], float(max_radius), _ptr(out_idx),
                        _ptr(out_d2), _stream_handle(stream)))
    return out_idx, out_d2


def kd_knn(tree: Tree, queries, k, max_radius=math.inf, out_idx=None, out_d2=None, want_d2=True,
           stream=None):
    import torch
    _require(queries, torch.float32, "queries")
    out_idx, out_d2 = _outputs(queries, k, out_idx, out_d2, want_d2)
    _check(lib().kd_knn(tree.handle, _ptr(queries), queries.shape[0], int(k), float(max_radius),
                        _ptr(out_idx), _ptr(out_d2), _stream_handle(stream)))
    return out_idx, out_d2


def kd_knn_noalloc(tree: Tree, queries, k, max_radius=math.inf, out_idx=None, out_d2=None, want_d2=True,
                   stream=None):
    """kd_knn through the entry point that allocates no device memory (its
    scratch is a fixed library array; output tensors allocated here when not
    given)."""
    import torch
    _require(queries, torch.float32, "queries")
    out_idx, out_d2 = _outputs(queries, k, out_idx, out_d2, want_d2)
    _check(lib().kd_knn_noalloc(tree.handle, _ptr(queries), queries.shape[0], int(k), float(max_radius),
                                _ptr(out_idx), _ptr(out_d2), _stream_handle(stream)))
    return out_idx, out_d2


KD_RANGE_BOXES = 1


def kd_radius_search(tree: Tree, queries, max_radius, cap=0, want_d2=True, visited=None, flags=0, stream=None):
    """Points within max_radius of each query: (count [Q], idx int32 [Q][cap],
    d2 float32 [Q][cap]); idx/d2 are None when cap is 0.  Counts come back
    in an int32 tensor (the library writes uint32; counts stay below 2^30).
    visited: optional int32 [Q] tensor receiving the entered-node counts.
    flags: 0 (split planes only) or KD_RANGE_BOXES (also subtree boxes)."""
    import torch
    _require(queries, torch.float32, "queries")
    Q = queries.shape[0]
    count = torch.empty(Q, dtype=torch.int32, device=queries.device)
    idx = d2 = None
    if cap > 0:
        idx = torch.empty((Q, cap), dtype=torch.int32, device=queries.device)
        if want_d2:
            d2 = torch.empty((Q, cap), dtype=torch.float32, device=queries.device)
    if visited is not None:
        _require(visited, torch.int32, "visited", (Q,))
    _check(lib().kd_radius_search(tree.handle, _ptr(queries), Q, float(max_radius), int(cap), _ptr(idx),
                                  _ptr(d2), _ptr(count), _ptr(visited), int(flags), _stream_handle(stream)))
    return count, idx, d2


def kd_box_search(tree: Tree, lo, hi, cap=0, visited=None, flags=0, stream=None):
    """Points inside the boxes [lo, hi] (inclusive): (count [Q], idx int32
    [Q][cap] or None when cap is 0); visited as kd_radius_search."""
    import torch
    _require(lo, torch.float32, "lo")
    _require(hi, torch.float32, "hi")
    if lo.shape != hi.shape:
        raise ValueError("lo and hi must have the same shape")
    boxes = torch.stack([lo, hi], dim=1).contiguous()  # [Q][2][dim]
    Q = lo.shape[0]
    count = torch.empty(Q, dtype=torch.int32, device=lo.device)
    idx = torch.empty((Q, cap), dtype=torch.int32, device=lo.device) if cap > 0 else None
    if visited is not None:
        _require(visited, torch.int32, "visited", (Q,))
    _check(lib().kd_box_search(tree.handle, _ptr(boxes), Q, int(cap), _ptr(idx), _ptr(count), _ptr(visited),
                               int(flags), _stream_handle(stream)))
    return count, idx


def _range_all(call, Q, dev, capacity):
    import torch
    offsets = torch.empty(Q + 1, dtype=torch.int64, device=dev)
    cap = int(capacity) if capacity is not None else max(1024, 16 * Q)
    out = torch.empty(cap, dtype=torch.int32, device=dev)
    total = ctypes.c_int64()
    _check(call(offsets, out, cap, total))
    if total.value > cap:
        cap = total.value
        out = torch.empty(cap, dtype=torch.int32, device=dev)
        _check(call(offsets, out, cap, total))
    return offsets, out[: total.value]


def kd_radius_search_all(tree: Tree, queries, max_radius, flags=0, capacity=None, stream=None):
    """Every point within max_radius of each query: (offsets int64 [Q + 1],
    idx int32 [total]); query q's points are idx[offsets[q]:offsets[q + 1]]."""
    import torch
    _require(queries, torch.float32, "queries")
    Q = queries.shape[0]
    sh = _stream_handle(stream)
    call = lambda off, out, cap, tot: lib().kd_radius_search_all(
        tree.handle, _ptr(queries), Q, float(max_radius), _ptr(off), _ptr(out), cap, ctypes.byref(tot), int(flags), sh)
    return _range_all(call, Q, queries.device, capacity)


def kd_box_search_all(tree: Tree, lo, hi, flags=0, capacity=None, stream=None):
    """Every point inside the boxes [lo, hi] (inclusive): (offsets, idx) as
    kd_radius_search_all."""
    import torch
    _require(lo, torch.float32, "lo")
    _require(hi, torch.float32, "hi")
    if lo.shape != hi.shape:
        raise ValueError("lo and hi must have the same shape")
    boxes = torch.stack([lo, hi], dim=1).contiguous()
    Q = lo.shape[0]
    sh = _stream_handle(stream)
    call = lambda off, out, cap, tot: lib().kd_box_search_all(
        tree.handle, _ptr(boxes), Q, _ptr(off), _ptr(out), cap, ctypes.byref(tot), int(flags), sh)
    return _range_all(call, Q, lo.device, capacity)


def kd_knn_ex(tree: Tree, queries, k, max_radius=math.inf, out_idx=None, out_d2=None, visited=None,
              want_d2=True, want_visited=False, opts=None, stream=None):
    import torch
    _require(queries, torch.float32, "queries")
    out_idx, out_d2 = _outputs(queries, k, out_idx, out_d2, want_d2)
    if visited is None and want_visited:
        visited = torch.empty(queries.shape[0], dtype=torch.int32, device=queries.device)
    if visited is not None:
        _require(visited, torch.int32, "visited", (queries.shape[0],))
    _check(lib().kd_knn_ex(tree.handle, _ptr(queries), queries.shape[0], int(k), float(max_radius),
                           _ptr(out_idx), _ptr(out_d2), _ptr(visited), _opts(opts), _stream_handle(stream)))
    return out_idx, out_d2, visited


MLP_NPARAM = 4481


class Model:
    """Handle of a kd_model (learned initial-radius MLP)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        if not self._h:
            raise ValueError("model is closed")
        return self._h

    def info(self):
        k = ctypes.c_int()
        margin = ctypes.c_float()
        rmse = ctypes.c_float()
        ne = ctypes.c_int()
        curve = (ctypes.c_float * 1024)()
        _check(lib().kd_model_info(self.handle, ctypes.byref(k), ctypes.byref(margin), ctypes.byref(rmse),
                                   ctypes.byref(ne), curve, 1024))
        return dict(k=k.value, margin=margin.value, holdout_rmse=rmse.value,
                    loss_curve=list(curve)[: min(ne.value, 1024)])

    def params(self):
        import numpy as np
        p = np.empty(MLP_NPARAM, np.float32)
        lo = np.empty(3, np.float32)
        inv = np.empty(3, np.float32)
        _check(lib().kd_model_get_params(self.handle, p.ctypes.data_as(ctypes.c_void_p),
                                         lo.ctypes.data_as(ctypes.c_void_p), inv.ctypes.data_as(ctypes.c_void_p)))
        return p, lo, inv

    def save(self, path: str):
        _check(lib().kd_model_save(self.handle, str(path).encode()))

    def close(self):
        if self._h:
            lib().kd_model_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kd_radius_model_train(tree: Tree, train_q, k, epochs=20, batch=8192, lr=1e-3, seed=0, holdout=0,
                          margin_quantile=0.999, stream=None) -> Model:
    import torch
    _require(train_q, torch.float32, "train_q")
    o = KdTrainOpts(int(epochs), int(batch), float(lr), int(seed), int(holdout), float(margin_quantile))
    h = ctypes.c_void_p()
    _check(lib().kd_radius_model_train(tree.handle, _ptr(train_q), train_q.shape[0], int(k), ctypes.byref(o),
                                       ctypes.byref(h), _stream_handle(stream)))
    return Model(h.value)


def kd_model_create(params, lo, inv, margin, k) -> Model:
    import numpy as np
    p = np.ascontiguousarray(params, np.float32)
    lo = np.ascontiguousarray(lo, np.float32)
    inv = np.ascontiguousarray(inv, np.float32)
    h = ctypes.c_void_p()
    _check(lib().kd_model_create(p.ctypes.data_as(ctypes.c_void_p), lo.ctypes.data_as(ctypes.c_void_p),
                                 inv.ctypes.data_as(ctypes.c_void_p), float(margin), int(k), ctypes.byref(h)))
    return Model(h.value)


def kd_model_load(path) -> Model:
    h = ctypes.c_void_p()
    _check(lib().kd_model_load(str(path).encode(), ctypes.byref(h)))
    return Model(h.value)


def kd_knn_learned(tree: Tree, model: Model, queries, k, max_radius=math.inf, out_idx=None, out_d2=None,
                   visited=None, want_d2=True, want_visited=False, want_stats=False, opts=None, stream=None):
    """Returns (idx, d2, visited, stats dict or None)."""
    import torch
    _require(queries, torch.float32, "queries")
    out_idx, out_d2 = _outputs(queries, k, out_idx, out_d2, want_d2)
    if visited is None and want_visited:
        visited = torch.empty(queries.shape[0], dtype=torch.int32, device=queries.device)
    st = KdStats() if want_stats else None
    _check(lib().kd_knn_learned(tree.handle, model.handle, _ptr(queries), queries.shape[0], int(k),
                                float(max_radius), _ptr(out_idx), _ptr(out_d2), _ptr(visited),
                                ctypes.byref(st) if st is not None else None, _opts(opts), _stream_handle(stream)))
    stats = {name: getattr(st, name) for name, _ in KdStats._fields_} if st is not None else None
    return out_idx, out_d2, visited, stats


def kd_knn_with_radius(tree: Tree, r0, queries, k, max_radius=math.inf, out_idx=None, out_d2=None, visited=None,
                       fell_back=None, want_d2=True, want_visited=False, want_flags=False, opts=None, stream=None):
    """Returns (idx, d2, visited, fell_back uint8)."""
    import torch
    _require(queries, torch.float32, "queries")
    _require(r0, torch.float32, "r0", (queries.shape[0],))
    out_idx, out_d2 = _outputs(queries, k, out_idx, out_d2, want_d2)
    if visited is None and want_visited:
        visited = torch.empty(queries.shape[0], dtype=torch.int32, device=queries.device)
    if fell_back is None and want_flags:
        fell_back = torch.empty(queries.shape[0], dtype=torch.uint8, device=queries.device)
    _check(lib().kd_knn_with_radius(tree.handle, _ptr(r0), _ptr(queries), queries.shape[0], int(k),
                                    float(max_radius), _ptr(out_idx), _ptr(out_d2), _ptr(visited), _ptr(fell_back),
                                    _opts(opts), _stream_handle(stream)))
    return out_idx, out_d2, visited, fell_back


def kd_workspace_size(Q: int, k: int, learned: bool = False) -> int:
    """Device scratch bytes a query call of Q queries needs (upper bound over
    dim and options; kept per stream by the library).  Host only."""
    b = ctypes.c_size_t()
    _check(lib().kd_workspace_size(int(Q), int(k), 1 if learned else 0, ctypes.byref(b)))
    return b.value


def kd_mlp_predict(model: Model, queries, out=None, stream=None):
    import torch
    _require(queries, torch.float32, "queries")
    if out is None:
        out = torch.empty(queries.shape[0], dtype=torch.float32, device=queries.device)
    _check(lib().kd_mlp_predict(model.handle, _ptr(queries), queries.shape[0], _ptr(out), _stream_handle(stream)))
    return out


def kd_mlp_grad(model: Model, queries, targets, stream=None):
    """(loss, gradient as a numpy float32 [4481])."""
    import numpy as np
    import torch
    _require(queries, torch.float32, "queries")
    _require(targets, torch.float32, "targets", (queries.shape[0],))
    g = np.empty(MLP_NPARAM, np.float32)
    loss = ctypes.c_float()
    _check(lib().kd_mlp_grad(model.handle, _ptr(queries), _ptr(targets), queries.shape[0],
                             g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss), _stream_handle(stream)))
    return loss.value, g


def kd_mlp_worst0(model: Model, queries, max_radius: float = math.inf, out=None, stream=None):
    """Initial squared radius per query (device float32 [n], queries' order)."""
    import torch
    _require(queries, torch.float32, "queries")
    if out is None:
        out = torch.empty(queries.shape[0], dtype=torch.float32, device=queries.device)
    _require(out, torch.float32, "out", (queries.shape[0],))
    _check(lib().kd_mlp_worst0(model.handle, _ptr(queries), queries.shape[0], float(max_radius), _ptr(out),
                               _stream_handle(stream)))
    return out


def kd_mlp_train_step(model: Model, queries, targets, step: int, lr: float, m, v, stream=None):
    """One trainer step on the model (its parameters change in place).  m, v:
    numpy float32 [4481] Adam moments, updated in place.  Returns (loss,
    gradient as numpy float32 [4481])."""
    import numpy as np
    import torch
    _require(queries, torch.float32, "queries")
    _require(targets, torch.float32, "targets", (queries.shape[0],))
    for name, a in (("m", m), ("v", v)):
        if not (isinstance(a, np.ndarray) and a.dtype == np.float32 and a.shape == (MLP_NPARAM,)
                and a.flags["C_CONTIGUOUS"]):
            raise TypeError(f"{name} must be a contiguous numpy float32 array of {MLP_NPARAM}")
    g = np.empty(MLP_NPARAM, np.float32)
    loss = ctypes.c_float()
    _check(lib().kd_mlp_train_step(model.handle, _ptr(queries), _ptr(targets), queries.shape[0], int(step),
                                   float(lr), m.ctypes.data_as(ctypes.c_void_p), v.ctypes.data_as(ctypes.c_void_p),
                                   g.ctypes.data_as(ctypes.c_void_p), ctypes.byref(loss), _stream_handle(stream)))
    return loss.value, g


def _job_array(jobs):
    """jobs: list of dicts {tree, queries, k, max_radius=inf, out_idx, out_d2=None, model=None}."""
    import torch
    arr = (KdJob * max(1, len(jobs)))()
    for i, j in enumerate(jobs):
        q = j["queries"]
        _require(q, torch.float32, f"jobs[{i}].queries")
        _require(j["out_idx"], torch.int32, f"jobs[{i}].out_idx")
        if j["out_idx"].numel() != q.shape[0] * j["k"]:
            raise ValueError(f"jobs[{i}].out_idx must hold Q*k entries")
        d2 = j.get("out_d2")
        if d2 is not None:
            _require(d2, torch.float32, f"jobs[{i}].out_d2")
            if d2.numel() != q.shape[0] * j["k"]:
                raise ValueError(f"jobs[{i}].out_d2 must hold Q*k entries")
        m = j.get("model")
        arr[i] = KdJob(j["tree"].handle, q.data_ptr(), q.shape[0], int(j["k"]), float(j.get("max_radius", math.inf)),
                       j["out_idx"].data_ptr(), d2.data_ptr() if d2 is not None else None,
                       m.handle if m is not None else None)
    return arr


class Batch:
    """A captured batched pipeline (kd_batch); run() replays its hipGraph."""

    def __init__(self, jobs, opts=None, model=None, stream=None):
        self._jobs = jobs  # keep the tensors (and models) alive
        self._model = model
        arr = _job_array(jobs)
        h = ctypes.c_void_p()
        _check(lib().kd_batch_create(arr, len(jobs), model.handle if model is not None else None, _opts(opts),
                                     _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def run(self, stream=None):
        _check(lib().kd_batch_run(self._h, _stream_handle(stream)))

    def info(self):
        """[(dim, list size, queries)] of the batch's (dimension, list size) groups."""
        n = ctypes.c_int()
        cap = 64
        dims, ks, qs = (ctypes.c_int * cap)(), (ctypes.c_int * cap)(), (ctypes.c_int64 * cap)()
        _check(lib().kd_batch_info(self._h, ctypes.byref(n), dims, ks, qs, cap))
        return [(dims[i], ks[i], qs[i]) for i in range(min(n.value, cap))]

    def autotune(self, reps=3, stream=None):
        """Times launch options per group, keeps the fastest; returns their options."""
        cap = 64
        arr = (KdOpts * cap)()
        n = ctypes.c_int(cap)
        _check(lib().kd_batch_autotune(self._h, int(reps), _stream_handle(stream), arr, ctypes.byref(n)))
        return [_opts_dict(arr[i]) for i in range(min(n.value, cap))]

    def close(self):
        if self._h:
            lib().kd_batch_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kd_knn_batched(jobs, opts=None, model=None, stream=None):
    arr = _job_array(jobs)
    _check(lib().kd_knn_batched(arr, len(jobs), model.handle if model is not None else None, _opts(opts),
                                _stream_handle(stream)))


def _opts_dict(o: KdOpts):
    return dict(block=o.block, lds_levels=o.lds_levels, sort_bits=o.sort_bits, waves_per_cu=o.waves_per_cu,
                heavy_trips=o.heavy_trips, prune=o.prune)


def kd_autotune(tree: Tree, sample_q, k, max_radius=math.inf, stream=None):
    """Tunes the launch options for (tree, k) on a sample; returns (opts dict, ms)."""
    import torch
    _require(sample_q, torch.float32, "sample_q")
    o = KdOpts()
    ms = ctypes.c_float()
    _check(lib().kd_autotune(tree.handle, _ptr(sample_q), sample_q.shape[0], int(k), float(max_radius),
                             ctypes.byref(o), ctypes.byref(ms), _stream_handle(stream)))
    return _opts_dict(o), ms.value


def kd_tree_get_tuned(tree: Tree, k):
    o = KdOpts()
    _check(lib().kd_tree_get_tuned(tree.handle, int(k), ctypes.byref(o)))
    return _opts_dict(o)


def kd_tree_set_tuned(tree: Tree, k, opts: dict):
    o = KdOpts(opts.get("block", 0), opts.get("lds_levels", -1), opts.get("sort_bits", -1),
               opts.get("waves_per_cu", 0), opts.get("heavy_trips", 0), opts.get("prune", 0))
    _check(lib().kd_tree_set_tuned(tree.handle, int(k), ctypes.byref(o)))


def save_tuning(tree: Tree, ks, path):
    """Writes the tuned options of the given k values to a JSON cache file."""
    import json
    out = {}
    for k in ks:
        try:
            out[str(k)] = kd_tree_get_tuned(tree, k)
        except KdError:
            pass
    with open(path, "w") as f:
        json.dump(out, f)


def load_tuning(tree: Tree, path):
    """Applies a JSON cache file written by save_tuning."""
    import json
    with open(path) as f:
        for k, o in json.load(f).items():
            kd_tree_set_tuned(tree, int(k), o)


def kd_timing_enable(on: bool = True):
    _check(lib().kd_timing_enable(1 if on else 0))


def kd_timing_collect(kernel: str = "traverse"):
    """(total milliseconds, launches) of the named kernel since the last collect."""
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(lib().kd_timing_collect(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return ms.value, n.value


def version() -> str:
    return lib().kd_version().decode()
