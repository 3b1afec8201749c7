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


class KdOpts(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int), ("lds_levels", ctypes.c_int),
                ("sort_bits", ctypes.c_int), ("waves_per_cu", ctypes.c_int)]


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
        "kd_build_host": ([P, i64, i32, P], i32),
        "kd_build_order_host": ([P, i64, i32, P], i32),
        "kd_tree_free": ([P], i32),
        "kd_tree_info": ([P, P, P, P, P], i32),
        "kd_tree_order": ([P, P], i32),
        "kd_fcp": ([P, P, i64, f32, P, P, P], i32),
        "kd_knn": ([P, P, i64, i32, f32, P, P, P], i32),
        "kd_knn_ex": ([P, P, i64, i32, f32, P, P, P, P, P], i32),
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

    def close(self):
        if self._h:
            lib().kd_tree_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def kd_build(points, stream=None) -> Tree:
    """Canonical left-balanced tree over device float32 points [N][dim]."""
    import torch
    _require(points, torch.float32, "points")
    if points.dim() != 2:
        raise ValueError("points must be [N][dim]")
    h = ctypes.c_void_p()
    _check(lib().kd_build(_ptr(points), points.shape[0], points.shape[1], _stream_handle(stream),
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
               opts.get("waves_per_cu", 0))
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
