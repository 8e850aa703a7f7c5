"""ctypes wrapper around the plain-C oracle (oracle/ebc_ref.c).

Test infrastructure only. Inputs are NumPy arrays on the host; every result
is float64. Build the library first with ``oracle.build_ref.build()``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from .build_ref import LIB

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"oracle C library not built: {LIB} (run oracle.build_ref.build())")
        L = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        L.ebc_ref_threads.restype = ctypes.c_int
        ci = ctypes.c_int
        L.ebc_ref_min_dist.argtypes = [P, i64, i32, P, i64, P, P, ci]
        L.ebc_ref_gains.argtypes = [P, i64, i32, P, P, i64, P, ci]
        L.ebc_ref_eval_sets.argtypes = [P, i64, i32, P, P, i64, P, P, ci]
        L.ebc_ref_eval_sets_f32.argtypes = [P, i64, i32, P, P, i64, P, ctypes.c_int]
        L.ebc_ref_gains_f32.argtypes = [P, i64, i32, P, P, i64, P, ctypes.c_int]
        L.ebc_ref_greedy.argtypes = [P, i64, i32, i32, P, P, P, P, ci]
        L.ebc_ref_greedy.restype = ctypes.c_int
        L.ebc_ref_greedy_lazy.argtypes = [P, i64, i32, i32, P, P, P, P, P, ci]
        L.ebc_ref_greedy_lazy.restype = ctypes.c_int
        _lib = L
    return _lib


# dissimilarities: the squared Euclidean distance (the paper's experiments,
# Sec. 5) and the L1 distance (Sec. 4 defines f for any dissimilarity)
METRICS = {"sqeuclidean": 0, "l1": 1}


def _metric(dist: str) -> int:
    if dist not in METRICS:
        raise ValueError(f"dist must be one of {sorted(METRICS)}")
    return METRICS[dist]


def _f32(x):
    return np.ascontiguousarray(x, dtype=np.float32)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _e0(x, e0):
    """(keep-alive array, pointer) of the auxiliary vector; None = zero vector."""
    if e0 is None:
        return None, None
    a = np.ascontiguousarray(np.asarray(e0, dtype=np.float32).reshape(x.shape[1]))
    return a, _p(a)


def threads() -> int:
    return int(lib().ebc_ref_threads())


def min_dist(x, s_idx, e0=None, dist: str = "sqeuclidean") -> np.ndarray:
    x = _f32(x)
    s = np.ascontiguousarray(s_idx, dtype=np.int32)
    m = np.empty(x.shape[0])
    keep, pe = _e0(x, e0)
    lib().ebc_ref_min_dist(_p(x), x.shape[0], x.shape[1], _p(s), s.size, _p(m), pe, _metric(dist))
    return m


def gains(x, m, cand=None, dist: str = "sqeuclidean") -> np.ndarray:
    x = _f32(x)
    m = np.ascontiguousarray(m, dtype=np.float64)
    cand = np.arange(x.shape[0], dtype=np.int32) if cand is None else np.ascontiguousarray(cand, dtype=np.int32)
    out = np.empty(cand.size)
    lib().ebc_ref_gains(_p(x), x.shape[0], x.shape[1], _p(m), _p(cand), cand.size, _p(out), _metric(dist))
    return out


def eval_sets(x, offsets, idx, e0=None, dist: str = "sqeuclidean") -> np.ndarray:
    x = _f32(x)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.empty(off.size - 1)
    keep, pe = _e0(x, e0)
    lib().ebc_ref_eval_sets(_p(x), x.shape[0], x.shape[1], _p(off), _p(idx), off.size - 1, _p(out), pe,
                            _metric(dist))
    return out


def eval_sets_f32(x, offsets, idx, threads: int) -> np.ndarray:
    """Paper-style single-precision CPU baseline of eval_sets (timing only)."""
    x = _f32(x)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    out = np.empty(off.size - 1)
    lib().ebc_ref_eval_sets_f32(_p(x), x.shape[0], x.shape[1], _p(off), _p(idx), off.size - 1, _p(out), int(threads))
    return out


def gains_f32(x, m, cand, threads: int) -> np.ndarray:
    """Paper-style single-precision CPU baseline of gains (timing only)."""
    x = _f32(x)
    m = np.ascontiguousarray(m, dtype=np.float64)
    cand = np.ascontiguousarray(cand, dtype=np.int32)
    out = np.empty(cand.size)
    lib().ebc_ref_gains_f32(_p(x), x.shape[0], x.shape[1], _p(m), _p(cand), cand.size, _p(out), int(threads))
    return out


def greedy(x, k: int, e0=None, dist: str = "sqeuclidean"):
    x = _f32(x)
    sel = np.empty(k, dtype=np.int32)
    f = np.empty(k)
    g = np.empty(k)
    keep, pe = _e0(x, e0)
    rc = lib().ebc_ref_greedy(_p(x), x.shape[0], x.shape[1], int(k), _p(sel), _p(f), _p(g), pe, _metric(dist))
    if rc != 0:
        raise ValueError(f"ebc_ref_greedy failed ({rc})")
    return sel.astype(np.int64), f, g


def greedy_lazy(x, k: int, e0=None, dist: str = "sqeuclidean"):
    """Same result as greedy(), by lazy re-evaluation of stale upper bounds.
    Returns (sel, f, gain, gain evaluations)."""
    x = _f32(x)
    sel = np.empty(k, dtype=np.int32)
    f = np.empty(k)
    g = np.empty(k)
    ev = ctypes.c_int64(0)
    keep, pe = _e0(x, e0)
    rc = lib().ebc_ref_greedy_lazy(_p(x), x.shape[0], x.shape[1], int(k), _p(sel), _p(f), _p(g), ctypes.byref(ev),
                                   pe, _metric(dist))
    if rc != 0:
        raise ValueError(f"ebc_ref_greedy_lazy failed ({rc})")
    return sel.astype(np.int64), f, g, int(ev.value)
