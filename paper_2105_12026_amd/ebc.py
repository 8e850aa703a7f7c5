"""Thin ctypes binding of libebc.so (C ABI in include/ebc.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libebc.so. torch provides device memory (the dataset workspace
and the outputs) and the HIP stream; nothing here falls back to a CPU or
PyTorch computation. If the library is missing the import of this module
raises, so a product call can never run without the native code.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

import torch  # loads the process's HIP runtime before libebc.so binds to it

__all__ = ["EBCError", "Dataset", "Batch", "Server", "Arena", "request_bytes", "lib", "status_string", "DTYPES", "DISTS",
           "LIB_PATH", "ABI_FUNCTIONS"]

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libebc.so")
DTYPES = {"f32": 0, "f16": 1, "bf16": 2, "fp8": 3}
# dissimilarity -> ebc_dataset_create flags (EBC_FLAG_L1 = 1)
DISTS = {"sqeuclidean": 0, "l1": 1}
MAX_DIM = 4096  # EBC_MAX_DIM of include/ebc.h
FIXED_SCRATCH_BYTES = 16 << 20  # EBC_FIXED_SCRATCH_BYTES of include/ebc.h
ABI_FUNCTIONS = (
    "ebc_dataset_bytes", "ebc_dataset_create", "ebc_dataset_destroy", "ebc_eval_sets_bytes", "ebc_eval_sets",
    "ebc_eval_sets_in_dtype", "ebc_marginal_gains", "ebc_greedy", "ebc_three_sieves_bytes", "ebc_three_sieves",
    "ebc_sieve_streaming_bytes", "ebc_sieve_streaming", "ebc_sync_status",
    "ebc_status_string",
    "ebc_dataset_get_info", "ebc_dataset_set_e0", "ebc_profile_enable", "ebc_profile_read", "ebc_set_gains_variant",
    "ebc_gains_variant_count", "ebc_set_greedy_graph", "ebc_batch_bytes", "ebc_batch_create",
    "ebc_batch_destroy", "ebc_batch_set_graph", "ebc_greedy_batched", "ebc_batch_info", "ebc_autotune",
    "ebc_tune_cache_load", "ebc_tune_cache_save", "ebc_tune_cache_size", "ebc_request_bytes",
    "ebc_server_create", "ebc_server_destroy", "ebc_server_submit", "ebc_server_step", "ebc_server_poll",
    "ebc_server_stats", "ebc_server_now", "ebc_arena_create", "ebc_arena_alloc", "ebc_arena_free",
    "ebc_arena_free_bytes", "ebc_arena_largest_free", "ebc_arena_destroy", "ebc_eval_sets_noalloc",
)
_NON_STATUS = ("ebc_dataset_bytes", "ebc_eval_sets_bytes", "ebc_three_sieves_bytes", "ebc_sieve_streaming_bytes",
               "ebc_status_string", "ebc_batch_bytes", "ebc_request_bytes", "ebc_server_now",
               "ebc_arena_free_bytes", "ebc_arena_largest_free", "ebc_tune_cache_size")


class EBCError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {status_string(code)} (status {code})")
        self.code = code


class _Stats(ctypes.Structure):
    _fields_ = [("window_max", ctypes.c_int32), ("window_overflow", ctypes.c_int32),
                ("steps", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class _Info(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("n_pad", ctypes.c_int64), ("d", ctypes.c_int32),
                ("k_pad", ctypes.c_int32), ("v_splits", ctypes.c_int32), ("cand_tile", ctypes.c_int32),
                ("window_cap", ctypes.c_int32), ("dtype", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("reserved", ctypes.c_int32), ("l0", ctypes.c_double)]


class _Profile(ctypes.Structure):
    _fields_ = [("gains_ms", ctypes.c_double), ("select_ms", ctypes.c_double),
                ("gains_launches", ctypes.c_int32), ("steps", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libebc.so is not built ({LIB_PATH}); run `python -m paper_2105_12026_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
        L.ebc_dataset_bytes.argtypes = [i64, i32, ctypes.c_int]
        L.ebc_dataset_bytes.restype = ctypes.c_size_t
        L.ebc_dataset_create.argtypes = [P, i64, i32, ctypes.c_int, u32, P, ctypes.c_size_t, P,
                                         ctypes.POINTER(P)]
        L.ebc_dataset_destroy.argtypes = [P]
        sz = ctypes.c_size_t
        L.ebc_eval_sets_bytes.argtypes = [i64, i64]
        L.ebc_eval_sets_bytes.restype = sz
        L.ebc_eval_sets.argtypes = [P, P, P, i64, P, P, sz, P]
        L.ebc_eval_sets_in_dtype.argtypes = [P, P, P, i64, P, P, sz, P]
        L.ebc_eval_sets_noalloc.argtypes = [P, P, P, i64, P, i32, P]
        L.ebc_three_sieves_bytes.argtypes = [i64, i32, ctypes.c_double, i64, i32]
        L.ebc_three_sieves_bytes.restype = sz
        L.ebc_sieve_streaming_bytes.argtypes = [i64, i32, ctypes.c_double, i64, i32]
        L.ebc_sieve_streaming_bytes.restype = sz
        L.ebc_marginal_gains.argtypes = [P, P, P, i64, P, P]
        L.ebc_greedy.argtypes = [P, i32, P, P, P, P]
        L.ebc_three_sieves.argtypes = [P, i32, ctypes.c_double, i64, ctypes.c_double, P, i64, i32, P, P,
                                       ctypes.POINTER(i32), ctypes.POINTER(i64), P, sz, P]
        L.ebc_sieve_streaming.argtypes = [P, i32, ctypes.c_double, ctypes.c_double, P, i64, i32, P, P,
                                          ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double),
                                          ctypes.POINTER(i64), P, sz, P]
        L.ebc_sync_status.argtypes = [P, P, ctypes.POINTER(_Stats)]
        L.ebc_status_string.argtypes = [ctypes.c_int]
        L.ebc_status_string.restype = ctypes.c_char_p
        L.ebc_dataset_get_info.argtypes = [P, ctypes.POINTER(_Info)]
        L.ebc_profile_enable.argtypes = [P, i32]
        L.ebc_set_gains_variant.argtypes = [P, i32]
        L.ebc_dataset_set_e0.argtypes = [P, P, P]
        L.ebc_set_greedy_graph.argtypes = [P, i32]
        L.ebc_gains_variant_count.argtypes = [ctypes.c_int]
        L.ebc_profile_read.argtypes = [P, ctypes.POINTER(_Profile), i32]
        L.ebc_batch_bytes.argtypes = [i32]
        L.ebc_batch_bytes.restype = ctypes.c_size_t
        L.ebc_batch_create.argtypes = [P, i32, P, ctypes.c_size_t, P, ctypes.POINTER(P)]
        L.ebc_batch_destroy.argtypes = [P]
        L.ebc_batch_set_graph.argtypes = [P, i32]
        L.ebc_greedy_batched.argtypes = [P, P, P, P, P, P]
        L.ebc_batch_info.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(i64)]
        L.ebc_autotune.argtypes = [P, i32, i32, P, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_float)]
        L.ebc_tune_cache_load.argtypes = [ctypes.c_char_p]
        L.ebc_tune_cache_save.argtypes = [ctypes.c_char_p]
        L.ebc_tune_cache_size.argtypes = []
        L.ebc_request_bytes.argtypes = [i64, i32, i32, ctypes.c_int]
        L.ebc_request_bytes.restype = ctypes.c_size_t
        L.ebc_server_create.argtypes = [P, ctypes.c_size_t, i32, P, ctypes.POINTER(P)]
        L.ebc_server_destroy.argtypes = [P]
        L.ebc_server_submit.argtypes = [P, P, i64, i32, i32, ctypes.c_int, ctypes.c_double, ctypes.POINTER(i64)]
        L.ebc_server_step.argtypes = [P, ctypes.POINTER(i32)]
        dp = ctypes.POINTER(ctypes.c_double)
        L.ebc_server_poll.argtypes = [P, i64, ctypes.POINTER(i32), P, P, P, dp, dp, dp]
        L.ebc_server_stats.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64),
                                       ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_size_t)]
        L.ebc_server_now.argtypes = []
        L.ebc_server_now.restype = ctypes.c_double
        L.ebc_arena_create.argtypes = [ctypes.c_size_t, ctypes.POINTER(P)]
        L.ebc_arena_alloc.argtypes = [P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]
        L.ebc_arena_free.argtypes = [P, ctypes.c_size_t]
        L.ebc_arena_free_bytes.argtypes = [P]
        L.ebc_arena_free_bytes.restype = ctypes.c_size_t
        L.ebc_arena_largest_free.argtypes = [P]
        L.ebc_arena_largest_free.restype = ctypes.c_size_t
        L.ebc_arena_destroy.argtypes = [P]
        for name in ABI_FUNCTIONS:
            if name not in _NON_STATUS:
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def status_string(code: int) -> str:
    return lib().ebc_status_string(int(code)).decode()


def _check(code: int, what: str):
    if code != 0:
        raise EBCError(code, what)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _stream(stream) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _scratch(nbytes: int, device, stream=None) -> torch.Tensor:
    """Caller-owned device scratch for one call (torch's allocator is 256-byte
    aligned; at least one byte so the pointer is never NULL). With an explicit
    stream the block is recorded on it, so the caching allocator reuses it
    only after that stream's work."""
    t = torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)
    if stream is not None:
        t.record_stream(stream)
    return t


class Dataset:
    """A ground set V resident on the GPU (ebc_dataset_create).

    ``x`` is a float32 CUDA tensor [n, d]; it is kept alive by this object
    because the library borrows it. The workspace is a uint8 CUDA tensor of
    exactly ``ebc_dataset_bytes(n, d, dtype)`` bytes."""

    def __init__(self, x: torch.Tensor, dtype: str = "f32", stream=None, dist: str = "sqeuclidean"):
        if not (isinstance(x, torch.Tensor) and x.is_cuda and x.dtype == torch.float32 and x.dim() == 2):
            raise TypeError("x must be a float32 CUDA tensor of shape [n, d]")
        self.x = x.contiguous()
        self.n, self.d = map(int, self.x.shape)
        self.dtype = dtype
        self.dist = dist
        L = lib()
        if dtype not in DTYPES:
            raise ValueError(f"dtype must be one of {sorted(DTYPES)}")
        if dist not in DISTS:
            raise ValueError(f"dist must be one of {sorted(DISTS)}")
        nbytes = L.ebc_dataset_bytes(self.n, self.d, DTYPES[dtype])
        if nbytes == 0:
            raise EBCError(1 if self.d <= MAX_DIM else 7, f"ebc_dataset_bytes(n={self.n}, d={self.d})")
        self.workspace_bytes = int(nbytes)
        self.workspace = torch.empty(self.workspace_bytes, dtype=torch.uint8, device=self.x.device)
        h = ctypes.c_void_p()
        _check(L.ebc_dataset_create(_ptr(self.x), self.n, self.d, DTYPES[dtype], DISTS[dist], _ptr(self.workspace),
                                    self.workspace_bytes, _stream(stream), ctypes.byref(h)),
               "ebc_dataset_create")
        self._h = h

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            lib().ebc_dataset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> ctypes.c_void_p:
        return self._h

    # -- entry points -----------------------------------------------------
    def sync(self, stream=None) -> dict:
        st = _Stats()
        _check(lib().ebc_sync_status(self._h, _stream(stream), ctypes.byref(st)), "ebc_sync_status")
        return {"window_max": st.window_max, "window_overflow": st.window_overflow, "steps": st.steps}

    def info(self) -> dict:
        inf = _Info()
        _check(lib().ebc_dataset_get_info(self._h, ctypes.byref(inf)), "ebc_dataset_get_info")
        return {f: getattr(inf, f) for f, _ in _Info._fields_}

    def set_e0(self, e0=None, stream=None):
        """Auxiliary vector e0 of f (ebc_dataset_set_e0): a float32 CUDA
        tensor [d], or None for the origin. Resets the greedy state."""
        if e0 is not None:
            if not (isinstance(e0, torch.Tensor) and e0.is_cuda and e0.dtype == torch.float32
                    and e0.numel() == self.d):
                raise TypeError("e0 must be a float32 CUDA tensor with d elements")
            e0 = e0.contiguous()
        self._e0 = e0  # kept alive until the stream work has read it
        _check(lib().ebc_dataset_set_e0(self._h, None if e0 is None else _ptr(e0), _stream(stream)),
               "ebc_dataset_set_e0")

    def set_variant(self, variant: int):
        """Tile shape of the gains kernel (results are identical across variants)."""
        _check(lib().ebc_set_gains_variant(self._h, int(variant)), "ebc_set_gains_variant")

    def set_graph(self, on: bool = True):
        """Record greedy runs into a HIP graph and replay it (identical results)."""
        _check(lib().ebc_set_greedy_graph(self._h, int(bool(on))), "ebc_set_greedy_graph")

    @staticmethod
    def variant_count(dtype: str) -> int:
        return int(lib().ebc_gains_variant_count(DTYPES[dtype]))

    def autotune(self, reps: int = 3, force: bool = False, stream=None) -> dict:
        """Pick the fastest gains tile variant for this dataset's (dtype, row
        length, size bucket), from the tuning table or by timing (blocking)."""
        nv = self.variant_count(self.dtype)
        v = ctypes.c_int32(-1)
        times = (ctypes.c_float * nv)(*([float("nan")] * nv))
        _check(lib().ebc_autotune(self._h, int(reps), int(bool(force)), _stream(stream), ctypes.byref(v), times),
               "ebc_autotune")
        return {"variant": v.value, "times_ms": list(times)}

    def profile(self, on: bool = True):
        """Turn per-step HIP-event timing of greedy on or off."""
        _check(lib().ebc_profile_enable(self._h, int(bool(on))), "ebc_profile_enable")

    def profile_read(self, reset: bool = True) -> dict:
        pr = _Profile()
        _check(lib().ebc_profile_read(self._h, ctypes.byref(pr), int(bool(reset))), "ebc_profile_read")
        return {f: getattr(pr, f) for f, _ in _Profile._fields_}

    def eval_sets_bytes(self, l: int) -> int:
        """Device scratch of one eval_sets call over l sets (ebc_eval_sets_bytes)."""
        return int(lib().ebc_eval_sets_bytes(self.n, int(l)))

    def eval_sets(self, offsets: torch.Tensor, idx: torch.Tensor, out: torch.Tensor | None = None,
                  stream=None, in_dtype: bool = False, scratch: torch.Tensor | None = None) -> torch.Tensor:
        """f(S_j) for CSR sets (offsets int64 [l+1], idx int32 [nnz]); float64 [l].
        in_dtype: dot products in the dataset's distance dtype instead of float32.
        scratch: a uint8 CUDA tensor of at least eval_sets_bytes(l) bytes to use
        instead of a fresh one."""
        offsets = offsets.to(device=self.x.device, dtype=torch.int64).contiguous()
        idx = idx.to(device=self.x.device, dtype=torch.int32).contiguous()
        l = offsets.numel() - 1
        if out is None:
            out = torch.empty(max(l, 0), dtype=torch.float64, device=self.x.device)
        idx_arg = idx if idx.numel() > 0 else offsets  # any valid pointer when there are no members
        fn = lib().ebc_eval_sets_in_dtype if in_dtype else lib().ebc_eval_sets
        if scratch is None:
            scratch = _scratch(lib().ebc_eval_sets_bytes(self.n, max(l, 0)), self.x.device, stream)
        _check(fn(self._h, _ptr(offsets), _ptr(idx_arg), l, _ptr(out), _ptr(scratch), scratch.numel(),
                  _stream(stream)), "ebc_eval_sets")
        return out

    def eval_sets_noalloc(self, offsets: torch.Tensor, idx: torch.Tensor, out: torch.Tensor,
                          stream=None, in_dtype: bool = False) -> torch.Tensor:
        """f(S_j) as eval_sets, with the library's fixed device scratch instead of a
        caller one (ebc_eval_sets_noalloc); ``out`` (float64 [l]) is required, and
        offsets/idx must already be int64/int32 contiguous tensors on the device."""
        for t, dt in ((offsets, torch.int64), (idx, torch.int32), (out, torch.float64)):
            if t.dtype != dt or t.device != self.x.device or not t.is_contiguous():
                raise ValueError(f"eval_sets_noalloc: expected a contiguous {dt} tensor on {self.x.device}")
        l = offsets.numel() - 1
        if out.numel() < max(l, 0):
            raise ValueError("eval_sets_noalloc: out holds fewer than l values")
        idx_arg = idx if idx.numel() > 0 else offsets  # any valid pointer when there are no members
        _check(lib().ebc_eval_sets_noalloc(self._h, _ptr(offsets), _ptr(idx_arg), l, _ptr(out),
                                           1 if in_dtype else 0, _stream(stream)), "ebc_eval_sets_noalloc")
        return out

    def marginal_gains(self, m: torch.Tensor | None = None, cand: torch.Tensor | None = None,
                       out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """Delta(c|S) for candidates (default all n). ``m`` (float64 [n]) replaces the running minima."""
        if m is not None:
            m = m.to(device=self.x.device, dtype=torch.float64).contiguous()
        if cand is not None:
            cand = cand.to(device=self.x.device, dtype=torch.int32).contiguous()
        nc = self.n if cand is None else cand.numel()
        if out is None:
            out = torch.empty(nc, dtype=torch.float64, device=self.x.device)
        _check(lib().ebc_marginal_gains(self._h, _ptr(m), _ptr(cand), nc, _ptr(out), _stream(stream)),
               "ebc_marginal_gains")
        return out

    def three_sieves(self, k: int, eps: float, T: int, m_max: float = 0.0, order=None, batch: int = 0,
                     stream=None):
        """Three Sieves over a stream of points (ebc_three_sieves). Returns
        (accepted indices int32, f after each acceptance float64, points examined)."""
        dev = self.x.device
        if order is not None:
            order = order.to(device=dev, dtype=torch.int32).contiguous()
        n_order = self.n if order is None else order.numel()
        sel = torch.empty(k, dtype=torch.int32, device=dev)
        f = torch.empty(k, dtype=torch.float64, device=dev)
        cnt = ctypes.c_int32(0)
        seen = ctypes.c_int64(0)
        nb = int(lib().ebc_three_sieves_bytes(self.n, int(k), float(eps), n_order, int(batch)))
        scratch = _scratch(nb, dev, stream)
        _check(lib().ebc_three_sieves(self._h, int(k), float(eps), int(T), float(m_max), _ptr(order), n_order,
                                      int(batch), _ptr(sel), _ptr(f), ctypes.byref(cnt), ctypes.byref(seen),
                                      _ptr(scratch), nb, _stream(stream)), "ebc_three_sieves")
        return sel[:cnt.value], f[:cnt.value], int(seen.value)

    def sieve_streaming(self, k: int, eps: float, m_max: float = 0.0, order=None, batch: int = 0, stream=None):
        """Sieve Streaming over a stream of points (ebc_sieve_streaming). Returns
        (best summary int32, f after each of its acceptances float64, its guess v,
        points examined)."""
        dev = self.x.device
        if order is not None:
            order = order.to(device=dev, dtype=torch.int32).contiguous()
        n_order = self.n if order is None else order.numel()
        sel = torch.empty(k, dtype=torch.int32, device=dev)
        f = torch.empty(k, dtype=torch.float64, device=dev)
        cnt = ctypes.c_int32(0)
        v = ctypes.c_double(0.0)
        seen = ctypes.c_int64(0)
        nb = int(lib().ebc_sieve_streaming_bytes(self.n, int(k), float(eps), n_order, int(batch)))
        scratch = _scratch(nb, dev, stream)
        _check(lib().ebc_sieve_streaming(self._h, int(k), float(eps), float(m_max), _ptr(order), n_order,
                                         int(batch), _ptr(sel), _ptr(f), ctypes.byref(cnt), ctypes.byref(v),
                                         ctypes.byref(seen), _ptr(scratch), nb, _stream(stream)),
               "ebc_sieve_streaming")
        return sel[:cnt.value], f[:cnt.value], float(v.value), int(seen.value)

    def greedy(self, k: int, stream=None, sel=None, f=None, gain=None):
        """Greedy to cardinality k on the device; returns (sel int32 [k], f float64 [k], gain float64 [k])."""
        dev = self.x.device
        sel = torch.empty(k, dtype=torch.int32, device=dev) if sel is None else sel
        f = torch.empty(k, dtype=torch.float64, device=dev) if f is None else f
        gain = torch.empty(k, dtype=torch.float64, device=dev) if gain is None else gain
        _check(lib().ebc_greedy(self._h, int(k), _ptr(sel), _ptr(f), _ptr(gain), _stream(stream)), "ebc_greedy")
        return sel, f, gain


def tune_cache_load(path: str) -> bool:
    return lib().ebc_tune_cache_load(path.encode()) == 0


def tune_cache_save(path: str):
    _check(lib().ebc_tune_cache_save(path.encode()), "ebc_tune_cache_save")


def tune_cache_size() -> int:
    return int(lib().ebc_tune_cache_size())


class Batch:
    """Many datasets advanced together by ebc_greedy_batched (one launch per
    kernel bucket and stage per step tick). Results equal solo runs bitwise."""

    def __init__(self, datasets, stream=None):
        self.datasets = list(datasets)
        if not self.datasets:
            raise ValueError("empty batch")
        n = len(self.datasets)
        L = lib()
        dev = self.datasets[0].x.device
        self.workspace = torch.empty(int(L.ebc_batch_bytes(n)), dtype=torch.uint8, device=dev)
        handles = (ctypes.c_void_p * n)(*[d.handle.value for d in self.datasets])
        h = ctypes.c_void_p()
        _check(L.ebc_batch_create(ctypes.cast(handles, ctypes.c_void_p), n, _ptr(self.workspace),
                                  self.workspace.numel(), _stream(stream), ctypes.byref(h)), "ebc_batch_create")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().ebc_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_graph(self, on: bool = True):
        _check(lib().ebc_batch_set_graph(self._h, int(bool(on))), "ebc_batch_set_graph")

    def info(self) -> dict:
        b, w, r = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().ebc_batch_info(self._h, ctypes.byref(b), ctypes.byref(w), ctypes.byref(r)), "ebc_batch_info")
        return {"buckets": b.value, "gains_workgroups_per_tick": w.value, "row_blocks_per_tick": r.value}

    def greedy(self, ks, stream=None, outs=None):
        """Greedy on every dataset; ks[i] steps for dataset i. Returns a list
        of (sel int32 [k], f float64 [k], gain float64 [k]) per dataset."""
        n = len(self.datasets)
        if len(ks) != n:
            raise ValueError("one k per dataset")
        if outs is None:
            outs = []
            for d, k in zip(self.datasets, ks):
                dev = d.x.device
                outs.append((torch.empty(max(k, 1), dtype=torch.int32, device=dev),
                             torch.empty(max(k, 1), dtype=torch.float64, device=dev),
                             torch.empty(max(k, 1), dtype=torch.float64, device=dev)))
        karr = (ctypes.c_int32 * n)(*[int(k) for k in ks])
        sel = (ctypes.c_void_p * n)(*[o[0].data_ptr() for o in outs])
        f = (ctypes.c_void_p * n)(*[o[1].data_ptr() for o in outs])
        g = (ctypes.c_void_p * n)(*[o[2].data_ptr() for o in outs])
        _check(lib().ebc_greedy_batched(self._h, ctypes.cast(karr, ctypes.c_void_p), ctypes.cast(sel, ctypes.c_void_p),
                                        ctypes.cast(f, ctypes.c_void_p), ctypes.cast(g, ctypes.c_void_p),
                                        _stream(stream)), "ebc_greedy_batched")
        return [(o[0][:k], o[1][:k], o[2][:k]) for o, k in zip(outs, ks)]


def request_bytes(n: int, d: int, k: int, dtype: str = "bf16") -> int:
    """Device bytes one serving request occupies in the arena (0 if invalid)."""
    return int(lib().ebc_request_bytes(int(n), int(d), int(k), DTYPES[dtype]))


class Arena:
    """The serving core's first-fit allocator bookkeeping (host only)."""

    def __init__(self, capacity: int):
        h = ctypes.c_void_p()
        _check(lib().ebc_arena_create(int(capacity), ctypes.byref(h)), "ebc_arena_create")
        self._h = h

    def alloc(self, nbytes: int):
        """Offset of a new block of nbytes (rounded up to 256), or None when nothing fits."""
        off = ctypes.c_size_t()
        rc = lib().ebc_arena_alloc(self._h, int(nbytes), ctypes.byref(off))
        if rc == 5:  # EBC_E_NOMEM
            return None
        _check(rc, "ebc_arena_alloc")
        return int(off.value)

    def free(self, offset: int):
        _check(lib().ebc_arena_free(self._h, int(offset)), "ebc_arena_free")

    @property
    def free_bytes(self) -> int:
        return int(lib().ebc_arena_free_bytes(self._h))

    @property
    def largest_free(self) -> int:
        return int(lib().ebc_arena_largest_free(self._h))

    def close(self):
        if getattr(self, "_h", None):
            lib().ebc_arena_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SERVER_STATES = ("queued", "active", "done", "failed")


class Server:
    """Request loop with continuous batching at greedy-step granularity
    (ebc_server_*). Requests live in one device arena of ``arena_bytes``,
    admitted first-come first-served while a slot is free and their footprint
    fits; each ``step()`` advances every active request by one greedy step."""

    def __init__(self, arena_bytes: int, max_slots: int = 64, device="cuda", stream=None):
        self.arena_bytes = int(arena_bytes)
        self.max_slots = int(max_slots)
        self.arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=device)
        self._stream = stream
        h = ctypes.c_void_p()
        _check(lib().ebc_server_create(_ptr(self.arena), self.arena_bytes, self.max_slots, _stream(stream),
                                       ctypes.byref(h)), "ebc_server_create")
        self._h = h
        self._k = {}

    def close(self):
        if getattr(self, "_h", None):
            lib().ebc_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def now() -> float:
        return float(lib().ebc_server_now())

    def submit(self, x, k: int, dtype: str = "bf16", t_arrival: float = -1.0) -> int:
        """Queue a request (x: float32 host array [n, d], copied). Returns its id."""
        x = np.ascontiguousarray(x, dtype=np.float32)
        if x.ndim != 2:
            raise ValueError("x must be [n, d]")
        rid = ctypes.c_int64()
        _check(lib().ebc_server_submit(self._h, ctypes.c_void_p(x.ctypes.data), x.shape[0], x.shape[1], int(k),
                                       DTYPES[dtype], float(t_arrival), ctypes.byref(rid)), "ebc_server_submit")
        self._k[rid.value] = int(k)
        return int(rid.value)

    def step(self) -> int:
        """One scheduler tick; returns how many requests completed in it."""
        c = ctypes.c_int32()
        _check(lib().ebc_server_step(self._h, ctypes.byref(c)), "ebc_server_step")
        return int(c.value)

    def poll(self, rid: int) -> dict:
        k = self._k[rid]
        st = ctypes.c_int32()
        sel = np.empty(k, np.int32)
        f = np.empty(k, np.float64)
        g = np.empty(k, np.float64)
        ta, tb, tc = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        rc = lib().ebc_server_poll(self._h, int(rid), ctypes.byref(st), ctypes.c_void_p(sel.ctypes.data),
                                   ctypes.c_void_p(f.ctypes.data), ctypes.c_void_p(g.ctypes.data), ctypes.byref(ta),
                                   ctypes.byref(tb), ctypes.byref(tc))
        out = {"state": SERVER_STATES[st.value], "status": int(rc), "t_arrive": ta.value, "t_admit": tb.value,
               "t_done": tc.value}
        if st.value == 2:
            out.update(sel=sel, f=f, gain=g)
        return out

    def stats(self) -> dict:
        q, a = ctypes.c_int32(), ctypes.c_int32()
        c, t = ctypes.c_int64(), ctypes.c_int64()
        fb = ctypes.c_size_t()
        _check(lib().ebc_server_stats(self._h, ctypes.byref(q), ctypes.byref(a), ctypes.byref(c), ctypes.byref(t),
                                      ctypes.byref(fb)), "ebc_server_stats")
        return {"queued": q.value, "active": a.value, "completed": c.value, "ticks": t.value,
                "free_bytes": int(fb.value)}
