"""Host-only checks of the C ABI (no GPU): the library loads, exports every
function include/ebc.h declares, and rejects bad arguments on the host before
touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ebc.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"EBC_API\s+[\w\s\*]+?\b(ebc_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    from paper_2105_12026_amd import ebc
    if not os.path.exists(ebc.LIB_PATH):
        from paper_2105_12026_amd import build
        build.build()
    return ebc.lib()


def test_header_declares_the_binding_functions():
    from paper_2105_12026_amd import ebc
    assert _declared() == sorted(ebc.ABI_FUNCTIONS)


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_status_strings(L):
    from paper_2105_12026_amd import ebc
    assert ebc.status_string(0) == "ok"
    for code in range(1, 8):
        assert ebc.status_string(code) != "unknown status"
    assert ebc.status_string(99) == "unknown status"


def test_workspace_size_is_exact_and_monotone(L):
    a = L.ebc_dataset_bytes(1000, 16, 0)
    b = L.ebc_dataset_bytes(100000, 100, 0)
    assert 0 < a < b
    assert a % 256 == 0 and b % 256 == 0
    # the padded float32 copy alone is n_pad * k_pad * 4 bytes
    assert b >= 100096 * 104 * 4
    assert L.ebc_dataset_bytes(0, 16, 0) == 0
    assert L.ebc_dataset_bytes(10, 0, 0) == 0
    assert L.ebc_dataset_bytes(10, 129, 0) > 0      # long rows are supported ...
    assert L.ebc_dataset_bytes(10, 4096, 3) > 0
    assert L.ebc_dataset_bytes(10, 4097, 0) == 0     # ... up to EBC_MAX_DIM
    assert L.ebc_dataset_bytes(10, 16, 9) == 0


def test_host_validation_without_device(L):
    P = ctypes.c_void_p
    h = P()
    # null x, null workspace, bad flags, bad dtype: rejected before any HIP call
    assert L.ebc_dataset_create(None, 10, 4, 0, 0, P(256), 1 << 20, None, ctypes.byref(h)) == 1
    assert L.ebc_dataset_create(P(256), 10, 4, 0, 0, None, 1 << 20, None, ctypes.byref(h)) == 1
    assert L.ebc_dataset_create(P(256), 10, 4, 0, 2, P(256), 1 << 20, None, ctypes.byref(h)) == 1  # unknown flag
    assert L.ebc_dataset_create(P(256), 10, 4, 2, 1, P(256), 1 << 20, None, ctypes.byref(h)) == 7  # L1 needs FP32
    assert L.ebc_dataset_create(P(256), 10, 4, 5, 0, P(256), 1 << 20, None, ctypes.byref(h)) == 1
    assert L.ebc_dataset_create(P(256), 10, 5000, 0, 0, P(256), 1 << 30, None, ctypes.byref(h)) == 7
    assert L.ebc_dataset_create(P(256), 10, 4, 0, 0, P(128), 1 << 20, None, ctypes.byref(h)) == 1  # misaligned
    assert L.ebc_dataset_create(P(256), 10, 4, 0, 0, P(256), 16, None, ctypes.byref(h)) == 1  # too small
    assert L.ebc_dataset_create(P(256), 10, 4, 0, 0, P(256), 1 << 20, None, None) == 1
    assert not h.value
    assert L.ebc_dataset_destroy(None) == 1
    assert L.ebc_greedy(None, 1, None, None, None, None) == 1
    assert L.ebc_eval_sets(None, None, None, 1, None, P(256), 1 << 20, None) == 1
    assert L.ebc_eval_sets_in_dtype(None, None, None, 1, None, P(256), 1 << 20, None) == 1
    assert L.ebc_marginal_gains(None, None, None, 1, None, None) == 1
    assert L.ebc_sync_status(None, None, None) == 1
    assert L.ebc_dataset_set_e0(None, None, None) == 1
    cnt, seen, v = ctypes.c_int32(7), ctypes.c_int64(7), ctypes.c_double(7.0)
    assert L.ebc_three_sieves(None, 3, 0.1, 5, 0.0, None, 10, 0, P(256), P(256), ctypes.byref(cnt),
                              ctypes.byref(seen), P(256), 1 << 20, None) == 1
    assert L.ebc_sieve_streaming(None, 3, 0.1, 0.0, None, 10, 0, P(256), P(256), ctypes.byref(cnt),
                                 ctypes.byref(v), ctypes.byref(seen), P(256), 1 << 20, None) == 1


def test_scratch_size_queries(L):
    """The calls that need device scratch take it from the caller; their size
    queries are host arithmetic (no dataset, no device)."""
    # multi-set evaluation: unit counts (8 + 4 + 4 bytes per set) + float64 partial
    # sums per ground-set split (ceil(n / 256) splits, at most 16), 256-byte pieces
    a = L.ebc_eval_sets_bytes(50000, 5000)
    assert a % 256 == 0
    assert a >= 5000 * (20 + 8 * 16)
    assert a <= 5000 * (20 + 8 * 16) + 6 * 256 + 8
    assert L.ebc_eval_sets_bytes(300, 5000) < a            # two splits instead of 16
    assert L.ebc_eval_sets_bytes(1000, 0) > 0               # the per-call counters
    assert L.ebc_eval_sets_bytes(0, 10) == 0
    assert L.ebc_eval_sets_bytes(1000, -1) == 0
    assert L.ebc_eval_sets_bytes(1000, 2 * 10 ** 6) > L.ebc_eval_sets_bytes(1000, 10 ** 6)
    # Three Sieves: one stretch of float64 distance rows (1000 stream points x
    # n_pad 1024), the float64 minima, the summary state, the guesses
    k, eps, n = 50, 0.1, 1000
    guesses = int(__import__("math").floor(__import__("math").log(k) / __import__("math").log1p(eps))) + 2
    t = L.ebc_three_sieves_bytes(n, k, eps, n, 0)
    assert t % 256 == 0
    assert n * 1024 * 8 + 1024 * 8 + guesses * 8 <= t <= n * 1024 * 8 + 1024 * 8 + guesses * 8 + 4 * 256
    assert L.ebc_three_sieves_bytes(n, k, eps, n, 64) < t      # a shorter stretch
    assert L.ebc_three_sieves_bytes(n, k, eps, 100, 0) < t     # a stream shorter than the default stretch
    assert L.ebc_three_sieves_bytes(0, k, eps, 10, 0) == 0
    assert L.ebc_three_sieves_bytes(100, k, eps, -1, 0) == 0
    assert L.ebc_three_sieves_bytes(100, 0, eps, 10, 0) == 0
    assert L.ebc_three_sieves_bytes(100, k, 0.0, 10, 0) == 0
    # Sieve Streaming: the same stretch, and per guess (at most
    # floor(log k / log(1+eps)) + 2) its minima, k members, k f values, state
    s = L.ebc_sieve_streaming_bytes(n, k, eps, n, 0)
    need = n * 1024 * 8 + guesses * (1024 * 8 + k * 4 + k * 8 + 32) + guesses * 8
    assert need <= s < need + 7 * 256
    assert L.ebc_sieve_streaming_bytes(n, k, 0.5, n, 0) < s   # fewer guesses
    assert L.ebc_sieve_streaming_bytes(n, 0, eps, n, 0) == 0
    assert L.ebc_sieve_streaming_bytes(n, n + 1, eps, n, 0) == 0
    assert L.ebc_sieve_streaming_bytes(n, k, 0.0, n, 0) == 0


def test_no_device_allocation_in_the_library():
    """Every device buffer comes from the caller: no source of the library
    calls the HIP allocator."""
    csrc = os.path.join(ROOT, "paper_2105_12026_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        text = open(os.path.join(csrc, name)).read()
        for call in ("hipMalloc(", "hipMallocAsync(", "hipMallocManaged(", "hipExtMallocWithFlags(",
                     "hipMallocPitch(", "hipMalloc3D(", "hipMallocFromPoolAsync("):
            assert call not in text, (name, call)
