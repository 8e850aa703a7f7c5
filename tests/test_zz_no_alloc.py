"""ebc_eval_sets_noalloc (the library's fixed device scratch, no allocation)
against ebc_eval_sets / ebc_eval_sets_in_dtype (caller scratch), through the
C ABI: two calls in a row on one device, the second with a smaller input, so
the second call runs over the first call's leftover scratch contents.

Bar: bitwise equal to the caller-scratch entry point (the same kernels and
summation order), and within the float32 bar (1e-5 relative) of the oracle.
"""
import numpy as np
import pytest

from paper_2105_12026_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)


def _csr(rng, n, sizes):
    sets = [rng.integers(0, n, sz) for sz in sizes]
    off = np.cumsum([0] + [len(q) for q in sets]).astype(np.int64)
    idx = np.concatenate(sets).astype(np.int32) if sum(sizes) else np.zeros(0, np.int32)
    return off, idx


@pytest.mark.parametrize("dt,in_dtype", [("f32", False), ("bf16", True), ("fp8", True)])
def test_noalloc_matches_caller_scratch(ref, dt, in_dtype):
    import torch
    from paper_2105_12026_amd import ebc

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(91)
    n, d = 5000, 64
    x = W.gaussian_mixture(rng, n, d, 6).astype(np.float32)
    ds = ebc.Dataset(torch.from_numpy(x).to(dev), dtype=dt)
    # first call: many sets of mixed sizes (several ground-set splits, ragged tail)
    sizes1 = [0, 1, 7, 8, 9, 33, 257] + list(rng.integers(1, 40, 3000))
    # second call: fewer, smaller sets
    sizes2 = [3, 0, 10, 1] + list(rng.integers(1, 12, 200))
    for call, sizes in (("first", sizes1), ("second", sizes2)):
        off, idx = _csr(rng, n, sizes)
        _say(f"eval_sets_noalloc {call} call n={n} d={d} dtype={dt} in_dtype={in_dtype} l={len(sizes)}")
        off_t = torch.from_numpy(off).to(dev)
        idx_t = torch.from_numpy(idx).to(dev)
        out = torch.full((len(sizes),), float("nan"), dtype=torch.float64, device=dev)
        got = ds.eval_sets_noalloc(off_t, idx_t, out, in_dtype=in_dtype).cpu().numpy()
        want = ds.eval_sets(off_t, idx_t, in_dtype=in_dtype).cpu().numpy()
        ds.sync()
        assert np.array_equal(got, want), float(np.max(np.abs(got - want)))
        if not in_dtype:
            rf = ref.eval_sets(x, off, idx)
            np.testing.assert_allclose(got, rf, rtol=1e-5, atol=1e-12)


def test_noalloc_rejects_beyond_fixed_scratch():
    import torch
    from paper_2105_12026_amd import ebc

    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    dev = torch.device("cuda:0")
    n, d = 100000, 16
    rng = np.random.default_rng(92)
    x = rng.standard_normal((n, d)).astype(np.float32)
    ds = ebc.Dataset(torch.from_numpy(x).to(dev))
    l = 200000  # 16 ground-set splits: about 144 bytes per set, above 16 MiB
    assert ebc.lib().ebc_eval_sets_bytes(n, l) > ebc.FIXED_SCRATCH_BYTES
    off = torch.zeros(l + 1, dtype=torch.int64, device=dev)
    idx = torch.zeros(1, dtype=torch.int32, device=dev)
    out = torch.zeros(l, dtype=torch.float64, device=dev)
    _say(f"eval_sets_noalloc above the fixed scratch n={n} l={l}")
    with pytest.raises(ebc.EBCError) as e:
        ds.eval_sets_noalloc(off, idx, out)
    assert e.value.code == 5  # EBC_E_NOMEM, nothing enqueued
    ds.sync()
    assert float(out.abs().sum()) == 0.0
