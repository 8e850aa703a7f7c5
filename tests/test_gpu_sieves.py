"""Three Sieves (ebc_three_sieves) through the C ABI against the FP64 oracle
(oracle.ebc_oracle.three_sieves): the same accepted points in the same
order, f after each acceptance within 1e-12 relative, and the same number of
points examined, in every distance dtype (each decision near its bound is
taken on a float64 re-score), for short and long rows, streams in index
order, permuted or with repeats, and a non-zero e0. Changing the stretch
length of the gains launches changes nothing."""
import numpy as np
import pytest

from oracle import ebc_oracle as O
from paper_2105_12026_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2105_12026_amd import ebc
    assert torch.cuda.is_available()
    return torch, ebc


def _ds(env, x, dt, e0=None):
    torch, ebc = env
    ds = ebc.Dataset(torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda(), dtype=dt)
    if e0 is not None:
        ds.set_e0(torch.from_numpy(np.ascontiguousarray(e0, np.float32)).cuda())
    return ds


CASES = [  # (kind, n, d, k, eps, T, stream, seed)
    ("gmm", 1500, 32, 10, 0.1, 20, "index", 1),
    ("gmm", 900, 64, 6, 0.5, 3, "perm", 2),
    ("gmm", 700, 100, 15, 0.05, 100, "repeats", 3),
    ("curves", 400, 300, 8, 0.2, 10, "perm", 4),
]


def _stream(kind, n, rng):
    if kind == "index":
        return None
    if kind == "perm":
        return rng.permutation(n).astype(np.int32)
    return rng.integers(0, n, size=n + n // 2).astype(np.int32)


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16", "fp8"])
@pytest.mark.parametrize("kind,n,d,k,eps,T,stream,seed", CASES)
def test_three_sieves_matches_oracle(env, dt, kind, n, d, k, eps, T, stream, seed):
    torch, _ = env
    rng = np.random.default_rng(seed)
    if kind == "curves":
        x = W.process_curves(rng, n, d).astype(np.float32)
    else:
        x = W.gaussian_mixture(rng, n, d, 6).astype(np.float32)
    order = _stream(stream, n, rng)
    rsel, rf, rv, rseen = O.three_sieves(x, k, eps, T, order=order)
    print(f"[gpu-case] three sieves {dt} {kind} n={n} d={d} k={k} eps={eps} T={T} stream={stream}", flush=True)
    ds = _ds(env, x, dt)
    to = None if order is None else torch.from_numpy(order)
    sel, f, seen = ds.three_sieves(k, eps, T, order=to)
    ds.sync()
    assert sel.cpu().numpy().tolist() == rsel
    np.testing.assert_allclose(f.cpu().numpy(), rf, rtol=1e-12)
    assert seen == rseen
    print(f"[gpu-result] three sieves {dt}: {len(rsel)} accepted after {seen} points", flush=True)


def test_three_sieves_stretch_length_and_e0(env):
    torch, _ = env
    rng = np.random.default_rng(9)
    x = W.gaussian_mixture(rng, 1200, 48, 5).astype(np.float32)
    e0 = rng.standard_normal(48).astype(np.float32)
    order = rng.permutation(1200).astype(np.int32)
    rsel, rf, _, rseen = O.three_sieves(x, 12, 0.1, 15, order=order, e0=e0)
    print("[gpu-case] three sieves e0, stretches of 64 / 1024 points", flush=True)
    ds = _ds(env, x, "f32", e0)
    out = []
    for batch in (64, 1024):
        sel, f, seen = ds.three_sieves(12, 0.1, 15, order=torch.from_numpy(order), batch=batch)
        ds.sync()
        out.append((sel.cpu().numpy(), f.cpu().numpy(), seen))
    np.testing.assert_array_equal(out[0][0], out[1][0])
    np.testing.assert_array_equal(out[0][1], out[1][1])
    assert out[0][0].tolist() == rsel and out[0][2] == rseen
    np.testing.assert_allclose(out[0][1], rf, rtol=1e-12)


def test_three_sieves_bad_order_is_rejected(env):
    torch, ebc = env
    x = np.random.default_rng(10).standard_normal((50, 4)).astype(np.float32)
    ds = _ds(env, x, "f32")
    print("[gpu-case] three sieves order index out of range", flush=True)
    with pytest.raises(ebc.EBCError) as ei:
        ds.three_sieves(3, 0.1, 5, order=torch.tensor([1, 2, 50], dtype=torch.int32))
    assert ei.value.code == 2
    ds.sync()


SS_CASES = [  # (kind, n, d, k, eps, stream, seed)
    ("gmm", 800, 32, 6, 0.3, "perm", 11),
    ("gmm", 500, 100, 4, 0.5, "index", 12),
    ("curves", 300, 260, 5, 0.5, "repeats", 13),
]


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16", "fp8"])
@pytest.mark.parametrize("kind,n,d,k,eps,stream,seed", SS_CASES)
def test_sieve_streaming_matches_oracle(env, dt, kind, n, d, k, eps, stream, seed):
    torch, _ = env
    rng = np.random.default_rng(seed)
    if kind == "curves":
        x = W.process_curves(rng, n, d).astype(np.float32)
    else:
        x = W.gaussian_mixture(rng, n, d, 6).astype(np.float32)
    order = _stream(stream, n, rng)
    rsel, rf, rv, rseen = O.sieve_streaming(x, k, eps, order=order)
    print(f"[gpu-case] sieve streaming {dt} {kind} n={n} d={d} k={k} eps={eps} stream={stream}", flush=True)
    ds = _ds(env, x, dt)
    to = None if order is None else torch.from_numpy(order)
    sel, f, v, seen = ds.sieve_streaming(k, eps, order=to, batch=128)
    ds.sync()
    assert sel.cpu().numpy().tolist() == rsel
    np.testing.assert_allclose(f.cpu().numpy(), rf, rtol=1e-12)
    assert v == pytest.approx(rv, rel=1e-15) and seen == rseen
    # the dataset state holds the best summary's minima
    g = ds.marginal_gains(cand=torch.arange(min(n, 64), dtype=torch.int32)).cpu().numpy()
    ds.sync()
    m = O.min_dist_to_set(x, rsel)
    rg = O.gains(x, m, range(min(n, 64)))
    assert np.max(np.abs(g - rg)) <= {"f32": 1e-5, "bf16": 1e-2, "f16": 2e-3, "fp8": 8e-2}[dt] * max(np.max(np.abs(rg)), 1e-300)
