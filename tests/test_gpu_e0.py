"""A non-zero auxiliary vector e0 (Sec. 4: f(S) = L({e0}) - L(S u {e0}) for
any fixed e0) through the C ABI, against the FP64 oracle with the same e0:
greedy selections identical in float32, f and gains within 1e-5, multi-set
evaluation in float32 and in each cast dtype at its bar, short and long
rows, batched runs equal to solo runs, and the origin restored bitwise."""
import numpy as np
import pytest

from paper_2105_12026_amd import workloads as W

pytestmark = pytest.mark.gpu

# multi-set f in the dataset dtype, |f - f_ref| / (|f_ref| + 1e-3 L({e0})):
# BF16 and FP16 at the proposed bars; FP8 at 3e-2, 1.3x the largest error
# measured over the committed cases (2.33e-2; about 0.4 of e4m3's unit
# roundoff 2^-4, like the other dtypes' maxima relative to theirs)
ES_TOL = {"bf16": 2e-3, "f16": 5e-4, "fp8": 3e-2}


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2105_12026_amd import ebc
    assert torch.cuda.is_available()
    return torch, ebc


def _ds(env, x, dt="f32", e0=None):
    torch, ebc = env
    ds = ebc.Dataset(torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda(), dtype=dt)
    if e0 is not None:
        ds.set_e0(torch.from_numpy(np.ascontiguousarray(e0, np.float32)).cuda())
    return ds


def _e0(kind, x, rng):
    if kind == "random":
        return rng.standard_normal(x.shape[1]).astype(np.float32) * 3.0
    if kind == "mean":
        return x.mean(axis=0).astype(np.float32)
    return x[7].copy()  # a data point: its own gain is 0


@pytest.mark.parametrize("kind", ["random", "mean", "point"])
@pytest.mark.parametrize("n,d,k,seed", [(2000, 64, 10, 1), (700, 100, 12, 2), (600, 300, 8, 3)])
def test_e0_greedy_and_gains_f32(env, ref, kind, n, d, k, seed):
    rng = np.random.default_rng(seed)
    x = W.gaussian_mixture(rng, n, d, 6).astype(np.float32)
    e0 = _e0(kind, x, rng)
    print(f"[gpu-case] e0={kind} greedy f32 n={n} d={d} k={k}", flush=True)
    ds = _ds(env, x, "f32", e0)
    g0 = ds.marginal_gains().cpu().numpy()
    ds.sync()
    rg0 = ref.gains(x, ref.min_dist(x, [], e0))
    assert np.max(np.abs(g0 - rg0)) <= 1e-5 * np.max(np.abs(rg0))
    sel, f, g = ds.greedy(k)
    ds.sync()
    rsel, rf, rg = ref.greedy(x, k, e0)
    assert sel.cpu().numpy().tolist() == rsel.tolist()
    np.testing.assert_allclose(f.cpu().numpy(), rf, rtol=1e-5)
    np.testing.assert_allclose(g.cpu().numpy(), rg, rtol=1e-5, atol=1e-12 * rf[-1])
    l0 = float(np.mean(np.sum((x.astype(np.float64) - e0.astype(np.float64)) ** 2, axis=1)))
    assert ds.info()["l0"] == pytest.approx(l0, rel=1e-12)


@pytest.mark.parametrize("n,d,seed", [(1500, 64, 11), (900, 100, 12), (500, 260, 13)])
def test_e0_eval_sets(env, ref, n, d, seed):
    torch, _ = env
    rng = np.random.default_rng(seed)
    x = W.gaussian_mixture(rng, n, d, 5).astype(np.float32)
    e0 = _e0("random", x, rng)
    sizes = [0, 1, 5, 9, 33, 64, 0, 3] + list(rng.integers(1, 30, 80))
    sets = [rng.integers(0, n, sz) for sz in sizes]
    off = np.cumsum([0] + [len(q) for q in sets]).astype(np.int64)
    idx = np.concatenate(sets).astype(np.int32)
    rf = ref.eval_sets(x, off, idx, e0)
    l0 = float(np.mean(np.sum((x.astype(np.float64) - e0.astype(np.float64)) ** 2, axis=1)))
    to, ti = torch.from_numpy(off), torch.from_numpy(idx)
    for dt in ("f32", "bf16", "f16", "fp8"):
        print(f"[gpu-case] e0 eval_sets {dt} n={n} d={d}", flush=True)
        ds = _ds(env, x, dt, e0)
        f32 = ds.eval_sets(to, ti).cpu().numpy()
        ds.sync()
        assert np.all(f32[np.array(sizes) == 0] == 0.0)
        assert np.all(np.abs(f32 - rf) <= 1e-5 * np.abs(rf) + 1e-12 * l0), dt
        if dt != "f32":
            fl = ds.eval_sets(to, ti, in_dtype=True).cpu().numpy()
            ds.sync()
            rel = np.abs(fl - rf) / (np.abs(rf) + 1e-3 * l0)
            print(f"[gpu-result] e0 eval_sets in {dt} n={n} d={d}: max rel err {rel.max():.3e}", flush=True)
            assert rel.max() <= ES_TOL[dt]


def test_e0_origin_restored_bitwise(env):
    torch, _ = env
    rng = np.random.default_rng(21)
    x = W.gaussian_mixture(rng, 1200, 48, 5).astype(np.float32)
    print("[gpu-case] e0 set and restored", flush=True)
    plain = _ds(env, x)
    a = [t.cpu().numpy() for t in plain.greedy(6)]
    plain.sync()
    ds = _ds(env, x, "f32", rng.standard_normal(48))
    other = [t.cpu().numpy() for t in ds.greedy(6)]
    ds.set_e0(None)
    b = [t.cpu().numpy() for t in ds.greedy(6)]
    ds.sync()
    for u, v in zip(a, b):
        np.testing.assert_array_equal(u, v)
    assert not np.array_equal(a[1], other[1])


def test_e0_batched_equals_solo(env, ref):
    torch, ebc = env
    rng = np.random.default_rng(31)
    specs = [(900, 32, "f32", 5), (1300, 64, "bf16", 6), (500, 200, "f32", 4)]
    print("[gpu-case] e0 batched vs solo", flush=True)
    xs = [W.gaussian_mixture(rng, n, d, 4).astype(np.float32) for n, d, _, _ in specs]
    e0s = [rng.standard_normal(d).astype(np.float32) for _, d, _, _ in specs]
    solos = []
    for x, e0, (n, d, dt, k) in zip(xs, e0s, specs):
        ds = _ds(env, x, dt, e0)
        solos.append([t.cpu().numpy() for t in ds.greedy(k)])
        ds.sync()
    dss = [_ds(env, x, dt, e0) for x, e0, (_, _, dt, _) in zip(xs, e0s, specs)]
    batch = ebc.Batch(dss)
    outs = batch.greedy([s[3] for s in specs])
    for ds in dss:
        ds.sync()
    for so, bo in zip(solos, outs):
        for u, v in zip(so, bo):
            np.testing.assert_array_equal(v.cpu().numpy(), u)
    for x, e0, so, (n, d, dt, k) in zip(xs, e0s, solos, specs):
        if dt == "f32":
            rsel, _, _ = ref.greedy(x, k, e0)
            assert so[0].tolist() == rsel.tolist()
