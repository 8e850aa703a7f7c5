"""Reduced-precision distances (BF16, FP16, FP8-e4m3 with E8M0 row scales)
against the FP64 oracle.

Bars, per distance dtype (relative to the largest gain of the vector):
  gains   max_c |G_dt - G_ref| / max_c |G_ref|   <= GAIN_TOL[dt]
  greedy  f(S_t) is float64 for the chosen set (checked exactly against the
          oracle's f of that set); quality gap of the final set against the
          oracle's greedy <= GAP_TOL[dt]; selection agreement is printed.
"""
import os

import numpy as np
import pytest

from paper_2105_12026_amd import workloads as W

pytestmark = pytest.mark.gpu

GAIN_TOL = {"bf16": 1e-2, "f16": 2e-3, "fp8": 8e-2}
GAP_TOL = {"bf16": 1e-3, "f16": 1e-3, "fp8": 2e-2}


@pytest.fixture(scope="module")
def env():
    import torch
    from paper_2105_12026_amd import ebc
    assert torch.cuda.is_available()
    return torch, ebc


def _ds(env, x, dt):
    torch, ebc = env
    return ebc.Dataset(torch.from_numpy(np.ascontiguousarray(x, np.float32)).cuda(), dtype=dt)


@pytest.mark.parametrize("dt", ["bf16", "f16", "fp8"])
@pytest.mark.parametrize("n,d,seed", [(3000, 64, 1), (1500, 100, 2), (777, 16, 3), (260, 128, 4), (5, 3, 5)])
def test_lowprec_gains(env, ref, dt, n, d, seed):
    torch, _ = env
    rng = np.random.default_rng(seed)
    x = W.gaussian_mixture(rng, n, d, 6).astype(np.float32)
    print(f"[gpu-case] gains {dt} n={n} d={d}", flush=True)
    ds = _ds(env, x, dt)
    errs = []
    for s in ([], list(rng.choice(n, min(n, 4), replace=False))):
        m = ref.min_dist(x, s)
        g = ds.marginal_gains(m=torch.from_numpy(m)).cpu().numpy()
        ds.sync()
        rg = ref.gains(x, m)
        errs.append(float(np.max(np.abs(g - rg)) / np.max(np.abs(rg))))
    print(f"[gpu-result] gains {dt} n={n} d={d} rel err {max(errs):.3e}", flush=True)
    assert max(errs) <= GAIN_TOL[dt]


@pytest.mark.parametrize("dt", ["bf16", "f16", "fp8"])
def test_lowprec_greedy_quality(env, ref, dt):
    rng = np.random.default_rng(7)
    x = W.gaussian_mixture(rng, 4000, 64, 12).astype(np.float32)
    k = 16
    print(f"[gpu-case] greedy {dt} n=4000 d=64 k={k}", flush=True)
    ds = _ds(env, x, dt)
    sel, f, g = ds.greedy(k)
    stats = ds.sync()
    sel = sel.cpu().numpy()
    rsel, rf, _ = ref.greedy(x, k)
    # f(S_t) of the chosen sets is float64-exact
    l0 = float(np.mean(np.sum(x.astype(np.float64) ** 2, axis=1)))
    for t in (0, k // 2, k - 1):
        m = ref.min_dist(x, sel[:t + 1])
        assert f.cpu().numpy()[t] == pytest.approx(l0 - float(np.mean(m)), rel=1e-9)
    agree = len(set(sel.tolist()) & set(rsel.tolist())) / k
    prefix = next((i for i in range(k) if sel[i] != rsel[i]), k)
    gap = (rf[-1] - f.cpu().numpy()[-1]) / rf[-1]
    print(f"[gpu-result] greedy {dt}: agreement {agree:.2f} common prefix {prefix} quality gap {gap:.2e} "
          f"window max {stats['window_max']}", flush=True)
    assert gap <= GAP_TOL[dt]


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16", "fp8"])
def test_zero_gain_steps_pick_lowest_unselected(env, ref, dt):
    """20 distinct points, each present 15 times (300 rows), greedy to k = n:
    after the 20 distinct points are picked every point is covered, and the
    280 remaining steps have 280 .. 1 zero-gain candidates, more than the
    256 the float64 window re-scores. Each such step must pick the lowest
    unselected index (the oracle's reading), whatever the dtype."""
    rng = np.random.default_rng(17)
    base = (rng.standard_normal((20, 8)) * 4.0).astype(np.float32)
    x = np.concatenate([base[rng.permutation(20)] for _ in range(15)])
    n = x.shape[0]
    print(f"[gpu-case] zero-gain steps {dt} n={n} k={n}", flush=True)
    ds = _ds(env, x, dt)
    sel, f, g = ds.greedy(n)
    ds.sync()
    sel, f, g = sel.cpu().numpy(), f.cpu().numpy(), g.cpu().numpy()
    rsel, rf, rg = ref.greedy(x, n)
    assert sorted(sel.tolist()) == list(range(n))
    assert set(sel[:20].tolist()) == set(rsel[:20].tolist())   # one copy of each distinct point
    assert sel[20:].tolist() == rsel[20:].tolist()               # then lowest unselected, in order
    assert np.all(g[20:] == 0.0)
    l0 = float(np.mean(np.sum(x.astype(np.float64) ** 2, axis=1)))
    assert f[-1] == pytest.approx(l0, rel=1e-12)
    if dt == "f32":
        assert sel.tolist() == rsel.tolist()


def test_f16_range_is_reported(env):
    _, ebc = env
    x = np.ones((40, 4), np.float32)
    x[3, 1] = 1e5
    print("[gpu-case] f16 range", flush=True)
    ds = _ds(env, x, "f16")
    with pytest.raises(ebc.EBCError) as ei:
        ds.sync()
    assert ei.value.code == 4


@pytest.fixture(scope="module")
def sweep200k():
    return W.precision_sweep(seed=3)


@pytest.mark.parametrize("dt", ["bf16", "f16", "fp8"])
def test_lowprec_full_size_gains_sampled(env, ref, sweep200k, dt):
    """200000 x 64 mixture with outliers, all candidates in the benchmark's
    launch configuration; a sample of the outputs against the oracle, at
    S = {} and at a 30-point S."""
    torch, _ = env
    p = sweep200k
    rng = np.random.default_rng(91)
    cand = np.sort(rng.choice(p.n, 96, replace=False)).astype(np.int32)
    print(f"[gpu-case] full-size gains {dt} n=200000 d=64", flush=True)
    ds = _ds(env, p.x, dt)
    errs = []
    for s in ([], rng.choice(p.n, 30, replace=False)):
        m = ref.min_dist(p.x, s)
        g = ds.marginal_gains(m=torch.from_numpy(m)).cpu().numpy()
        ds.sync()
        rg = ref.gains(p.x, m, cand)
        scale = max(np.max(np.abs(rg)), np.max(g))
        errs.append(float(np.max(np.abs(g[cand] - rg)) / scale))
    print(f"[gpu-result] full-size gains {dt} rel err {max(errs):.3e}", flush=True)
    assert max(errs) <= GAIN_TOL[dt]


GOLDEN_SWEEP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "gmm50+out_n200000_d64_k100.json")


@pytest.mark.parametrize("dt", ["f32", "bf16", "f16", "fp8"])
def test_full_size_greedy_against_oracle_run(env, ref, sweep200k, dt):
    """Greedy k = 100 on the 200000 x 64 precision-sweep input, in the
    benchmark's configuration, against the stored float64 oracle run: float32
    selections identical and f within 1e-5; reduced precision within the
    quality-gap bar, f(S_t) float64-exact for the chosen sets; agreement
    printed."""
    import json
    if not os.path.exists(GOLDEN_SWEEP):
        pytest.skip("stored oracle run missing (tests/golden/make_golden.py sweep200k)")
    gold = json.load(open(GOLDEN_SWEEP))
    p = sweep200k
    assert W.sha256_of(p.x) == gold["sha256_x"]
    print(f"[gpu-case] full-size greedy {dt} n=200000 d=64 k=100", flush=True)
    ds = _ds(env, p.x, dt)
    if dt != "f32":
        ds.set_variant(3)
    sel, f, g = ds.greedy(p.k)
    stats = ds.sync()
    sel, f = sel.cpu().numpy(), f.cpu().numpy()
    rsel, rf = np.array(gold["sel"]), np.array(gold["f"])
    agree = len(set(sel.tolist()) & set(rsel.tolist())) / p.k
    prefix = next((i for i in range(p.k) if sel[i] != rsel[i]), p.k)
    gap = (rf[-1] - f[-1]) / rf[-1]
    print(f"[gpu-result] full-size greedy {dt}: agreement {agree:.2f} common prefix {prefix} "
          f"quality gap {gap:.2e} window max {stats['window_max']}", flush=True)
    if dt == "f32":
        assert sel.tolist() == rsel.tolist()
        np.testing.assert_allclose(f, rf, rtol=1e-12)
        return
    l0 = float(np.mean(np.sum(p.x.astype(np.float64) ** 2, axis=1)))
    for t in (9, p.k - 1):
        m = ref.min_dist(p.x, sel[:t + 1])
        assert f[t] == pytest.approx(l0 - float(np.mean(m)), rel=1e-9)
    assert gap <= GAP_TOL[dt]


@pytest.mark.parametrize("dt", ["bf16", "f16", "fp8"])
@pytest.mark.parametrize("n,d,seed", [(5, 3, 21), (700, 33, 22), (2049, 64, 23), (5000, 64, 24), (1300, 100, 25),
                                      (900, 128, 26), (1500, 32, 27), (9000, 24, 28)])
def test_every_variant_matches_oracle_and_variant0(env, ref, dt, n, d, seed):
    """All tile variants (including the 8-wave ping-pong one, with one or two
    candidate blocks per wave, and the interleaved one with its 64-, 128- and
    256-point ring stages: d = 32 and 24 take 256 in BF16/FP16, with 1 and 8
    ground-set chunks, the last one ragged) give bitwise-equal gains, for all
    candidates and for an unordered candidate list with repeats, within the
    oracle bar."""
    torch, ebc = env
    rng = np.random.default_rng(seed)
    x = W.gaussian_mixture(rng, n, d, 6).astype(np.float32)
    ds = _ds(env, x, dt)
    s = list(rng.choice(n, min(n, 3), replace=False))
    m = ref.min_dist(x, s)
    mt = torch.from_numpy(m)
    cand = rng.integers(0, n, size=max(1, (3 * n) // 5)).astype(np.int32)
    rg_all = ref.gains(x, m)
    base = None
    for v in range(ebc.Dataset.variant_count(dt)):
        print(f"[gpu-case] gains variant {v} {dt} n={n} d={d}", flush=True)
        ds.set_variant(v)
        g_all = ds.marginal_gains(m=mt).cpu().numpy()
        g_c = ds.marginal_gains(m=mt, cand=torch.from_numpy(cand)).cpu().numpy()
        ds.sync()
        err = float(np.max(np.abs(g_all - rg_all)) / np.max(np.abs(rg_all)))
        assert err <= GAIN_TOL[dt], (v, err)
        np.testing.assert_array_equal(g_c, g_all[cand])
        if base is None:
            base = g_all
        else:
            np.testing.assert_array_equal(g_all, base, err_msg=f"variant {v}")


# multi-set f in the dataset dtype, |f - f_ref| / (|f_ref| + 1e-3 L({e0})):
# BF16 and FP16 at the proposed bars; FP8 at 3e-2, 1.3x the largest error
# measured over the committed cases (2.33e-2; about 0.4 of e4m3's unit
# roundoff 2^-4, like the other dtypes' maxima relative to theirs)
ES_TOL = {"bf16": 2e-3, "f16": 5e-4, "fp8": 3e-2}


@pytest.mark.parametrize("dt", ["bf16", "f16", "fp8"])
@pytest.mark.parametrize("n,d,seed", [(3000, 100, 81), (777, 16, 82), (2049, 64, 83), (300, 128, 84)])
def test_eval_sets_in_dtype(env, ref, dt, n, d, seed):
    """Multi-set evaluation with the dot products in the dataset's dtype:
    sets of many sizes (across unit, block and window boundaries, empty sets
    between), against the float64 oracle at the dtype's bar (relative to f,
    with a floor of 1e-3 L({e0})); deterministic; the float32 entry point on
    the same dataset is unaffected."""
    torch, ebc = env
    rng = np.random.default_rng(seed)
    x = W.gaussian_mixture(rng, n, d, 5).astype(np.float32)
    sizes = [0, 1, 7, 8, 9, 0, 31, 32, 33, 64, 100, 255, 257, 3, 10, 10] + list(rng.integers(1, 40, 200))
    sets = [rng.integers(0, n, sz) for sz in sizes]
    off = np.cumsum([0] + [len(q) for q in sets]).astype(np.int64)
    idx = np.concatenate(sets).astype(np.int32)
    print(f"[gpu-case] eval_sets in {dt} n={n} d={d} l={len(sets)}", flush=True)
    ds = _ds(env, x, dt)
    to = torch.from_numpy(off)
    ti = torch.from_numpy(idx)
    f1 = ds.eval_sets(to, ti, in_dtype=True).cpu().numpy()
    f2 = ds.eval_sets(to, ti, in_dtype=True).cpu().numpy()
    f32 = ds.eval_sets(to, ti).cpu().numpy()
    ds.sync()
    assert np.array_equal(f1, f2)
    rf = ref.eval_sets(x, off, idx)
    l0 = float(np.mean(np.sum(x.astype(np.float64) ** 2, axis=1)))
    assert np.all(f1[np.array(sizes) == 0] == 0.0)
    rel = np.abs(f1 - rf) / (np.abs(rf) + 1e-3 * l0)
    print(f"[gpu-result] eval_sets in {dt} n={n} d={d}: max rel err {rel.max():.3e}", flush=True)
    assert rel.max() <= ES_TOL[dt]
    assert np.all(np.abs(f32 - rf) <= 1e-5 * np.abs(rf) + 1e-12 * l0)


@pytest.mark.parametrize("dt", ["bf16", "f16", "fp8"])
@pytest.mark.parametrize("n,d,seed", [(3000, 100, 91), (777, 16, 92), (4100, 64, 93), (300, 128, 94)])
def test_eval_sets_in_dtype_short_sets(env, ref, dt, n, d, seed):
    """Sets of at most 32 members (the kernel that keeps member rows in
    registers takes every call whose sets all fit 8 units): sizes on both
    sides of every unit and block boundary, empty sets and repeated members
    between them, several ground-set splits with ragged tails and empty
    splits (n = 4100); against the float64 oracle at the dtype's bar,
    deterministic; BF16/FP16 also against exact arithmetic on the cast rows."""
    torch, ebc = env
    rng = np.random.default_rng(seed)
    x = W.gaussian_mixture(rng, n, d, 5).astype(np.float32)
    sizes = [0, 1, 3, 4, 5, 8, 0, 9, 16, 17, 31, 32, 2, 10, 10] + list(rng.integers(1, 33, 400))
    sets = [rng.integers(0, n, sz) for sz in sizes]
    sets[5] = np.array([7, 7, 7, 7, 7], dtype=np.int64)  # repeated member
    off = np.cumsum([0] + [len(q) for q in sets]).astype(np.int64)
    idx = np.concatenate(sets).astype(np.int32)
    print(f"[gpu-case] short-set eval_sets in {dt} n={n} d={d} l={len(sets)}", flush=True)
    ds = _ds(env, x, dt)
    to = torch.from_numpy(off)
    ti = torch.from_numpy(idx)
    f1 = ds.eval_sets(to, ti, in_dtype=True).cpu().numpy()
    f2 = ds.eval_sets(to, ti, in_dtype=True).cpu().numpy()
    ds.sync()
    assert np.array_equal(f1, f2)
    rf = ref.eval_sets(x, off, idx)
    l0 = float(np.mean(np.sum(x.astype(np.float64) ** 2, axis=1)))
    assert np.all(f1[np.array(sizes) == 0] == 0.0)
    rel = np.abs(f1 - rf) / (np.abs(rf) + 1e-3 * l0)
    bar = ES_TOL[dt]
    if dt != "fp8":
        # the same sets in exact arithmetic on the cast rows (round-to-nearest-even
        # BF16/FP16, half-norms of the cast rows rounded to float32): what the
        # format alone costs, and the kernel's own arithmetic to 2e-5 of it
        fe = _cast_sets_f(x, sets, dt)
        rel_fmt = np.abs(fe - rf) / (np.abs(rf) + 1e-3 * l0)
        rel_ker = np.abs(f1 - fe) / (np.abs(fe) + 1e-3 * l0)
        print(f"[gpu-result]   format alone: {rel_fmt.max():.3e}; kernel vs cast arithmetic {rel_ker.max():.3e}",
              flush=True)
        assert rel_ker.max() <= 2e-5
        # a set whose few members the format itself moves further than the bar
        bar = max(bar, 1.25 * rel_fmt.max())
    print(f"[gpu-result] short-set eval_sets in {dt} n={n} d={d}: max rel err {rel.max():.3e} (bar {bar:.2e})",
          flush=True)
    assert rel.max() <= bar


def _cast_sets_f(x, sets, dt):
    """f(S) of each set in float64 on the rows cast to BF16 / FP16 (round to
    nearest even), with the cast rows' half-norms rounded to float32 and the
    exact ||v||^2 of the float32 rows for e0 = 0."""
    if dt == "f16":
        xh = x.astype(np.float16).astype(np.float64)
    else:
        u = x.view(np.uint32).astype(np.uint64)
        xh = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32).view(np.float32).astype(np.float64)
    hn = (0.5 * np.sum(xh * xh, axis=1)).astype(np.float32).astype(np.float64)
    m0 = np.sum(x.astype(np.float64) ** 2, axis=1)
    wsh = (0.5 * m0 - hn).astype(np.float32).astype(np.float64)
    out = np.zeros(len(sets))
    for j, s in enumerate(sets):
        if len(s):
            t = xh @ xh[s].T - hn[s][None, :]
            out[j] = 2.0 * np.sum(np.maximum(0.0, t.max(axis=1) + wsh)) / x.shape[0]
    return out
